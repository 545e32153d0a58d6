"""Pins of the oracle's asymmetric peak (the paper's asymmetry factor
A(x; alpha), Appendix A.2): unit area and continuity for any alpha,
half-maximum points at rho - w/2 and rho + alpha w/2, reduction to the
symmetric model at alpha = 1, the windowed areas, and central differences
of the ELBO in all five coordinates per phase."""
import itertools
import math

import numpy as np
import pytest
from scipy import special, stats

from paper_2501_09308_amd import workloads as W


def peak(orc, x, w, r, al, c=0.0):
    phi = np.array([[1.0], [0.0], [w], [r], [al]])
    return orc.profile_asym(x, np.zeros(len(x)), np.array([0, 1]),
                            np.array([30.0]), np.array([1.0]), c, phi)[0]


def _simpson(y, h):
    return h / 3 * (y[0] + y[-1] + 4 * y[1:-1:2].sum() + 2 * y[2:-1:2].sum())


@pytest.mark.parametrize("al", [0.5, 1.0, 1.7])
@pytest.mark.parametrize("r", [0.0, 0.6, 1.0])
def test_unit_area_any_asymmetry(orc, al, r):
    w, R = 0.1, 5.0
    # integrate each side on its own grid (the peak has a kink at rho)
    xl = np.linspace(30.0 - R, 30.0, 100001)
    xr = np.linspace(30.0, 30.0 + R, 100001)
    area = _simpson(peak(orc, xl, w, r, al), xl[1] - xl[0]) \
        + _simpson(peak(orc, xr, w, r, al), xr[1] - xr[0])
    # Gaussian tails are negligible; the Lorentz tails beyond R on each side
    tail = r * (2 / (1 + al)) * (0.5 - math.atan(2 * R / w) / math.pi) \
        + r * (2 * al / (1 + al)) * (0.5 - math.atan(2 * R / (al * w)) / math.pi)
    assert area + tail == pytest.approx(1.0, rel=1e-9)


@pytest.mark.parametrize("al", [0.6, 1.4])
def test_continuous_at_centre_and_half_maximum(orc, al):
    w, r = 0.25, 0.4
    x = np.array([30.0 - 1e-12, 30.0, 30.0 - w / 2, 30.0 + al * w / 2])
    v = peak(orc, x, w, r, al)
    assert v[0] == pytest.approx(v[1], rel=1e-9)
    assert v[2] == pytest.approx(v[1] / 2, rel=1e-12)
    assert v[3] == pytest.approx(v[1] / 2, rel=1e-12)
    # height 2/(1+alpha) times the symmetric height at width w
    sym = (1 - r) * 2 * math.sqrt(math.log(2) / math.pi) / w + r * 2 / (math.pi * w)
    assert v[1] == pytest.approx(2 / (1 + al) * sym, rel=1e-12)


def test_alpha_one_is_the_symmetric_model(orc):
    prob = W.make_problem("tiny", seed=41, K=5, M=10)
    phi4 = W.random_phi(prob.K, 3, 42)
    phi5 = np.concatenate([phi4, np.ones((3, 1, prob.K))], axis=1)
    for c in (0.0, 6.0):
        f4 = orc.profile(prob.x, prob.bg, prob.peak_off, prob.peak_pos,
                         prob.peak_int, c, phi4)
        f5 = orc.profile_asym(prob.x, prob.bg, prob.peak_off, prob.peak_pos,
                              prob.peak_int, c, phi5)
        np.testing.assert_allclose(f5, f4, rtol=1e-13)


def test_asymmetric_windows_brute_force(orc):
    prob = W.make_problem("tiny", seed=43, N=500, K=4, M=9)
    phi = np.concatenate([W.random_phi(prob.K, 2, 44),
                          np.random.default_rng(1).uniform(0.5, 1.8, (2, 1, prob.K))], axis=1)
    c = 5.0
    lo, hi = orc.windows_asym(prob.x, prob.peak_off, prob.peak_pos, c, phi)
    for s in range(2):
        for k in range(prob.K):
            for m in range(prob.peak_off[k], prob.peak_off[k + 1]):
                rho = prob.peak_pos[m] + phi[s, 1, k]
                hw = c * phi[s, 2, k]
                inside = np.nonzero((rho - hw <= prob.x) & (prob.x <= rho + hw * phi[s, 4, k]))[0]
                if len(inside):
                    assert lo[s, m] == inside[0] and hi[s, m] == inside[-1] + 1
                else:
                    assert lo[s, m] == hi[s, m]


def test_alpha_one_elbo_matches_symmetric_plus_alpha_terms(orc):
    # with z_alpha fixed at 0 (alpha = 1, sigma -> 0 through eps = 0) the
    # likelihood equals the symmetric one; the ELBO adds the alpha prior,
    # its Jacobian z_alpha = 0 and its entropy
    prob = W.make_problem("tiny", seed=45, N=600, K=3, M=6)
    f = orc.profile(prob.x, prob.bg, prob.peak_off, prob.peak_pos,
                    prob.peak_int, 0.0, prob.phi_true)[0]
    y = W.poisson_counts(f, 46)
    loc4, ls4 = W.random_params(prob.K, 47, (y - prob.bg).max())
    eps4 = np.zeros((2, 4, prob.K))
    e4, ll4, _, _ = orc.elbo(prob, y, loc4, ls4, eps4, grad=False)
    loc5 = np.concatenate([loc4, np.zeros((1, prob.K))])
    ls5 = np.concatenate([ls4, np.full((1, prob.K), -2.0)])
    e5, ll5, _, _ = orc.elbo_asym(prob, y, loc5, ls5, np.zeros((2, 5, prob.K)),
                                  grad=False)
    np.testing.assert_allclose(ll5, ll4, rtol=1e-13)
    extra = prob.K * (stats.norm.logpdf(1.0, 1.0, 0.2) + 0.0) \
        + ls5[4].sum() + 0.5 * prob.K * (1 + math.log(2 * math.pi))
    assert e5 == pytest.approx(e4 + extra, rel=1e-12)


@pytest.mark.parametrize("c", [0.0, 8.0])
def test_asymmetric_gradient_central_differences(orc, c):
    prob = W.make_problem("tiny", seed=48, N=800, K=3, M=5)
    f = orc.profile(prob.x, prob.bg, prob.peak_off, prob.peak_pos,
                    prob.peak_int, 0.0, prob.phi_true)[0]
    y = W.poisson_counts(f, 49)
    loc4, ls4 = W.random_params(prob.K, 50, (y - prob.bg).max(), spread=0.2)
    rng = np.random.default_rng(51)
    loc = np.concatenate([loc4, rng.normal(0, 0.3, (1, prob.K))])
    ls = np.concatenate([ls4, np.log(0.1) + rng.normal(0, 0.2, (1, prob.K))])
    eps = rng.standard_normal((2, 5, prob.K))
    lam = 1 / (y - prob.bg).max()
    _, _, gl, gs = orc.elbo_asym(prob, y, loc, ls, eps, c=c, lam=lam)
    h = 1e-5
    fd, an = [], []
    for t, k, which in itertools.product(range(5), range(prob.K), (0, 1)):
        plus = [loc.copy(), ls.copy()]; minus = [loc.copy(), ls.copy()]
        plus[which][t, k] += h; minus[which][t, k] -= h
        if c > 0:
            wins = []
            for pr in (plus, minus):
                z = pr[0][None] + np.exp(pr[1])[None] * eps
                phi = np.stack([np.exp(z[:, 0]), z[:, 1], np.exp(z[:, 2]),
                                1 / (1 + np.exp(-z[:, 3])), np.exp(z[:, 4])], axis=1)
                wins.append(orc.windows_asym(prob.x, prob.peak_off, prob.peak_pos, c, phi))
            if not (np.array_equal(wins[0][0], wins[1][0])
                    and np.array_equal(wins[0][1], wins[1][1])):
                continue
        ep = orc.elbo_asym(prob, y, *plus, eps, grad=False, c=c, lam=lam)[0]
        em = orc.elbo_asym(prob, y, *minus, eps, grad=False, c=c, lam=lam)[0]
        fd.append((ep - em) / (2 * h))
        an.append((gl if which == 0 else gs)[t, k])
    fd, an = np.array(fd), np.array(an)
    assert len(fd) >= 20
    np.testing.assert_allclose(an, fd, rtol=2e-6, atol=1e-6 * np.abs(an).max())
