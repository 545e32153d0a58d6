"""Pins of the FP64 oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: closed
forms, library densities (scipy), identities of the estimator, central
finite differences, brute-force enumeration and published known-answer
vectors.  A plausible slip in the oracle (a dropped term, a wrong sign,
index or width convention) fails at least one of them.
"""
import itertools
import math
import os

import numpy as np
import pytest
from scipy import special, stats

from paper_2501_09308_amd import workloads as W

from selection_common import map_support, phase_basis

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def one_peak(orc, x, rho, w, r, c=0.0, B=0.0):
    """Profile of one unit peak (h=1, I=1, mu=0) on grid x."""
    phi = np.array([[1.0], [0.0], [w], [r]])
    f = orc.profile(x, np.full(len(x), B), np.array([0, 1]),
                    np.array([rho]), np.array([1.0]), c, phi)[0]
    return f - B


# ---- peak shape (Appendix A.2: pseudo-Voigt of Gaussian and Lorentzian) --

@pytest.mark.parametrize("w", [0.03, 0.1, 0.3])
def test_gaussian_limit_is_normal_pdf(orc, w):
    # r = 0: unit-area Gaussian with FWHM w = normal with sigma = w/(2 sqrt(2 ln 2))
    x = np.linspace(28.0, 32.0, 4001)
    v = one_peak(orc, x, 30.0, w, 0.0)
    ref = stats.norm.pdf(x, loc=30.0, scale=w / (2 * math.sqrt(2 * math.log(2))))
    np.testing.assert_allclose(v, ref, rtol=1e-12, atol=1e-300)


@pytest.mark.parametrize("w", [0.03, 0.1, 0.3])
def test_lorentz_limit_is_cauchy_pdf(orc, w):
    # r = 1: unit-area Lorentzian with FWHM w = Cauchy with half width w/2
    x = np.linspace(20.0, 40.0, 4001)
    v = one_peak(orc, x, 30.0, w, 1.0)
    ref = stats.cauchy.pdf(x, loc=30.0, scale=w / 2)
    np.testing.assert_allclose(v, ref, rtol=1e-12)


@pytest.mark.parametrize("r", [0.0, 0.3, 0.7, 1.0])
def test_half_maximum_at_half_width(orc, r):
    # both components share FWHM w, so V(rho +- w/2) = V(rho)/2 for any r
    w = 0.25
    x = np.array([29.875, 30.0, 30.125])      # exact in binary
    v = one_peak(orc, x, 30.0, w, r)
    assert v[0] == pytest.approx(v[1] / 2, rel=1e-14)
    assert v[2] == pytest.approx(v[1] / 2, rel=1e-14)


def _simpson(y, h):
    return h / 3 * (y[0] + y[-1] + 4 * y[1:-1:2].sum() + 2 * y[2:-1:2].sum())


@pytest.mark.parametrize("r", [0.0, 0.4, 1.0])
def test_unit_area_dense(orc, r):
    # area over [rho-R, rho+R]: Gaussian -> 1, Lorentzian -> (2/pi) atan(2R/w)
    w, R = 0.1, 5.0
    n = 200001
    x = np.linspace(30.0 - R, 30.0 + R, n)
    v = one_peak(orc, x, 30.0, w, r)
    area = _simpson(v, x[1] - x[0])
    expect = (1 - r) * 1.0 + r * (2 / math.pi) * math.atan(2 * R / w)
    assert area == pytest.approx(expect, rel=1e-9)


@pytest.mark.parametrize("c", [2.0, 8.0])
def test_windowed_area_closed_form(orc, c):
    # with a window of +-c w the areas are erf(2 sqrt(ln2) c) and
    # (2/pi) atan(2c); place grid points exactly on the window edges
    w, r = 0.125, 0.35                      # c*w exact in binary
    hw = c * w
    n = 2 ** 16 + 1
    x = np.linspace(30.0 - hw, 30.0 + hw, n)
    xx = np.concatenate([[30.0 - hw - 0.5], x, [30.0 + hw + 0.5]])
    v = one_peak(orc, xx, 30.0, w, r, c=c)
    assert v[0] == 0.0 and v[-1] == 0.0      # outside the window
    area = _simpson(v[1:-1], x[1] - x[0])
    expect = ((1 - r) * special.erf(2 * math.sqrt(math.log(2)) * c)
              + r * (2 / math.pi) * math.atan(2 * c))
    assert area == pytest.approx(expect, rel=1e-9)
    if c == 8.0:
        # 1 - (2/pi) atan(16) of the Lorentz area lies outside +-8 FWHM
        assert (2 / math.pi) * math.atan(16) == pytest.approx(0.960263, abs=1e-6)


# ---- window rule ----------------------------------------------------------

def test_window_edges_inclusive(orc):
    # rho = 20, w = 0.125, c = 8: window [19, 21] lands on grid points
    x = 18.0 + 0.125 * np.arange(33)           # 18 .. 22
    lo, hi = orc.windows(x, np.array([0, 1]), np.array([20.0]), 8.0,
                         np.array([[1.0], [0.0], [0.125], [0.5]]))
    assert x[lo[0, 0]] == 19.0 and x[hi[0, 0] - 1] == 21.0


def test_windows_match_brute_force(orc):
    prob = W.make_problem("tiny", seed=11, N=600, K=5, M=12)
    rng = np.random.default_rng(3)
    S, K = 3, prob.K
    phi = np.empty((S, 4, K))
    phi[:, 0] = rng.uniform(0, 100, (S, K))
    phi[:, 1] = rng.normal(0, 0.05, (S, K))
    phi[:, 2] = rng.uniform(0.02, 0.3, (S, K))
    phi[:, 3] = rng.uniform(0, 1, (S, K))
    c = 6.0
    lo, hi = orc.windows(prob.x, prob.peak_off, prob.peak_pos, c, phi)
    for s in range(S):
        for k in range(K):
            for m in range(prob.peak_off[k], prob.peak_off[k + 1]):
                rho = prob.peak_pos[m] + phi[s, 1, k]
                hw = c * phi[s, 2, k]
                inside = np.nonzero((rho - hw <= prob.x) & (prob.x <= rho + hw))[0]
                if len(inside):
                    assert lo[s, m] == inside[0] and hi[s, m] == inside[-1] + 1
                else:
                    assert lo[s, m] == hi[s, m]


# ---- profile (signal eq.: f = B + sum_k h_k C_k) ---------------------------

def _scipy_profile(prob, phi, c=0.0):
    f = prob.bg.copy()
    for k in range(prob.K):
        h, mu, w, r = phi[:, k]
        for m in range(prob.peak_off[k], prob.peak_off[k + 1]):
            rho = prob.peak_pos[m] + mu
            g = stats.norm.pdf(prob.x, rho, w / (2 * math.sqrt(2 * math.log(2))))
            l = stats.cauchy.pdf(prob.x, rho, w / 2)
            v = (1 - r) * g + r * l
            if c > 0:
                v = np.where((rho - c * w <= prob.x) & (prob.x <= rho + c * w), v, 0)
            f += h * prob.peak_int[m] * v
    return f


@pytest.mark.parametrize("c", [0.0, 8.0])
def test_noise_free_profile_reproduced(orc, c):
    prob = W.make_problem("tiny", seed=1001)
    f = orc.profile(prob.x, prob.bg, prob.peak_off, prob.peak_pos,
                    prob.peak_int, c, prob.phi_true)[0]
    ref = _scipy_profile(prob, prob.phi_true, c)
    np.testing.assert_allclose(f, ref, rtol=1e-12)


def test_background_only_at_zero_weight(orc):
    prob = W.make_problem("tiny", seed=5)
    phi = prob.phi_true.copy()
    phi[0] = 0.0
    f = orc.profile(prob.x, prob.bg, prob.peak_off, prob.peak_pos,
                    prob.peak_int, 0.0, phi)[0]
    assert np.array_equal(f, prob.bg)


def test_profile_invariances(orc):
    prob = W.make_problem("tiny", seed=21, K=6, M=15)
    phi = prob.phi_true.copy()
    phi[0] = np.linspace(100, 600, prob.K)
    args = (prob.x, prob.bg)
    f0 = orc.profile(*args, prob.peak_off, prob.peak_pos, prob.peak_int, 0.0, phi)[0]
    # permutation of phases (with their parameters) and of peaks in a phase
    rng = np.random.default_rng(0)
    perm = rng.permutation(prob.K)
    pos, inten, off = [], [], [0]
    for k in perm:
        a, b = prob.peak_off[k], prob.peak_off[k + 1]
        order = rng.permutation(b - a)
        pos.append(prob.peak_pos[a:b][order]); inten.append(prob.peak_int[a:b][order])
        off.append(off[-1] + b - a)
    f1 = orc.profile(*args, np.array(off), np.concatenate(pos),
                     np.concatenate(inten), 0.0, phi[:, perm])[0]
    np.testing.assert_allclose(f1, f0, rtol=1e-13)
    # zero-intensity padding peaks change nothing (the paper's dummy peaks)
    pos2, int2, off2 = [], [], [0]
    for k in range(prob.K):
        a, b = prob.peak_off[k], prob.peak_off[k + 1]
        pos2.append(np.concatenate([prob.peak_pos[a:b], [20.0, 55.0]]))
        int2.append(np.concatenate([prob.peak_int[a:b], [0.0, 0.0]]))
        off2.append(off2[-1] + b - a + 2)
    f2 = orc.profile(*args, np.array(off2), np.concatenate(pos2),
                     np.concatenate(int2), 0.0, phi)[0]
    assert np.array_equal(f2, f0)
    # common translation of grid and peak positions
    f3 = orc.profile(prob.x + 7.5, prob.bg, prob.peak_off, prob.peak_pos + 7.5,
                     prob.peak_int, 0.0, phi)[0]
    np.testing.assert_allclose(f3, f0, rtol=1e-10)


# ---- likelihood and priors -------------------------------------------------

def test_loglik_is_poisson_logpmf(orc):
    rng = np.random.default_rng(4)
    f = rng.uniform(1, 5000, 3000)
    y = rng.poisson(f).astype(float)
    y[:10] = 0.0
    ref = stats.poisson.logpmf(y, f).sum()
    assert orc.loglik(y, f)[0] == pytest.approx(ref, rel=1e-13)


def test_priors_match_library_densities(orc):
    lam = 1 / 3000.0
    for h, mu, w, r in [(10.0, 0.01, 0.05, 0.2), (5000.0, -0.07, 0.2, 0.9),
                        (0.5, 0.0, 0.01, 0.5)]:
        ref = (stats.expon.logpdf(h, scale=1 / lam)
               + stats.norm.logpdf(mu, 0, 0.03)
               + stats.gamma.logpdf(w, a=3.0, scale=1 / 100.0)
               + stats.uniform.logpdf(r, 0, 1))
        assert orc.log_prior(h, mu, w, r, lam) == pytest.approx(ref, rel=1e-13)


# ---- ELBO estimator --------------------------------------------------------

def _small(seed=7, **kw):
    cfg = dict(N=500, K=4, M=6)
    cfg.update(kw)
    prob = W.make_problem("tiny", seed=seed, **cfg)
    return prob


def _y(orc, prob, seed):
    f = orc.profile(prob.x, prob.bg, prob.peak_off, prob.peak_pos,
                    prob.peak_int, 0.0, prob.phi_true)[0]
    return W.poisson_counts(f, seed)


def _transform(z):
    return np.stack([np.exp(z[0]), z[1], np.exp(z[2]), 1 / (1 + np.exp(-z[3]))])


def test_elbo_zero_noise_identity(orc):
    prob = _small()
    y = _y(orc, prob, 1)
    ymax = (y - prob.bg).max()
    loc, logscale = W.random_params(prob.K, 3, ymax)
    S = 3
    eps = np.zeros((S, 4, prob.K))
    e, ll, _, _ = orc.elbo(prob, y, loc, logscale, eps, grad=False)
    phi = _transform(loc)
    f = orc.profile(prob.x, prob.bg, prob.peak_off, prob.peak_pos,
                    prob.peak_int, 0.0, phi)[0]
    ell = stats.poisson.logpmf(y, f).sum()
    lam = 1 / ymax
    lp = sum(stats.expon.logpdf(phi[0, k], scale=1 / lam)
             + stats.norm.logpdf(phi[1, k], 0, 0.03)
             + stats.gamma.logpdf(phi[2, k], a=3, scale=0.01)
             for k in range(prob.K))
    # log|J| of h=e^z, w=e^z, r=logistic(z)
    r = phi[3]
    lj = np.sum(loc[0] + loc[2] + np.log(r) + np.log1p(-r))
    P = 4 * prob.K
    expect = ell + lp + lj + logscale.sum() + P / 2 * (1 + math.log(2 * math.pi))
    assert e == pytest.approx(expect, rel=1e-12)
    assert np.allclose(ll, ell, rtol=1e-12)
    # raising every omega by 3 at eps=0 raises the ELBO by 3P exactly
    e3, _, _, _ = orc.elbo(prob, y, loc, logscale + 3.0, eps, grad=False)
    assert e3 - e == pytest.approx(3 * P, rel=1e-12)


def test_elbo_is_mean_over_samples(orc):
    prob = _small(seed=8)
    y = _y(orc, prob, 2)
    loc, logscale = W.random_params(prob.K, 4, (y - prob.bg).max())
    eps = W.eps_draw(5, prob.K, 9)
    eS, llS, gS, gsS = orc.elbo(prob, y, loc, logscale, eps)
    one = [orc.elbo(prob, y, loc, logscale, eps[s:s + 1]) for s in range(5)]
    assert eS == pytest.approx(np.mean([o[0] for o in one]), rel=1e-12)
    np.testing.assert_allclose(llS, [o[1][0] for o in one], rtol=1e-13)
    np.testing.assert_allclose(gS, np.mean([o[2] for o in one], axis=0),
                               rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("c", [0.0, 8.0])
def test_gradient_matches_central_differences(orc, c):
    prob = _small(seed=12, N=800, K=3, M=5)
    y = _y(orc, prob, 5)
    loc, logscale = W.random_params(prob.K, 6, (y - prob.bg).max(), spread=0.2)
    eps = W.eps_draw(2, prob.K, 13)
    _, _, gl, gs = orc.elbo(prob, y, loc, logscale, eps, c=c)
    h = 1e-5
    lam = 1 / (y - prob.bg).max()
    fd_l, fd_s, an_l, an_s = [], [], [], []
    for t, k in itertools.product(range(4), range(prob.K)):
        for which in (0, 1):
            base = [loc.copy(), logscale.copy()]
            plus = [a.copy() for a in base]; minus = [a.copy() for a in base]
            plus[which][t, k] += h; minus[which][t, k] -= h
            if c > 0:
                # skip coordinates whose window plan moves within +-h
                wins = []
                for pr in (plus, minus):
                    z = pr[0][None] + np.exp(pr[1])[None] * eps
                    wins.append(orc.windows(prob.x, prob.peak_off, prob.peak_pos,
                                            c, np.stack([_transform(zz) for zz in z])))
                if not (np.array_equal(wins[0][0], wins[1][0])
                        and np.array_equal(wins[0][1], wins[1][1])):
                    continue
            ep = orc.elbo(prob, y, *plus, eps, grad=False, c=c, lam=lam)[0]
            em = orc.elbo(prob, y, *minus, eps, grad=False, c=c, lam=lam)[0]
            fd = (ep - em) / (2 * h)
            (fd_l if which == 0 else fd_s).append(fd)
            (an_l if which == 0 else an_s).append((gl if which == 0 else gs)[t, k])
    fd = np.array(fd_l + fd_s); an = np.array(an_l + an_s)
    assert len(fd) >= 16
    scale = np.abs(an).max()
    np.testing.assert_allclose(an, fd, rtol=2e-6, atol=1e-6 * scale)


def test_gradient_vanishes_at_noise_free_truth(orc):
    # y = f* exactly, q concentrated at the truth: the likelihood part of
    # the gradient is zero, leaving prior + Jacobian terms in closed form
    prob = W.make_problem("tiny", seed=31, K=6, M=12)
    keep = prob.true_idx
    off = [0]; pos = []; inten = []
    for k in keep:
        a, b = prob.peak_off[k], prob.peak_off[k + 1]
        pos.append(prob.peak_pos[a:b]); inten.append(prob.peak_int[a:b])
        off.append(off[-1] + b - a)
    sub = W.Problem(x=prob.x, bg=prob.bg, peak_off=np.array(off, np.int32),
                    peak_pos=np.concatenate(pos), peak_int=np.concatenate(inten),
                    cutoff=0.0, true_idx=np.arange(len(keep)),
                    phi_true=prob.phi_true[:, keep])
    phi = sub.phi_true
    y = orc.profile(sub.x, sub.bg, sub.peak_off, sub.peak_pos, sub.peak_int,
                    0.0, phi)[0]
    loc = np.stack([np.log(phi[0]), phi[1], np.log(phi[2]),
                    np.log(phi[3] / (1 - phi[3]))])
    logscale = np.full_like(loc, -30.0)
    eps = W.eps_draw(2, sub.K, 3)
    lam = 1e-3
    _, ll, gl, _ = orc.elbo(sub, y, loc, logscale, eps, lam=lam)
    h, mu, w, r = phi
    expect = np.stack([1 - lam * h, -mu / 0.03 ** 2, 3 - 100 * w, 1 - 2 * r])
    np.testing.assert_allclose(gl, expect, rtol=1e-6, atol=1e-6)
    exact = np.sum(special.xlogy(y, y) - y - special.gammaln(y + 1))
    assert ll[0] == pytest.approx(exact, rel=1e-10)


# ---- selection: brute force over all 2^K phase subsets ---------------------

def test_bruteforce_subset_map(orc):
    prob = W.make_problem("tiny", seed=1003, K=8, M=20)
    phi = prob.phi_true.copy()
    # fixed profile parameters for absent phases
    for k in range(prob.K):
        if k not in prob.true_idx:
            phi[1:, k] = [0.0, 0.1, 0.5]
    K = prob.K
    C = phase_basis(orc, prob, phi)
    fstar = orc.profile(prob.x, prob.bg, prob.peak_off, prob.peak_pos,
                        prob.peak_int, 0.0, phi)[0]
    y = W.poisson_counts(fstar, 77)
    lam = 1 / (y - prob.bg).max()
    obj, hmap, T = map_support(C, y, prob.bg, lam)
    # selection by area ratio above 1 % (Sec. 4): a phase's area is
    # h_k sum_m I_m for unit-area peaks; it recovers the generating phases
    area = np.array([hmap[k] * prob.peak_int[prob.peak_off[k]:prob.peak_off[k + 1]].sum()
                     for k in range(K)])
    selected = np.nonzero(area / area.sum() > 0.01)[0]
    assert selected.tolist() == sorted(prob.true_idx.tolist())
    assert set(selected) <= set(T)
    # KKT through the oracle's gradient: for h_k > 0, d/dh [lnL + ln p] = 0,
    # i.e. the z-gradient equals the Jacobian term 1 (sigma -> 0, eps = 0)
    sub = np.array(T)
    loc = np.stack([np.log(hmap[sub]), phi[1, sub], np.log(phi[2, sub]),
                    np.log(phi[3, sub] / (1 - phi[3, sub]))])
    off = [0]; pos = []; inten = []
    for k in sub:
        a, b = prob.peak_off[k], prob.peak_off[k + 1]
        pos.append(prob.peak_pos[a:b]); inten.append(prob.peak_int[a:b])
        off.append(off[-1] + b - a)
    sp = W.Problem(x=prob.x, bg=prob.bg, peak_off=np.array(off, np.int32),
                   peak_pos=np.concatenate(pos), peak_int=np.concatenate(inten),
                   cutoff=0.0, true_idx=np.arange(len(sub)), phi_true=phi[:, sub])
    _, _, gl, _ = orc.elbo(sp, y, loc, np.full_like(loc, -40.0),
                           np.zeros((1, 4, len(sub))), lam=lam)
    np.testing.assert_allclose(gl[0], 1.0, atol=1e-6)
    # absent phases: the one-sided derivative at h=0 is not positive
    f = prob.bg + C.T @ hmap
    for k in range(K):
        if k not in T:
            assert C[k] @ (y / f - 1) - lam <= 1e-9


# ---- random numbers and optimiser -----------------------------------------

def test_philox_known_answers(orc):
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for row in rows:
        v = [int(t, 16) for t in row]
        assert orc.philox4x32_10(v[0:4], v[4:6]) == v[6:10]


def test_philox_normals_are_standard(orc):
    e = orc.eps_philox(64, 50, seed=12345, step=7)
    assert e.shape == (64, 4, 50)
    assert abs(e.mean()) < 0.05 and abs(e.std() - 1) < 0.05
    assert stats.kstest(e.ravel(), "norm").pvalue > 1e-3
    e2 = orc.eps_philox(64, 50, seed=12345, step=8)
    assert not np.allclose(e, e2)
    # the stream of one sample does not depend on S
    e3 = orc.eps_philox(3, 50, seed=12345, step=7)
    assert np.array_equal(e3, e[:3])


def test_adam_first_step_is_signed_lr(orc):
    th = np.array([1.0, -2.0, 0.5]); m1 = np.zeros(3); m2 = np.zeros(3)
    g = np.array([3.0, -0.01, 0.0])
    orc.adam(th, m1, m2, g, 1, lr=0.01)
    np.testing.assert_allclose(th, [1.01, -2.01, 0.5], rtol=1e-6)


def test_adam_constant_gradient_moves_lr_per_step(orc):
    # Kingma & Ba, Algorithm 1: from zero moments under a constant gradient
    # g, m_t = (1 - b1^t) g and v_t = (1 - b2^t) g^2, so the bias-corrected
    # moments are exactly g and g^2 at every t and each step moves theta by
    # lr g / (|g| + eps).  A correction by (1 - b1) instead of (1 - b1^t)
    # would shrink the moves after the first.
    g = np.array([3.0, -0.25, 1e-3, -40.0])
    th = np.array([0.5, -1.0, 2.0, 0.0]); th0 = th.copy()
    m1 = np.zeros(4); m2 = np.zeros(4)
    lr, e = 0.01, 1e-8
    for t in range(1, 11):
        orc.adam(th, m1, m2, g, t, lr=lr, e=e)
        np.testing.assert_allclose(th, th0 + t * lr * g / (np.abs(g) + e),
                                   rtol=1e-12, atol=1e-14)


def test_adam_two_steps_with_a_sign_change(orc):
    # b1 = 0.9, b2 = 0.999, gradients g1 then g2, worked by hand:
    #   m2 = 0.09 g1 + 0.1 g2,  v2 = 0.000999 g1^2 + 0.001 g2^2,
    #   bias corrections 1 - 0.9^2 = 0.19 and 1 - 0.999^2 = 0.001999.
    # (g1, g2) = (1, -1):  m^ = -0.01 / 0.19 = -1/19, v^ = 1, so the two
    #                      steps move lr (1 - 1/19) = lr 18/19;
    # (g1, g2) = (2, -0.5): m^ = 0.13 / 0.19 = 13/19,
    #                      v^ = 0.004246 / 0.001999 = 4246/1999.
    lr = 0.01
    th = np.zeros(2); m1 = np.zeros(2); m2 = np.zeros(2)
    orc.adam(th, m1, m2, np.array([1.0, 2.0]), 1, lr=lr, e=0.0)
    np.testing.assert_allclose(th, [lr, lr], rtol=1e-13)
    orc.adam(th, m1, m2, np.array([-1.0, -0.5]), 2, lr=lr, e=0.0)
    want = [lr * 18.0 / 19.0, lr + lr * (13.0 / 19.0) / np.sqrt(4246.0 / 1999.0)]
    np.testing.assert_allclose(th, want, rtol=1e-12)
    np.testing.assert_allclose(m1, [-0.01, 0.13], rtol=1e-12)
    np.testing.assert_allclose(m2, [0.001999, 0.004246], rtol=1e-12)


def test_gradient_central_differences_at_stress200_scale(orc):
    # 200 phases x 60 peaks over 10-80 deg (the stress200 candidate set, on a
    # 0.07 deg grid to keep the oracle fast), S = 2, dense: 32 random
    # coordinates of (m, omega) against central differences, h = 1e-5
    prob = W.make_problem("stress200", 3101, N=1001, step=0.07)
    f = orc.profile(prob.x, prob.bg, prob.peak_off, prob.peak_pos,
                    prob.peak_int, 0.0, prob.phi_true)[0]
    y = W.poisson_counts(f, 3102)
    lam = 1 / (y - prob.bg).max()
    loc, ls = W.random_params(prob.K, 3103, (y - prob.bg).max(), spread=0.2)
    eps = W.eps_draw(2, prob.K, 3104)
    _, _, gl, gs = orc.elbo(prob, y, loc, ls, eps, lam=lam, c=0.0)
    rng = np.random.default_rng(3105)
    h = 1e-5
    fd, an = [], []
    for _ in range(32):
        which, t, k = rng.integers(2), rng.integers(4), rng.integers(prob.K)
        plus = [loc.copy(), ls.copy()]
        minus = [loc.copy(), ls.copy()]
        plus[which][t, k] += h
        minus[which][t, k] -= h
        ep = orc.elbo(prob, y, *plus, eps, lam=lam, c=0.0, grad=False)[0]
        em = orc.elbo(prob, y, *minus, eps, lam=lam, c=0.0, grad=False)[0]
        fd.append((ep - em) / (2 * h))
        an.append((gl if which == 0 else gs)[t, k])
    fd, an = np.array(fd), np.array(an)
    np.testing.assert_allclose(an, fd, rtol=2e-6, atol=1e-6 * np.abs(an).max())
