"""GPU parity of the angle-dependent width (FWHM w sec(rho / 2); Appendix
A.2 defines sec for the lost width formula) against the FP64 oracle,
through the C ABI, for symmetric and asymmetric peaks, dense and windowed:
profile relative error <= 1e-5, window plans bit for bit, ELBO relative
<= 1e-6, gradient relative L2 <= 1e-4.  Grids reach 160-170 deg, where
sec(theta) exceeds 5 and, for the wider peaks, the window bounds stop being
monotone in the peak position (the tile plan then covers whole phases)."""
import numpy as np
import pytest

import oracle
from paper_2501_09308_amd import workloads as W
from paper_2501_09308_amd import xrdvi as X

from gpu_common import context, dev, rel_l2

pytestmark = pytest.mark.gpu

PROFILE_RTOL = 1e-5
ELBO_RTOL = 1e-6
GRAD_RTOL = 1e-4

# grids: 20-160 deg at 0.04 (N = 3501), 120-170 deg at 0.02 (N = 2501)
WIDE = dict(x0=20.0, step=0.04, N=3501)
HIGH = dict(x0=120.0, step=0.02, N=2501)


def _phi(K, S, seed, D):
    phi = W.random_phi(K, S, seed)
    if D == 5:
        phi = np.concatenate([phi, W.random_alpha(K, S, seed)[:, None, :]], axis=1)
    return phi


def _case(name, seed, D, **over):
    """Problem with counts drawn from a sec-law truth."""
    prob = W.make_problem(name, seed, **over)
    phi_true = prob.phi_true
    if D == 5:
        phi_true = np.concatenate([phi_true, W.random_alpha(prob.K, 1, seed + 3)])
    fstar = oracle.profile_sec(prob.x, prob.bg, prob.peak_off, prob.peak_pos,
                               prob.peak_int, 0.0, phi_true)[0]
    return prob, W.poisson_counts(fstar, seed + 7)


def _problem(prob, y, c, D):
    return X.Problem.from_workload(context(), prob, y, cutoff=c,
                                   asymmetric=D == 5, width_law="sec")


PROFILE_CASES = [
    ("tiny", 801, WIDE, 2, 0.0, 4),
    ("paper50", 802, WIDE, 8, 0.0, 4),
    ("paper50", 803, WIDE, 8, 8.0, 4),
    ("paper50", 804, WIDE, 8, 0.0, 5),
    ("paper50", 805, WIDE, 8, 8.0, 5),
    ("paper50", 806, HIGH, 4, 8.0, 4),                       # fallback ranges
    ("paper50", 807, HIGH, 4, 8.0, 5),
    ("paper50", 808, dict(WIDE, N=1000), 4, 3.0, 5),         # ragged last tile
    ("stress200", 809, dict(WIDE, K=300, M=20, N=3001), 2, 8.0, 4),  # LDS staged
    ("stress200", 810, dict(WIDE, K=300, M=20, N=3001), 2, 8.0, 5),
    ("stress200", 811, dict(HIGH, K=260, M=100, N=600), 2, 8.0, 4),  # overflow
]


@pytest.mark.parametrize("name,seed,over,S,c,D", PROFILE_CASES)
def test_sec_profile_matches_oracle(name, seed, over, S, c, D):
    prob, y = _case(name, seed, D, **over)
    P = _problem(prob, y, c, D)
    phi = _phi(prob.K, S, seed, D)
    f = X.xrdvi_profile(context(), P, dev(phi)).cpu().numpy()
    ref = oracle.profile_sec(prob.x, prob.bg, prob.peak_off, prob.peak_pos,
                             prob.peak_int, c, phi)
    err = np.max(np.abs(f - ref) / ref)
    print(f"\nsec profile {name} N={prob.N} K={prob.K} S={S} c={c} D={D}: "
          f"max rel {err:.3e}")
    assert err <= PROFILE_RTOL


@pytest.mark.parametrize("D", [4, 5])
@pytest.mark.parametrize("over", [WIDE, HIGH])
def test_sec_window_plan_bit_exact(D, over):
    prob, y = _case("paper50", 820, D, **over)
    c = 8.0
    P = _problem(prob, y, c, D)
    phi = _phi(prob.K, 16, 821, D)
    lo, hi = X.xrdvi_window_plan(context(), P, dev(phi))
    rlo, rhi = oracle.windows_sec(prob.x, prob.peak_off, prob.peak_pos, c, phi)
    assert np.array_equal(lo.cpu().numpy(), rlo)
    assert np.array_equal(hi.cpu().numpy(), rhi)


ELBO_CASES = [
    ("tiny", 901, WIDE, 1, 0.0, 4),
    ("paper50", 902, WIDE, 64, 0.0, 4),
    ("paper50", 903, WIDE, 64, 8.0, 4),
    ("paper50", 904, WIDE, 16, 0.0, 5),
    ("paper50", 905, WIDE, 16, 8.0, 5),
    ("paper50", 906, HIGH, 8, 8.0, 4),
    ("paper50", 907, HIGH, 8, 0.0, 5),
    ("stress200", 908, dict(WIDE, K=300, M=20, N=3001), 3, 8.0, 4),
    ("stress200", 909, dict(WIDE, K=300, M=20, N=3001), 3, 8.0, 5),
]


def _elbo_case(name, seed, over, S, c, D):
    prob, y = _case(name, seed, D, **over)
    prob.cutoff = c
    P = _problem(prob, y, c, D)
    ymax = (y - prob.bg).max()
    loc, logscale = W.random_params(prob.K, seed, ymax, D=D)
    eps = W.eps_draw(S, prob.K, seed, D=D)
    return prob, y, P, loc, logscale, eps


@pytest.mark.parametrize("name,seed,over,S,c,D", ELBO_CASES)
def test_sec_elbo_and_gradient_match_oracle(name, seed, over, S, c, D):
    prob, y, P, loc, logscale, eps = _elbo_case(name, seed, over, S, c, D)
    ctx = context()
    tape = X.Tape(ctx, P, S)
    e, ll = X.xrdvi_elbo_fwd(ctx, P, tape, dev(loc), dev(logscale), eps=dev(eps))
    gl, gs = X.xrdvi_elbo_bwd(ctx, tape)
    re, rll, rgl, rgs = oracle.elbo_sec(prob, y, loc, logscale, eps)
    e = e.item()
    erel = abs(e - re) / abs(re)
    llrel = np.max(np.abs(ll.cpu().numpy() - rll) / np.abs(rll))
    gln, gsn = gl.cpu().numpy(), gs.cpu().numpy()
    grel = rel_l2(np.concatenate([gln.ravel(), gsn.ravel()]),
                  np.concatenate([rgl.ravel(), rgs.ravel()]))
    gmu = rel_l2(np.concatenate([gln[1], gsn[1]]), np.concatenate([rgl[1], rgs[1]]))
    print(f"\nsec elbo {name} S={S} c={c} D={D}: rel {erel:.2e}; loglik "
          f"{llrel:.2e}; grad rel-L2 {grel:.2e} (mu rows {gmu:.2e})")
    assert erel <= ELBO_RTOL
    assert llrel <= ELBO_RTOL
    assert grel <= GRAD_RTOL
    assert gmu <= GRAD_RTOL


def _wait(srv, tickets, timeout=120.0):
    import time
    out, t0 = {}, time.time()
    while len(out) < len(tickets):
        for t in tickets:
            if t not in out:
                rc, info, res = srv.poll(t)
                if rc != X.XRDVI_PENDING:
                    out[t] = (rc, info, res)
        assert time.time() - t0 < timeout, "server did not finish"
        time.sleep(0.002)
    return out


@pytest.mark.parametrize("cutoff,D", [(8.0, 4), (0.0, 5)])
def test_sec_served_trajectory_matches_oracle(cutoff, D):
    prob, y = _case("paper50", 950, D, **dict(WIDE, N=1500, K=6, M=10, n_true=2))
    prob.cutoff = cutoff
    S, steps, seed = 4, 5, 8765
    srv = X.Server(max_slots=4, steps_per_launch=2, arena_bytes=1 << 28)
    t = srv.submit(prob, y, S, steps, seed, lr=0.01, asymmetric=D == 5,
                   width_law="sec")
    rc, info, res = _wait(srv, [t])[t]
    srv.close()
    assert rc == X.XRDVI_OK
    loc, ls = W.init_params(prob.K, float((y - prob.bg).max()), D=D)
    m = [np.zeros((D, prob.K)) for _ in range(4)]
    trace = []
    for n in range(steps):
        eps = oracle.eps_philox(S, prob.K, seed, n, D=D)
        e, _, gl, gs = oracle.elbo_sec(prob, y, loc, ls, eps)
        trace.append(e)
        oracle.adam(loc, m[0], m[1], gl, n + 1, lr=0.01)
        oracle.adam(ls, m[2], m[3], gs, n + 1, lr=0.01)
    np.testing.assert_allclose(res["trace"], trace, rtol=1e-6)
    np.testing.assert_allclose(res["loc"], loc, rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(res["logscale"], ls, rtol=1e-6, atol=1e-6)


def test_sec_analyses_in_a_constant_width_mix_match_plain_runs():
    # the server switches to its graph with the sec-law kernels while a
    # sec-law analysis is resident and back when none is
    ctx = context()
    a, ya = _case("paper50", 960, 4, **dict(WIDE, N=2500, K=10, M=12, n_true=2))
    a.cutoff = 8.0
    b, yb = _case("paper50", 961, 5, **dict(WIDE, N=1800, K=7, M=9, n_true=2))
    b.cutoff = 0.0
    S, steps = 6, 8
    ref_a = X.xrdvi_plain_run(ctx, a, ya, S, steps, 5, width_law="sec")
    ref_b = X.xrdvi_plain_run(ctx, b, yb, S, steps, 6, asymmetric=True,
                              width_law="sec")
    ref_c = X.xrdvi_plain_run(ctx, a, ya, 4, 30, 7)
    srv = X.Server(max_slots=6, steps_per_launch=3, arena_bytes=1 << 28)
    tc = srv.submit(a, ya, 4, 30, 7)                 # constant width, longest
    ta = srv.submit(a, ya, S, steps, 5, width_law="sec")
    tb = srv.submit(b, yb, S, steps, 6, asymmetric=True, width_law="sec")
    res = _wait(srv, [tc, ta, tb])
    srv.close()
    assert all(r[0] == X.XRDVI_OK for r in res.values())
    for t, ref in ((ta, ref_a), (tb, ref_b), (tc, ref_c)):
        for k in ("loc", "logscale", "trace"):
            np.testing.assert_allclose(res[t][2][k], ref[k], rtol=1e-12, atol=1e-12)
