"""GPU parity on non-uniform grids (the C ABI takes any strictly ascending
grid): a jittered scan and two merged scans of different step.  The window
step's and the windowed tile's grid searches start from a uniform-grid
guess; on these grids the guess misses, so their fall-back steps (further
probes, then bisection) run.  Checks the window plan bit for bit, the
profile (max relative 1e-5), the ELBO (relative 1e-6) and the gradient
(relative L2 1e-4) against the FP64 oracle, with the constant and the sec
width law."""
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


def _grid(kind, rng):
    if kind == "jitter":        # 0.02 deg steps, each point moved by up to 0.006
        return 10.0 + 0.02 * np.arange(3000) + rng.uniform(-0.006, 0.006, 3000)
    # two scans: 10-25 deg at 0.01, then 25-70 deg at 0.03
    return np.concatenate([10.0 + 0.01 * np.arange(1500), 25.0 + 0.03 * np.arange(1500)])


def _problem(kind, seed, c):
    rng = np.random.default_rng(seed)
    x = _grid(kind, rng)
    K, M = 30, 20
    off = (M * np.arange(K + 1)).astype(np.int32)
    pos = rng.uniform(x[0], x[-1], K * M)
    inten = rng.uniform(0.0, 1.0, K * M) ** 3
    phi = np.zeros((4, K))
    phi[2], phi[3] = 0.1, 0.5
    true = rng.choice(K, 3, replace=False)
    phi[0, true] = W.PEAK_SCALE * rng.uniform(0.3, 1.0, 3)
    phi[1, true] = rng.uniform(-0.05, 0.05, 3)
    phi[2, true] = rng.uniform(0.03, 0.2, 3)
    phi[3, true] = rng.uniform(0.0, 1.0, 3)
    return W.Problem(x=x, bg=np.full(x.size, W.BACKGROUND), peak_off=off,
                     peak_pos=pos, peak_int=inten, cutoff=c, true_idx=np.sort(true),
                     phi_true=phi)


@pytest.mark.parametrize("sec", [False, True])
@pytest.mark.parametrize("c", [0.0, 8.0])
@pytest.mark.parametrize("kind", ["jitter", "two_scans"])
def test_non_uniform_grid_matches_oracle(kind, c, sec):
    seed = {"jitter": 501, "two_scans": 502}[kind] + (10 if sec else 0)
    prob = _problem(kind, seed, c)
    if sec:
        prof, wins, elbo = oracle.profile_sec, oracle.windows_sec, oracle.elbo_sec
    else:
        prof, wins, elbo = oracle.profile, oracle.windows, oracle.elbo
    fstar = prof(prob.x, prob.bg, prob.peak_off, prob.peak_pos, prob.peak_int, 0.0,
                 prob.phi_true)[0]
    y = W.poisson_counts(fstar, seed + 1)
    ctx = context()
    P = X.Problem.from_workload(ctx, prob, y, cutoff=c, width_law="sec" if sec else 0)
    S = 4
    phi = W.random_phi(prob.K, S, seed + 2)
    f = X.xrdvi_profile(ctx, P, dev(phi)).cpu().numpy()
    ref = prof(prob.x, prob.bg, prob.peak_off, prob.peak_pos, prob.peak_int, c, phi)
    err = np.max(np.abs(f - ref) / ref)
    print(f"\n{kind} c={c} sec={sec}: profile max rel {err:.2e}", flush=True)
    assert err <= PROFILE_RTOL
    if c > 0.0:
        lo, hi = X.xrdvi_window_plan(ctx, P, dev(phi))
        rlo, rhi = wins(prob.x, prob.peak_off, prob.peak_pos, c, phi)
        assert np.array_equal(lo.cpu().numpy(), rlo)
        assert np.array_equal(hi.cpu().numpy(), rhi)
    loc, ls = W.random_params(prob.K, seed + 3, float((y - prob.bg).max()))
    eps = W.eps_draw(S, prob.K, seed + 4)
    tape = X.Tape(ctx, P, S)
    e, ll = X.xrdvi_elbo_fwd(ctx, P, tape, dev(loc), dev(ls), eps=dev(eps))
    gl, gs = X.xrdvi_elbo_bwd(ctx, tape)
    re, rll, rgl, rgs = elbo(prob, y, loc, ls, eps)
    assert abs(e.item() - re) <= ELBO_RTOL * abs(re)
    np.testing.assert_allclose(ll.cpu().numpy(), rll, rtol=ELBO_RTOL)
    g = np.concatenate([gl.cpu().numpy().ravel(), gs.cpu().numpy().ravel()])
    assert rel_l2(g, np.concatenate([rgl.ravel(), rgs.ravel()])) <= GRAD_RTOL


@pytest.mark.parametrize("asym", [False, True])
def test_grid_step_records_agree_with_degree_records(asym):
    """On a uniform grid the constant-width forward stages its records in
    grid steps (exact point offsets); one point moved by 3e-9 of a step
    (beyond the 1e-9 the uniformity test allows, far below any physical
    effect) sends the same problem down the degree-coordinate path.  Both
    profiles match the FP64 oracle within the profile bar, and each other
    within 2e-6, symmetric and asymmetric."""
    rng = np.random.default_rng(530 + asym)
    N, K, M = 2500, 40, 30
    x = 10.0 + 0.02 * np.arange(N)
    off = (M * np.arange(K + 1)).astype(np.int32)
    pos = rng.uniform(x[0], x[-1], K * M)
    inten = rng.uniform(0.0, 1.0, K * M) ** 3
    ctx = context()
    S = 4
    phi = W.random_phi(K, S, 531 + asym)
    if asym:
        phi = np.concatenate([phi, rng.uniform(0.8, 1.3, (S, 1, K))], axis=1)
    x2 = x.copy()
    x2[N // 2] += 3e-9 * 0.02
    out = []
    for xx in (x, x2):
        P = X.Problem(ctx, xx, np.ones(N), np.full(N, W.BACKGROUND), off, pos, inten,
                      8.0, lambda_h=1.0, asymmetric=asym)
        out.append(X.xrdvi_profile(ctx, P, dev(phi)).cpu().numpy())
        P.close()
    prof = oracle.profile_asym if asym else oracle.profile
    ref = prof(x, np.full(N, W.BACKGROUND), off, pos, inten, 8.0, phi)
    e_steps = np.max(np.abs(out[0] - ref) / ref)
    e_deg = np.max(np.abs(out[1] - ref) / ref)
    e_both = np.max(np.abs(out[0] - out[1]) / ref)
    print(f"\nasym={asym}: grid steps {e_steps:.2e}, degrees {e_deg:.2e}, "
          f"between {e_both:.2e}", flush=True)
    assert e_steps <= PROFILE_RTOL and e_deg <= PROFILE_RTOL
    assert e_both <= 2e-6
