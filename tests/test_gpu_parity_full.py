"""GPU parity at the full sizes of the larger workloads: the ELBO, every
per-sample log-likelihood and the gradient at the stated sample counts,
plus window-plan properties and sampled profile points.

stress200: N=7001 (10-80 deg at 0.01), K=200 x 60 peaks, S=128, dense.
db2000:    N=14001 (10-150 deg at 0.01), K=2000 x 100 peaks, S=32, c=8.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2501_09308_amd import workloads as W
from paper_2501_09308_amd import xrdvi as X

from gpu_common import context, counts, dev, rel_l2

pytestmark = pytest.mark.gpu


def subgrid(prob, idx):
    return W.Problem(x=prob.x[idx], bg=prob.bg[idx], peak_off=prob.peak_off,
                     peak_pos=prob.peak_pos, peak_int=prob.peak_int,
                     cutoff=prob.cutoff, true_idx=prob.true_idx,
                     phi_true=prob.phi_true)


@pytest.fixture(scope="module")
def stress():
    prob = W.make_problem("stress200", 3001)
    y = counts(prob, 3002)
    return prob, y


@pytest.fixture(scope="module")
def db():
    prob = W.make_problem("db2000", 5001)
    # counts: the generating phases only contribute; profile them alone
    keep = prob.true_idx
    off = [0]; pos = []; inten = []
    for k in keep:
        a, b = prob.peak_off[k], prob.peak_off[k + 1]
        pos.append(prob.peak_pos[a:b]); inten.append(prob.peak_int[a:b])
        off.append(off[-1] + b - a)
    f = oracle.profile(prob.x, prob.bg, np.array(off), np.concatenate(pos),
                       np.concatenate(inten), 0.0, prob.phi_true[:, keep])[0]
    y = W.poisson_counts(f, 5002)
    return prob, y


def _compare(tag, e, ll, g, re, rll, rg):
    erel = abs(e - re) / abs(re)
    lrel = np.max(np.abs(ll - rll) / np.abs(rll))
    grel = rel_l2(g, rg)
    print(f"\n{tag}: elbo rel {erel:.2e}, max loglik rel {lrel:.2e}, "
          f"grad rel-L2 {grel:.2e}")
    assert erel <= 1e-6 and lrel <= 1e-6
    assert grel <= 1e-4


def test_stress200_full_size_S128_through_autograd(stress):
    """The stated differentiation-stress configuration as a whole: N=7001,
    K=200 x 60, S=128 (two 64-sample groups in the gradient and ELBO
    reductions), forward and recomputing adjoint through the autograd
    Function; every per-sample log-likelihood, the ELBO and the full
    gradient against the oracle (Sec. 3.2: the estimate and its gradient
    are averages of per-sample terms)."""
    prob, y = stress
    ctx = context()
    P = X.Problem.from_workload(ctx, prob, y)
    S = 128
    loc, logscale = W.random_params(prob.K, 3003, (y - prob.bg).max())
    eps = W.eps_draw(S, prob.K, 3004)
    tape = X.Tape(ctx, P, S)
    L = dev(loc).requires_grad_(True)
    Ls = dev(logscale).requires_grad_(True)
    out = X.elbo(ctx, P, tape, L, Ls, eps=dev(eps))
    out.backward()
    # the tape keeps the per-sample log-likelihoods of that forward
    _, ll = X.xrdvi_elbo_fwd(ctx, P, tape, dev(loc), dev(logscale), eps=dev(eps),
                             need_grad=False)
    re, rll, rgl, rgs = oracle.elbo(prob, y, loc, logscale, eps)
    g = np.concatenate([L.grad.cpu().numpy().ravel(), Ls.grad.cpu().numpy().ravel()])
    _compare("stress200 S=128", out.item(), ll.cpu().numpy(), g, re, rll,
             np.concatenate([rgl.ravel(), rgs.ravel()]))


def test_stress200_sample_count_not_a_multiple_of_64():
    """S = 100 (a full and a partial 64-sample group) on a shorter grid."""
    prob = W.make_problem("stress200", 3011, N=1500)
    y = counts(prob, 3012)
    ctx = context()
    P = X.Problem.from_workload(ctx, prob, y)
    S = 100
    loc, logscale = W.random_params(prob.K, 3013, (y - prob.bg).max())
    eps = W.eps_draw(S, prob.K, 3014)
    tape = X.Tape(ctx, P, S)
    e, ll = X.xrdvi_elbo_fwd(ctx, P, tape, dev(loc), dev(logscale), eps=dev(eps))
    gl, gs = X.xrdvi_elbo_bwd(ctx, tape)
    re, rll, rgl, rgs = oracle.elbo(prob, y, loc, logscale, eps)
    g = np.concatenate([gl.cpu().numpy().ravel(), gs.cpu().numpy().ravel()])
    _compare("stress200 N=1500 S=100", e.item(), ll.cpu().numpy(), g, re, rll,
             np.concatenate([rgl.ravel(), rgs.ravel()]))


def test_db2000_window_plan_properties(db):
    prob, y = db
    ctx = context()
    P = X.Problem.from_workload(ctx, prob, y)
    S = 4
    phi = W.random_phi(prob.K, S, 5003, w_range=(0.03, 0.3))
    lo, hi = X.xrdvi_window_plan(ctx, P, dev(phi))
    lo, hi = lo.cpu().numpy().astype(np.int64), hi.cpu().numpy().astype(np.int64)
    c, x, N = prob.cutoff, prob.x, prob.N
    phase = np.repeat(np.arange(prob.K), np.diff(prob.peak_off))
    for s in range(S):
        rho = prob.peak_pos + phi[s, 1, phase]      # one rounded FP64 add
        hw = c * phi[s, 2, phase]                   # one rounded FP64 multiply
        a, b = rho - hw, rho + hw
        l, h = lo[s], hi[s]
        assert np.all((0 <= l) & (l <= h) & (h <= N))
        ne = h > l
        assert np.all(x[l[ne]] >= a[ne]) and np.all(x[h[ne] - 1] <= b[ne])
        assert np.all((l[ne] == 0) | (x[np.maximum(l[ne] - 1, 0)] < a[ne]))
        assert np.all((h[ne] == N) | (x[np.minimum(h[ne], N - 1)] > b[ne]))
        # empty windows hold no grid point
        e = ~ne
        ins = np.searchsorted(x, a[e], side="left")
        assert np.all((ins >= N) | (x[np.minimum(ins, N - 1)] > b[e]))


def test_db2000_profile_on_sampled_points(db):
    prob, y = db
    ctx = context()
    P = X.Problem.from_workload(ctx, prob, y)
    S = 2
    phi = W.random_phi(prob.K, S, 5004, h_max=2000.0, w_range=(0.03, 0.3))
    f = X.xrdvi_profile(ctx, P, dev(phi)).cpu().numpy()
    idx = np.sort(np.random.default_rng(5).choice(prob.N, 300, replace=False))
    sub = subgrid(prob, idx)
    ref = oracle.profile(sub.x, sub.bg, sub.peak_off, sub.peak_pos, sub.peak_int,
                         prob.cutoff, phi)
    err = np.max(np.abs(f[:, idx] - ref) / ref)
    print(f"\ndb2000 sampled profile max rel {err:.2e}")
    assert err <= 1e-5


def test_db2000_full_size_S32_device_noise(db):
    """The stated database-screening configuration as a whole: N=14001,
    K=2000 x 100, S=32, c=8, with the device's Philox noise (the oracle
    draws the same numbers from its own generator).  Two runs are bitwise
    equal; all 32 per-sample log-likelihoods, the ELBO and the gradient
    match the oracle."""
    prob, y = db
    ctx = context()
    P = X.Problem.from_workload(ctx, prob, y)
    S = 32
    loc, logscale = W.random_params(prob.K, 5007, (y - prob.bg).max())
    tape = X.Tape(ctx, P, S)
    outs = []
    for _ in range(2):
        e, ll = X.xrdvi_elbo_fwd(ctx, P, tape, dev(loc), dev(logscale), eps=None,
                                 seed=11, step=3)
        gl, gs = X.xrdvi_elbo_bwd(ctx, tape)
        outs.append([t.cpu().numpy().copy() for t in (e, ll, gl, gs)])
    for a, b in zip(*outs):
        assert np.array_equal(a, b) and np.all(np.isfinite(a))
    eps = oracle.eps_philox(S, prob.K, 11, 3)
    re, rll, rgl, rgs = oracle.elbo(prob, y, loc, logscale, eps)
    e, ll, gl, gs = outs[0]
    g = np.concatenate([gl.ravel(), gs.ravel()])
    _compare("db2000 S=32", float(e[0]), ll, g, re, rll,
             np.concatenate([rgl.ravel(), rgs.ravel()]))
