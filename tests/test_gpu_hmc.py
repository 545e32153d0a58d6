"""GPU parity of the log posterior density and of Hamiltonian Monte Carlo
(the sampling method the paper compares stochastic VI with, Sec. 4 and
Table 1) against the FP64 oracle, through the C ABI."""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import hmc as OH
from paper_2501_09308_amd import workloads as W
from paper_2501_09308_amd import xrdvi as X

from gpu_common import case, context, counts, dev, rel_l2

pytestmark = pytest.mark.gpu


def _positions(prob, y, C, seed, D=4, spread=0.05):
    """Positions near the generating parameters (unconstrained)."""
    rng = np.random.default_rng(seed)
    h = np.where(prob.phi_true[0] > 0, prob.phi_true[0], 0.02 * (y - prob.bg).max())
    base = np.stack([np.log(h), prob.phi_true[1], np.log(prob.phi_true[2]),
                     np.log(prob.phi_true[3] / (1 - prob.phi_true[3]))])
    if D == 5:
        base = np.concatenate([base, np.zeros((1, prob.K))])
    return base[None] + spread * rng.standard_normal((C, D, prob.K))


# dense cases run the 16-wave tile (16 tiles x 6 chains is a small grid)
@pytest.mark.parametrize("c,asym,law", [(0.0, False, 0), (8.0, False, 0),
                                        (0.0, True, 0), (3.0, True, 0),
                                        (0.0, False, "sec"), (8.0, True, "sec")])
def test_logpost_and_gradient_match_oracle(c, asym, law):
    prob, y = case("paper50", 801, N=2000, K=12, M=15)
    prob.cutoff = c
    ctx = context()
    P = X.Problem.from_workload(ctx, prob, y, cutoff=c, asymmetric=asym,
                                width_law=law)
    C = 6
    z = _positions(prob, y, C, 802, D=P.D)
    tape = X.Tape(ctx, P, C)
    lp, g = X.xrdvi_logpost(ctx, P, tape, dev(z))
    lp, g = lp.cpu().numpy(), g.cpu().numpy()
    for s in range(C):
        rl, rg = OH.logpost(prob, y, z[s], asymmetric=asym, width_law=law)
        assert abs(lp[s] - rl) <= 1e-6 * abs(rl)
        assert rel_l2(g[s], rg) <= 1e-4


def test_short_hmc_run_matches_oracle():
    prob = W.make_problem("tiny", seed=811, N=1500, K=4, M=8, n_true=2)
    y = counts(prob, 812)
    ctx = context()
    P = X.Problem.from_workload(ctx, prob, y)
    C, warm, keep, L, eps0, seed = 4, 3, 3, 3, 2e-5, 4711
    z0 = _positions(prob, y, C, 813, spread=0.01)
    z = dev(z0)
    out = X.xrdvi_hmc(ctx, P, z, warm, keep, L, eps0, seed)

    def fn(x):
        v, gr = OH.logpost(prob, y, x.reshape(4, prob.K))
        return v, gr.ravel()

    ref = OH.run(fn, z0.reshape(C, -1), seed, warm, keep, L, eps0)
    # a chain is compared while no Metropolis decision was within rounding
    # of its threshold (FP32 peak values against FP64 ones)
    ok = [all(abs(it[c][1]) > 1e-3 for it in ref["decisions"]) for c in range(C)]
    assert sum(ok) >= 3
    d = out["draws"].cpu().numpy().reshape(keep, C, -1)
    for c in range(C):
        if not ok[c]:
            continue
        np.testing.assert_allclose(d[:, c], ref["draws"][:, c], rtol=1e-5, atol=1e-7)
        np.testing.assert_allclose(out["logp"].cpu().numpy()[:, c], ref["logp"][:, c],
                                   rtol=1e-6)
        assert out["step"][c] == pytest.approx(ref["step"][c], rel=1e-5)
        assert out["accept"][c] == ref["accept"][c]
    np.testing.assert_allclose(z.cpu().numpy()[ok], d[-1][ok].reshape(-1, 4, prob.K))


def test_hmc_samples_concentrate_on_the_generating_weights():
    prob = W.make_problem("tiny", seed=821, N=2000, K=5, M=12, n_true=2)
    y = counts(prob, 822)
    ctx = context()
    P = X.Problem.from_workload(ctx, prob, y)
    z = dev(_positions(prob, y, 8, 823, spread=0.02))
    out = X.xrdvi_hmc(ctx, P, z, 200, 200, 8, 1e-5, 99)
    d = out["draws"].cpu().numpy()
    assert np.all(out["accept"] > 0.4)
    assert np.all(np.isfinite(out["logp"].cpu().numpy()))
    # posterior mean weights of the generating phases within 10 % of truth
    hm = np.exp(d[:, :, 0, :]).mean(axis=(0, 1))
    t = prob.true_idx
    np.testing.assert_allclose(hm[t], prob.phi_true[0, t], rtol=0.1)
