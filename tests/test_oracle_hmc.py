"""Pins of the oracle's Hamiltonian Monte Carlo (test infrastructure):
leapfrog reversibility and second-order energy error on the XRD posterior,
and exact sampling of a standard normal target (mean, variance and the
dual-averaged acceptance rate)."""
import math

import numpy as np
import pytest

import oracle
from oracle import hmc
from paper_2501_09308_amd import workloads as W

from gpu_common import counts


def _xrd(seed=71):
    prob = W.make_problem("tiny", seed=seed, N=1200, K=3, M=6, n_true=2)
    y = counts(prob, seed + 1)
    z = np.stack([np.log(prob.phi_true[0] + 50.0), prob.phi_true[1],
                  np.log(prob.phi_true[2]), np.zeros(prob.K)])
    return prob, y, z


def test_logpost_is_the_zero_noise_elbo_without_entropy():
    prob, y, z = _xrd()
    lp, g = hmc.logpost(prob, y, z)
    ll = oracle.loglik(y, oracle.profile(prob.x, prob.bg, prob.peak_off,
                                         prob.peak_pos, prob.peak_int, 0.0,
                                         np.stack([np.exp(z[0]), z[1], np.exp(z[2]),
                                                   1 / (1 + np.exp(-z[3]))])[None]))[0]
    lam = 1 / (y - prob.bg).max()
    prior = sum(oracle.log_prior(math.exp(z[0, k]), z[1, k], math.exp(z[2, k]),
                                 1 / (1 + math.exp(-z[3, k])), lam)
                for k in range(prob.K))
    r = 1 / (1 + np.exp(-z[3]))
    logj = np.sum(z[0] + z[2] + np.log(r) + np.log1p(-r))
    assert lp == pytest.approx(ll + prior + logj, rel=1e-12)
    assert g.shape == z.shape


def test_leapfrog_is_reversible_and_second_order():
    prob, y, z = _xrd()
    n = z.size

    def fn(x):
        v, gr = hmc.logpost(prob, y, x.reshape(z.shape))
        return v, gr.reshape(n)

    lp0, g0 = fn(z.ravel())
    p0 = hmc.momenta(1, n, 5, 0)[0]
    # the posterior is stiff (|grad| ~ 1e5 in z near the truth), so the
    # integrator is stable only for small steps
    eps = 1e-5
    z1, p1, lp1, g1 = hmc.leapfrog(fn, z.ravel(), p0, g0, eps, 12)
    zb, pb, lpb, _ = hmc.leapfrog(fn, z1, -p1, g1, eps, 12)
    np.testing.assert_allclose(zb, z.ravel(), rtol=0, atol=1e-9)
    np.testing.assert_allclose(-pb, p0, rtol=0, atol=1e-7)

    def dH(e):
        zz, pp, ll, _ = hmc.leapfrog(fn, z.ravel(), p0, g0, e, round(12 * eps / e))
        return (-ll + 0.5 * pp @ pp) - (-lp0 + 0.5 * p0 @ p0)

    ratio = dH(eps) / dH(eps / 2)
    assert 3.0 < ratio < 5.0


def test_standard_normal_target_is_sampled_exactly():
    n, C = 3, 48

    def fn(x):
        return -0.5 * float(x @ x), -x

    rng = np.random.default_rng(0)
    out = hmc.run(fn, rng.normal(size=(C, n)) * 3.0, seed=11, n_warmup=150,
                  n_draws=200, n_leapfrog=4, step_size=0.05)
    d = out["draws"].reshape(-1, n)
    # effective sample size is below C * n_draws; 5 standard errors of the
    # independent-draw error are still a tight check of the correction
    se = 1.0 / math.sqrt(d.shape[0])
    assert np.all(np.abs(d.mean(axis=0)) < 5 * se * 3)
    assert np.all(np.abs(d.var(axis=0) - 1.0) < 0.1)
    assert 0.65 < out["accept"].mean() < 0.95
