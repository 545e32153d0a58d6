"""Converged stochastic VI and its posterior readout (Sec. 4): 1000
optimisation steps of whole analyses on the GPU server, then the phases
whose area ratio exceeds 1 % must be the generating phases and the support
of the exact MAP found by enumerating all 2^K phase subsets (K = 10, profile
parameters fixed, oracle arithmetic), with area ratios near the generating
ones (the paper compares its estimate with the prepared mixing ratio)."""
import time

import numpy as np
import pytest

import oracle
from paper_2501_09308_amd import workloads as W
from paper_2501_09308_amd import xrdvi as X

from gpu_common import counts
from selection_common import area_ratios, map_support, phase_basis

pytestmark = pytest.mark.gpu

SEEDS = (9011, 9012, 9013)


def _wait(srv, tickets, timeout=120.0):
    out, t0 = {}, time.time()
    while len(out) < len(tickets):
        for t in tickets:
            if t not in out:
                rc, info, res = srv.poll(t)
                if rc != X.XRDVI_PENDING:
                    out[t] = (rc, info, res)
        assert time.time() - t0 < timeout, "server did not finish"
        time.sleep(0.005)
    return out


def _map_ratios(prob, y):
    phi = prob.phi_true.copy()
    for k in range(prob.K):
        if k not in prob.true_idx:
            phi[1:, k] = [0.0, 0.1, 0.5]
    C = phase_basis(oracle, prob, phi)
    _, h, _ = map_support(C, y, prob.bg, 1.0 / (y - prob.bg).max())
    return area_ratios(prob, h)


def test_converged_svi_selects_the_brute_force_map_support():
    cases = []
    srv = X.Server(max_slots=8, steps_per_launch=50, arena_bytes=1 << 30)
    for seed in SEEDS:
        prob = W.make_problem("tiny", seed=seed, K=10, M=20, n_true=3)
        y = counts(prob, seed + 100)
        cases.append((prob, y, srv.submit(prob, y, 16, 1000, seed, lr=0.05)))
    res = _wait(srv, [t for _, _, t in cases])
    srv.close()
    for prob, y, t in cases:
        rc, info, out = res[t]
        assert rc == X.XRDVI_OK
        rd = X.xrdvi_readout(prob.peak_off, prob.peak_int, out["loc"],
                             out["logscale"], threshold=0.01)
        truth = sorted(prob.true_idx.tolist())
        map_ratio = _map_ratios(prob, y)
        true_ratio = area_ratios(prob, prob.phi_true[0])
        sel = rd["selected"].tolist()
        print(f"\nselected {sel} truth {truth} "
              f"svi {np.round(rd['area_ratio'][truth], 4)} "
              f"map {np.round(map_ratio[truth], 4)} true {np.round(true_ratio[truth], 4)} "
              f"sd/mean {np.round(rd['sd_h'][truth] / rd['mean_h'][truth], 4)}")
        assert sel == truth
        assert np.nonzero(map_ratio > 0.01)[0].tolist() == truth
        assert np.max(np.abs(rd["area_ratio"][truth] - true_ratio[truth])) <= 0.03
        assert np.all(rd["sd_h"][truth] / rd["mean_h"][truth] < 0.05)
        # the ELBO estimate rose over the run
        assert out["trace"][-1] > out["trace"][0]
