"""Shared helpers of the GPU parity tests: seeded cases whose observed
counts come from the oracle's noise-free profile."""
import functools

import numpy as np
import torch

import oracle
from paper_2501_09308_amd import workloads as W
from paper_2501_09308_amd import xrdvi as X


@functools.lru_cache(maxsize=None)
def context():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    return X.Context(0)


def counts(prob, seed):
    fstar = oracle.profile(prob.x, prob.bg, prob.peak_off, prob.peak_pos,
                           prob.peak_int, 0.0, prob.phi_true)[0]
    return W.poisson_counts(fstar, seed)


def case(name, seed, **over):
    prob = W.make_problem(name, seed, **over)
    y = counts(prob, seed + 7)
    return prob, y


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64,
                           device="cuda")


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
