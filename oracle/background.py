"""Asymmetric least squares background (Eilers and Boelens, 2005) in FP64
with a sparse direct solve (TEST INFRASTRUCTURE ONLY).

Starting from unit weights, n_iter times: solve (W + lambda D^T D) z = W y
with D the second-difference matrix and W = diag(w), then set w_i = p where
y_i > z_i and 1 - p elsewhere.  The background is the last z.
"""
from __future__ import annotations

import numpy as np
from scipy import sparse
from scipy.sparse.linalg import spsolve


def second_difference(N):
    """The (N-2) x N matrix with rows (1, -2, 1)."""
    return sparse.diags([1.0, -2.0, 1.0], [0, 1, 2], shape=(N - 2, N))


def asls(y, lam, p, n_iter):
    y = np.asarray(y, dtype=np.float64)
    N = len(y)
    if N < 3:
        return y.copy()
    D = second_difference(N)
    P = (lam * (D.T @ D)).tocsc()
    w = np.ones(N)
    for it in range(n_iter):
        z = spsolve((sparse.diags(w) + P).tocsc(), w * y)
        if it + 1 < n_iter:
            w = np.where(y > z, p, 1.0 - p)
    return z
