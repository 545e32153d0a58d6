"""GPU asymmetric-least-squares background against the oracle's sparse
direct solve (same reweighting), through the C ABI."""
import numpy as np
import pytest
import torch

from oracle import background as BG
from paper_2501_09308_amd import workloads as W
from paper_2501_09308_amd import xrdvi as X

from gpu_common import context, counts

pytestmark = pytest.mark.gpu


# grids from one partition block (N < 18) through two (18, 21), 64 blocks
# of the minimum 8 rows (655) and long blocks (7001)
@pytest.mark.parametrize("N,lam,p,n_iter", [(3501, 1e6, 0.01, 10),
                                            (1200, 1e5, 0.05, 4),
                                            (7001, 1e7, 0.001, 6),
                                            (655, 1e4, 0.01, 5),
                                            (21, 100.0, 0.05, 3),
                                            (18, 100.0, 0.05, 3),
                                            (17, 50.0, 0.05, 3),
                                            (3, 10.0, 0.1, 3),
                                            (2, 1.0, 0.1, 2)])
def test_background_matches_oracle(N, lam, p, n_iter):
    ys = []
    for b in range(3):
        prob = W.make_problem("tiny", seed=900 + b, N=max(N, 3), K=4, M=10,
                              step=min(0.02, 69.0 / max(N, 3)))
        ys.append(counts(prob, 950 + b)[:N])
    y = np.stack(ys)
    out = X.xrdvi_background(context(), torch.as_tensor(y, device="cuda"), lam, p,
                             n_iter).cpu().numpy()
    # two different direct solves of W + lambda D^T D agree, normwise, to
    # about its condition number, at most (1 + 16 lambda / p), times the
    # FP64 epsilon
    rtol = 2.0 * (1.0 + 16.0 * lam / p) * 2.2e-16
    for b in range(3):
        ref = BG.asls(y[b], lam, p, n_iter)
        err = np.max(np.abs(out[b] - ref)) / np.max(np.abs(ref))
        assert err <= max(rtol, 1e-12), (err, rtol)
