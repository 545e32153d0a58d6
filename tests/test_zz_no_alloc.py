"""The allocation-free profile entry point (xrdvi_profile_static) against
xrdvi_profile through the C ABI: two calls in a row on one GPU, the second
with a smaller problem and sample count, dense and windowed, each output
equal bit for bit to xrdvi_profile's (same kernels, same order) and within
the profile bar of the FP64 oracle; a request whose per-call state exceeds
the static scratch is rejected on the host."""
import numpy as np
import pytest
import torch

import oracle
from paper_2501_09308_amd import workloads as W
from paper_2501_09308_amd import xrdvi as X

from gpu_common import case, context, dev

pytestmark = pytest.mark.gpu

PROFILE_RTOL = 1e-5


def _one(ctx, name, seed, S, c, **over):
    prob, y = case(name, seed, **over)
    P = X.Problem.from_workload(ctx, prob, y, cutoff=c)
    phi = W.random_phi(prob.K, S, seed + 1)
    ref = X.xrdvi_profile(ctx, P, dev(phi)).cpu().numpy()
    out = torch.full((S, prob.N), float("nan"), dtype=torch.float32, device="cuda")
    X.xrdvi_profile_static(ctx, P, dev(phi), out)
    f = out.cpu().numpy()
    assert np.array_equal(f, ref), f"{name} S={S} c={c}: differs from xrdvi_profile"
    o = oracle.profile(prob.x, prob.bg, prob.peak_off, prob.peak_pos,
                       prob.peak_int, c, phi)
    err = float(np.max(np.abs(f - o) / o))
    print(f"\nstatic profile {name} N={prob.N} K={prob.K} S={S} c={c}: "
          f"bitwise equal to xrdvi_profile, max rel vs oracle {err:.2e}")
    assert err <= PROFILE_RTOL


@pytest.mark.parametrize("c", [0.0, 8.0])
def test_static_profile_equals_profile_twice_second_smaller(c):
    ctx = context()
    _one(ctx, "paper50", 7101, 16, c)                      # larger first
    _one(ctx, "tiny", 7102, 3, c, N=900, K=5, M=12)        # then smaller


def test_static_profile_rejects_state_beyond_the_scratch():
    ctx = context()
    prob, y = case("paper50", 7103)
    P = X.Problem.from_workload(ctx, prob, y)
    S = 1024                       # dense per-call state of about 73 MB
    phi = dev(W.random_phi(prob.K, S, 7104))
    out = torch.empty((S, prob.N), dtype=torch.float32, device="cuda")
    with pytest.raises(X.XrdviError) as ei:
        X.xrdvi_profile_static(ctx, P, phi, out)
    assert ei.value.code == X.XRDVI_EINVAL
    assert "static scratch" in str(ei.value)
