"""CPU checks of the C-ABI library: it loads, exports every declared symbol,
and its host-side validation rejects malformed problems (no GPU call)."""
import ctypes as C

import numpy as np
import pytest

from paper_2501_09308_amd import workloads as W
from paper_2501_09308_amd import xrdvi as X


def test_library_exports_every_declared_symbol():
    lib = X.load()
    names = X.exported_symbols()
    assert len(names) >= 14
    for n in ["xrdvi_profile", "xrdvi_window_plan", "xrdvi_elbo_fwd",
              "xrdvi_elbo_bwd"]:
        assert n in names
    for n in names:
        assert hasattr(lib, n), n
    assert lib.xrdvi_version() == 1


def _args(**over):
    prob = W.make_problem("tiny", seed=3, N=300, K=3, M=4)
    kw = dict(x=prob.x, y=np.full(prob.N, 60.0), bg=prob.bg,
              peak_off=prob.peak_off, peak_pos=prob.peak_pos,
              peak_int=prob.peak_int, cutoff=0.0)
    kw.update(over)
    return kw


def test_validate_accepts_good_problem():
    assert X.xrdvi_validate(**_args()) == 0
    assert X.xrdvi_validate(**_args(asymmetric=True)) == 0
    assert X.xrdvi_validate(**_args(width_law="sec")) == 0
    assert X.xrdvi_validate(**_args(asymmetric=True, width_law=1)) == 0


def test_validate_rejects_unknown_width_law():
    d, keep = X.make_desc(**_args())
    d.width_law = 2
    lib = X.load()
    assert lib.xrdvi_validate(C.byref(d)) == X.XRDVI_EINVAL
    assert b"width_law" in lib.xrdvi_last_error()


def test_validate_rejects_unknown_asymmetry_flag():
    d, keep = X.make_desc(**_args())
    d.asymmetric = 2
    lib = X.load()
    assert lib.xrdvi_validate(C.byref(d)) == X.XRDVI_EINVAL
    assert b"asymmetric" in lib.xrdvi_last_error()


@pytest.mark.parametrize("mutate,msg", [
    (lambda a: a.update(x=a["x"][::-1].copy()), "ascending"),
    (lambda a: a.update(x=np.concatenate([[0.0], a["x"][1:]])), "(0, 180)"),
    (lambda a: a.update(bg=np.zeros_like(a["bg"])), "bg"),
    (lambda a: a.update(y=np.concatenate([[-1.0], a["y"][1:]])), "y must"),
    (lambda a: a.update(y=a["bg"].copy()), "max(y - bg)"),
    (lambda a: a.update(peak_off=np.array([0, 3, 2, 12])), "non-decreasing"),
    (lambda a: a.update(peak_off=np.array([1, 4, 8, 12])), "peak_off[0]"),
    (lambda a: a.update(peak_int=a["peak_int"] * 2), "[0, 1]"),
    (lambda a: a.update(cutoff=-1.0), "cutoff"),
    (lambda a: a.update(mu_sd=0.0), "mu_sd"),
    (lambda a: a.update(w_rate=-1.0), "w_rate"),
    (lambda a: a.update(peak_pos=np.full_like(a["peak_pos"], np.nan)), "finite"),
    (lambda a: a.update(asymmetric=True, alpha_sd=0.0), "alpha_sd"),
    (lambda a: a.update(asymmetric=True, alpha_mean=np.inf), "alpha_mean"),
    (lambda a: a.update(width_law=1, peak_pos=np.concatenate(
        [[180.0], a["peak_pos"][1:]])), "inside (0, 180)"),
    (lambda a: a.update(width_law=1, peak_pos=np.concatenate(
        [[-1.0], a["peak_pos"][1:]])), "inside (0, 180)"),
])
def test_validate_rejects(mutate, msg):
    a = _args()
    mutate(a)
    with pytest.raises(X.XrdviError) as ei:
        X.xrdvi_validate(**a)
    assert ei.value.code == X.XRDVI_EINVAL
    assert msg in str(ei.value)


def test_validate_explicit_lambda_allows_flat_counts():
    a = _args()
    a["y"] = a["bg"].copy()
    assert X.xrdvi_validate(**a, lambda_h=1e-4) == 0


def test_null_description_is_rejected():
    lib = X.load()
    assert lib.xrdvi_validate(None) == X.XRDVI_EINVAL
    assert b"NULL" in lib.xrdvi_last_error()


def test_request_footprint_is_host_only_and_grows_with_the_request():
    prob = W.make_problem("tiny", seed=3, N=300, K=3, M=4)
    y = np.full(prob.N, 60.0)
    small = X.request_footprint(prob, y, S=4, steps=10)
    assert small > 0 and small % 256 == 0
    assert X.request_footprint(prob, y, S=32, steps=10) > small
    assert X.request_footprint(prob, y, S=4, steps=5000) > small
    big = W.make_problem("tiny", seed=3, N=3000, K=30, M=40)
    assert X.request_footprint(big, np.full(big.N, 60.0), S=4, steps=10) > small
    with pytest.raises(X.XrdviError) as ei:
        X.request_footprint(prob, y, S=0, steps=10)
    assert ei.value.code == X.XRDVI_EINVAL
