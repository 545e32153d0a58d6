"""Posterior readout (Sec. 4, selection of phases by area ratio above 1 %):
the oracle pinned to scipy's log-normal moments, and the library's host
readout (no GPU work) against the oracle."""
import numpy as np
import pytest
from scipy import stats

import oracle
from paper_2501_09308_amd import workloads as W
from paper_2501_09308_amd import xrdvi as X


def _case(seed, K=12):
    prob = W.make_problem("tiny", seed=seed, K=K, M=15)
    rng = np.random.default_rng(seed)
    m = rng.normal(5.0, 3.0, K)
    ls = rng.normal(-2.0, 1.0, K)
    return prob, m, ls


def test_oracle_readout_matches_lognormal_moments():
    prob, m, ls = _case(1)
    mean, sd, ratio, sel = oracle.readout(prob.peak_off, prob.peak_int, m, ls)
    ref = stats.lognorm(s=np.exp(ls), scale=np.exp(m))
    np.testing.assert_allclose(mean, ref.mean(), rtol=1e-13)
    np.testing.assert_allclose(sd, ref.std(), rtol=1e-12)
    isum = np.add.reduceat(prob.peak_int, prob.peak_off[:-1])
    np.testing.assert_allclose(ratio, ref.mean() * isum / (ref.mean() * isum).sum(),
                               rtol=1e-13)
    assert ratio.sum() == pytest.approx(1.0, abs=1e-14)
    assert sel.tolist() == np.nonzero(ratio > 0.01)[0].tolist()


def test_oracle_readout_equal_phases_split_evenly():
    # three identical phases with identical posteriors: 1/3 each
    off = np.array([0, 2, 4, 6]); I = np.array([1.0, 0.5] * 3)
    _, _, ratio, sel = oracle.readout(off, I, np.full(3, 2.0), np.full(3, -1.0))
    np.testing.assert_allclose(ratio, 1 / 3, rtol=1e-15)
    assert sel.tolist() == [0, 1, 2]


@pytest.mark.parametrize("seed", [2, 3, 4])
def test_library_readout_matches_oracle(seed):
    prob, m, ls = _case(seed)
    out = X.xrdvi_readout(prob.peak_off, prob.peak_int, m[None], ls[None],
                          threshold=0.02)
    mean, sd, ratio, sel = oracle.readout(prob.peak_off, prob.peak_int, m, ls,
                                          threshold=0.02)
    np.testing.assert_allclose(out["mean_h"], mean, rtol=1e-14)
    # the library uses expm1, the oracle exp(s^2) - 1
    np.testing.assert_allclose(out["sd_h"], sd, rtol=1e-12)
    np.testing.assert_allclose(out["area_ratio"], ratio, rtol=1e-14)
    assert out["selected"].tolist() == sel.tolist()


def test_library_readout_rejects_bad_input():
    prob, m, ls = _case(5)
    with pytest.raises(X.XrdviError) as ei:
        X.xrdvi_readout(prob.peak_off, np.zeros_like(prob.peak_int), m[None], ls[None])
    assert ei.value.code == X.XRDVI_EINVAL
    with pytest.raises(X.XrdviError):
        X.xrdvi_readout(prob.peak_off, prob.peak_int, m[None], ls[None], threshold=1.5)
