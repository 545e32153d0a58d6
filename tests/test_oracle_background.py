"""Pins of the oracle's asymmetric-least-squares background (Eilers and
Boelens 2005): limits with closed forms and recovery of a known smooth
baseline under positive peaks; plus the library's argument checks."""
import numpy as np
import pytest

from oracle import background as BG
from paper_2501_09308_amd import xrdvi as X


def test_no_penalty_reproduces_the_data():
    y = np.random.default_rng(1).uniform(10, 100, 200)
    np.testing.assert_allclose(BG.asls(y, 0.0, 0.01, 5), y, rtol=1e-12)


def test_infinite_penalty_is_the_weighted_straight_line():
    # lambda -> infinity removes all curvature: one iteration with w = 1 is
    # the least-squares line through the data
    # (N small enough that lambda can dwarf the smallest non-zero
    # eigenvalue of D^T D, about (pi / N)^4, without ruining the solve)
    rng = np.random.default_rng(2)
    i = np.arange(30.0)
    y = 40 + 0.1 * i + rng.normal(0, 3, i.size)
    z = BG.asls(y, 1e9, 0.01, 1)
    line = np.polyval(np.polyfit(i, y, 1), i)
    np.testing.assert_allclose(z, line, rtol=2e-6)


def test_recovers_a_smooth_baseline_under_positive_peaks():
    x = np.linspace(10, 80, 3501)
    base = 50 + 30 * np.exp(-(x - 10) / 25) + 0.002 * (x - 45) ** 2
    peaks = sum(a * (0.05 ** 2 / ((x - c) ** 2 + 0.05 ** 2))
                for a, c in [(800, 20.3), (500, 33.1), (900, 47.7), (300, 61.2), (650, 72.4)])
    z = BG.asls(base + peaks, 1e7, 0.001, 15)
    # within 2 % of the baseline away from the ends and 3 % at the ends
    # (peaks are 6-18x the baseline)
    err = np.abs(z - base) / base
    assert np.max(err[(x > 12) & (x < 78)]) < 0.02
    assert np.max(err) < 0.03


def test_library_rejects_bad_arguments():
    lib = X.load()
    assert lib.xrdvi_background(None, 1, 10, None, 1.0, 0.01, 3, None, None,
                                None) == X.XRDVI_EINVAL
