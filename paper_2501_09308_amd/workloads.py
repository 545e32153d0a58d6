"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws random numbers and lays them out; it contains none of
the method's arithmetic (no peak shape, no likelihood, no prior).  Both the
HIP path and the FP64 oracle take their inputs from here.

Stand-ins: the paper measures one TiO2 diffractogram (Cu K-alpha1, 2-theta
10-60 deg at 0.02 deg, Sec. 3.1) against 50 candidate phases from a crystal
database.  Neither is available, so every workload is synthetic: a 2-theta
grid, K candidate phases with ragged peak lists (Appendix A.1: positions
p in (0,180) deg, relative intensities I in [0,1]), a few "true" phases with
weights, shifts, widths and Lorentz fractions, a flat background, and
Poisson counts drawn around the noise-free profile (the noise-free profile
itself is computed by whoever calls ``poisson_counts``).
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

# Named workloads: the grid, candidate count, peaks per candidate, true
# phases, samples per step and window cutoff of each configuration the hot
# path is measured on.
WORKLOADS = {
    # tiny: one sample, dense, 8 candidates x 20 peaks
    "tiny": dict(x0=10.0, step=0.02, N=3501, K=8, M=20, n_true=2, S=1,
                 cutoff=0.0, fwhm=(0.05, 0.2)),
    # paper scale: 50 candidates (2^50 phase subsets), 40 peaks each, S=64
    "paper50": dict(x0=10.0, step=0.02, N=3501, K=50, M=40, n_true=3, S=64,
                    cutoff=0.0, fwhm=(0.05, 0.2)),
    "paper50_w8": dict(x0=10.0, step=0.02, N=3501, K=50, M=40, n_true=3,
                       S=64, cutoff=8.0, fwhm=(0.05, 0.2)),
    # differentiation stress: K=200 x 60 peaks, N=7001, S=128
    "stress200": dict(x0=10.0, step=0.01, N=7001, K=200, M=60, n_true=4,
                      S=128, cutoff=0.0, fwhm=(0.05, 0.2)),
    # database screening: K=2000 x 100 peaks, N=14001, windows at 8 FWHM
    "db2000": dict(x0=10.0, step=0.01, N=14001, K=2000, M=100, n_true=6,
                   S=32, cutoff=8.0, fwhm=(0.03, 0.3)),
}

PEAK_SCALE = 1.0e4      # area (counts*deg) of an I=1 peak at weight 1
BACKGROUND = 50.0       # flat background, counts


@dataclasses.dataclass
class Problem:
    """One diffractogram and its candidate set (host arrays, FP64)."""
    x: np.ndarray            # [N] 2-theta, strictly ascending
    bg: np.ndarray           # [N] background > 0
    peak_off: np.ndarray     # [K+1] int32 CSR offsets
    peak_pos: np.ndarray     # [sum M_k] positions (deg)
    peak_int: np.ndarray     # [sum M_k] relative intensities in [0,1]
    cutoff: float            # window half-width in FWHM units (0 = dense)
    true_idx: np.ndarray     # indices of the generating phases
    phi_true: np.ndarray     # [4][K] constrained (h, mu, w, r) of the truth
    y: Optional[np.ndarray] = None   # [N] counts, filled by poisson_counts

    @property
    def N(self) -> int:
        return int(self.x.shape[0])

    @property
    def K(self) -> int:
        return int(self.peak_off.shape[0] - 1)

    @property
    def total_peaks(self) -> int:
        return int(self.peak_off[-1])


def make_problem(name_or_cfg, seed: int, **overrides) -> Problem:
    """Draw one synthetic problem.  ``y`` is left unset."""
    cfg = dict(WORKLOADS[name_or_cfg]) if isinstance(name_or_cfg, str) \
        else dict(name_or_cfg)
    cfg.update(overrides)
    rng = np.random.default_rng(seed)
    N, K = int(cfg["N"]), int(cfg["K"])
    x0, step = float(cfg["x0"]), float(cfg["step"])
    # grid: x_i = x0 + i*step, not cumulated
    x = x0 + step * np.arange(N, dtype=np.float64)
    bg = np.full(N, BACKGROUND, dtype=np.float64)
    if "M_range" in cfg:
        lo, hi = cfg["M_range"]
        M = rng.integers(lo, hi + 1, size=K)
    else:
        M = np.full(K, int(cfg["M"]))
    off = np.zeros(K + 1, dtype=np.int32)
    off[1:] = np.cumsum(M)
    xmin, xmax = float(x[0]), float(x[-1])
    pos = np.empty(off[-1]); inten = np.empty(off[-1])
    for k in range(K):
        a, b = off[k], off[k + 1]
        pos[a:b] = rng.uniform(xmin, xmax, size=b - a)
        u = rng.uniform(0.0, 1.0, size=b - a)
        I = u ** 3
        I = I / I.max()          # strongest peak of each phase = 1
        inten[a:b] = I
    n_true = int(cfg["n_true"])
    true_idx = np.sort(rng.choice(K, size=n_true, replace=False))
    f_lo, f_hi = cfg["fwhm"]
    phi = np.zeros((4, K))
    phi[2, :] = 0.1          # width/ratio of absent phases: irrelevant (h=0)
    phi[3, :] = 0.5
    for k in true_idx:
        phi[0, k] = PEAK_SCALE * rng.uniform(0.3, 1.0)   # h
        phi[1, k] = rng.uniform(-0.05, 0.05)             # mu (shift)
        phi[2, k] = rng.uniform(f_lo, f_hi)              # w (FWHM)
        phi[3, k] = rng.uniform(0.0, 1.0)                # r (Lorentz frac.)
    return Problem(x=x, bg=bg, peak_off=off, peak_pos=pos, peak_int=inten,
                   cutoff=float(cfg["cutoff"]), true_idx=true_idx,
                   phi_true=phi)


def make_serving_problem(seed: int) -> Problem:
    """One request of the serving mix: N in [2000,12000], step in
    [0.01,0.035] clipped so the grid ends at or below 170 deg, K in
    [20,300], 20-80 peaks per phase, 1-5 true phases, windows at 8 FWHM."""
    rng = np.random.default_rng(seed)
    N = int(rng.integers(2000, 12001))
    step = float(rng.uniform(0.01, 0.035))
    step = min(step, (170.0 - 10.0) / (N - 1))
    K = int(rng.integers(20, 301))
    n_true = int(rng.integers(1, 6))
    cfg = dict(x0=10.0, step=step, N=N, K=K, M_range=(20, 80), n_true=n_true,
               S=32, cutoff=8.0, fwhm=(0.05, 0.2))
    return make_problem(cfg, seed=int(rng.integers(1 << 31)))


def poisson_counts(fstar: np.ndarray, seed: int) -> np.ndarray:
    """Observed counts y ~ Poisson(f*) for a noise-free profile f*."""
    rng = np.random.default_rng(seed)
    return rng.poisson(np.asarray(fstar, dtype=np.float64)).astype(np.float64)


def eps_draw(S: int, K: int, seed: int, step: int = 0, D: int = 4) -> np.ndarray:
    """Standard-normal reparameterisation noise [S][D][K] for one step."""
    rng = np.random.default_rng([seed, step])
    return rng.standard_normal((S, D, K))


def random_params(K: int, seed: int, y_max: float, spread: float = 0.3,
                  D: int = 4):
    """Variational parameters (loc, logscale) [D][K] scattered around the
    default initialisation, for parity tests away from any optimum."""
    rng = np.random.default_rng(seed)
    loc, logscale = init_params(K, y_max, D)
    loc = loc + spread * rng.standard_normal((D, K))
    logscale = logscale + spread * rng.standard_normal((D, K))
    return loc, logscale


def init_params(K: int, y_max: float, D: int = 4):
    """Default initial variational parameters (unconstrained space):
    m_h = ln(0.01*y_max), m_mu = 0, m_w = ln 0.1, m_r = 0 (and m_alpha = 0
    when D = 5), omega = ln 0.1."""
    loc = np.zeros((D, K))
    loc[0, :] = np.log(0.01 * y_max)
    loc[1, :] = 0.0
    loc[2, :] = np.log(0.1)
    loc[3, :] = 0.0
    logscale = np.full((D, K), np.log(0.1))
    return loc, logscale


def arrival_times(n: int, rate: float, seed: int) -> np.ndarray:
    """Poisson arrival process: cumulative exponential gaps (seconds)."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def random_phi(K: int, S: int, seed: int, h_max: float = 2.0e4,
               w_range=(0.03, 0.3)) -> np.ndarray:
    """Constrained latents [S][4][K] scattered over the prior's range:
    h ~ U(0, h_max), mu ~ N(0, 0.03), w ~ U(w_range), r ~ U(0, 1)."""
    rng = np.random.default_rng(seed)
    phi = np.empty((S, 4, K))
    phi[:, 0] = rng.uniform(0.0, h_max, (S, K))
    phi[:, 1] = rng.normal(0.0, 0.03, (S, K))
    phi[:, 2] = rng.uniform(w_range[0], w_range[1], (S, K))
    phi[:, 3] = rng.uniform(0.0, 1.0, (S, K))
    return phi


def random_alpha(K: int, S: int, seed: int, lo: float = 0.6,
                 hi: float = 1.8) -> np.ndarray:
    """Asymmetries alpha [S][K] ~ U(lo, hi), to append to random_phi as the
    fifth latent row."""
    rng = np.random.default_rng([seed, 5])
    return rng.uniform(lo, hi, (S, K))
