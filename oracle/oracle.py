"""ctypes binding of the FP64 oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
benchmark's CPU-baseline leg; never by the product path.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_D = C.POINTER(C.c_double)
_I = C.POINTER(C.c_int)


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, FP64, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off",
               "-fopenmp", "-fPIC", "-shared", "-std=c11", "-D_GNU_SOURCE",
               _SRC, "-o", _LIB + ".tmp", "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = C.CDLL(_LIB)
    lib.oracle_profile.argtypes = [C.c_int, C.c_int, _D, _D, _I, _D, _D,
                                   C.c_double, C.c_int, _D, _D]
    lib.oracle_windows.argtypes = [C.c_int, C.c_int, _D, _I, _D, C.c_double,
                                   C.c_int, _D, _I, _I]
    lib.oracle_loglik.argtypes = [C.c_int, C.c_int, _D, _D, _D]
    lib.oracle_log_prior.argtypes = [C.c_double] * 8
    lib.oracle_log_prior.restype = C.c_double
    lib.oracle_elbo.argtypes = ([C.c_int, C.c_int, _D, _D, _D, _I, _D, _D]
                                + [C.c_double] * 5
                                + [C.c_int, _D, _D, _D, _D, _D, _D, _D])
    lib.oracle_adam.argtypes = [C.c_int, _D, _D, _D, _D, C.c_int,
                                C.c_double, C.c_double, C.c_double,
                                C.c_double]
    lib.oracle_philox4x32_10.argtypes = [C.POINTER(C.c_uint32),
                                         C.POINTER(C.c_uint32),
                                         C.POINTER(C.c_uint32)]
    lib.oracle_eps_philox.argtypes = [C.c_int, C.c_int, C.c_uint64,
                                      C.c_uint64, _D]
    lib.oracle_eps_philox_n.argtypes = lib.oracle_eps_philox.argtypes
    lib.oracle_readout.argtypes = [C.c_int, _I, _D, _D, _D, C.c_double,
                                   _D, _D, _D, _I]
    lib.oracle_num_threads.restype = C.c_int
    lib.oracle_set_threads.argtypes = [C.c_int]
    lib.oracle_profile_asym.argtypes = lib.oracle_profile.argtypes
    lib.oracle_windows_asym.argtypes = lib.oracle_windows.argtypes
    lib.oracle_elbo_asym.argtypes = ([C.c_int, C.c_int, _D, _D, _D, _I, _D, _D]
                                     + [C.c_double] * 7
                                     + [C.c_int, _D, _D, _D, _D, _D, _D, _D])
    lib.oracle_profile_sec.argtypes = [C.c_int, C.c_int, _D, _D, _I, _D, _D,
                                       C.c_double, C.c_int, C.c_int, _D, _D]
    lib.oracle_windows_sec.argtypes = [C.c_int, C.c_int, _D, _I, _D,
                                       C.c_double, C.c_int, C.c_int, _D, _I,
                                       _I]
    lib.oracle_elbo_sec.argtypes = ([C.c_int, C.c_int, _D, _D, _D, _I, _D, _D]
                                    + [C.c_double] * 7
                                    + [C.c_int, C.c_int, _D, _D, _D, _D, _D,
                                       _D, _D])
    _lib = lib
    return lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_D)


def _i(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_I)


def profile(x, B, peak_off, p, I, c, phi):
    """f[S][N] for constrained phi[S][4][K]."""
    lib = load()
    phi = np.asarray(phi, dtype=np.float64)
    if phi.ndim == 2:
        phi = phi[None]
    S, _, K = phi.shape
    N = len(x)
    f = np.empty((S, N))
    keep = [_d(x), _d(B), _i(peak_off), _d(p), _d(I), _d(phi)]
    rc = lib.oracle_profile(N, K, keep[0][1], keep[1][1], keep[2][1],
                            keep[3][1], keep[4][1], float(c), S, keep[5][1],
                            f.ctypes.data_as(_D))
    assert rc == 0, rc
    return f


def windows(x, peak_off, p, c, phi):
    lib = load()
    phi = np.asarray(phi, dtype=np.float64)
    if phi.ndim == 2:
        phi = phi[None]
    S, _, K = phi.shape
    T = int(peak_off[-1])
    lo = np.empty((S, T), dtype=np.int32)
    hi = np.empty((S, T), dtype=np.int32)
    keep = [_d(x), _i(peak_off), _d(p), _d(phi)]
    lib.oracle_windows(len(x), K, keep[0][1], keep[1][1], keep[2][1],
                       float(c), S, keep[3][1], lo.ctypes.data_as(_I),
                       hi.ctypes.data_as(_I))
    return lo, hi


def loglik(y, f):
    lib = load()
    f = np.ascontiguousarray(np.atleast_2d(f), dtype=np.float64)
    S, N = f.shape
    out = np.empty(S)
    yy = _d(y)
    lib.oracle_loglik(N, S, yy[1], f.ctypes.data_as(_D),
                      out.ctypes.data_as(_D))
    return out


def log_prior(h, mu, w, r, lam, mu_sd=0.03, w_shape=3.0, w_rate=100.0):
    return load().oracle_log_prior(h, mu, w, r, lam, mu_sd, w_shape, w_rate)


def elbo(prob, y, loc, logscale, eps, *, lam=0.0, mu_sd=0.03, w_shape=3.0,
         w_rate=100.0, grad=True, c=None):
    """Returns (elbo, loglik[S], grad_loc[4][K], grad_logscale[4][K])."""
    lib = load()
    eps = np.ascontiguousarray(eps, dtype=np.float64)
    S = eps.shape[0]
    K = prob.K
    cut = prob.cutoff if c is None else c
    gl = np.empty((4, K)); gs = np.empty((4, K))
    ll = np.empty(S)
    out = C.c_double(0.0)
    keep = [_d(prob.x), _d(y), _d(prob.bg), _i(prob.peak_off),
            _d(prob.peak_pos), _d(prob.peak_int), _d(loc), _d(logscale),
            _d(eps)]
    rc = lib.oracle_elbo(prob.N, K, keep[0][1], keep[1][1], keep[2][1],
                         keep[3][1], keep[4][1], keep[5][1], float(cut),
                         float(lam), float(mu_sd), float(w_shape),
                         float(w_rate), S, keep[6][1], keep[7][1], keep[8][1],
                         C.byref(out), ll.ctypes.data_as(_D),
                         gl.ctypes.data_as(_D) if grad else None,
                         gs.ctypes.data_as(_D) if grad else None)
    if rc != 0:
        raise ValueError(f"oracle_elbo failed: {rc}")
    return out.value, ll, (gl if grad else None), (gs if grad else None)


def adam(theta, m1, m2, g, t, lr=1e-2, b1=0.9, b2=0.999, e=1e-8):
    """In-place Adam ascent step on float64 arrays."""
    lib = load()
    for a in (theta, m1, m2):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    gg = _d(g)
    lib.oracle_adam(theta.size, theta.ctypes.data_as(_D),
                    m1.ctypes.data_as(_D), m2.ctypes.data_as(_D), gg[1],
                    int(t), lr, b1, b2, e)


def philox4x32_10(ctr, key):
    lib = load()
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib.oracle_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def eps_philox(S, K, seed, step, D=4):
    """Device noise [S][D][K] of (seed, step)."""
    lib = load()
    out = np.empty((S, D, K))
    lib.oracle_eps_philox_n(S, D * K, C.c_uint64(seed), C.c_uint64(step),
                            out.ctypes.data_as(_D))
    return out


def profile_asym(x, B, peak_off, p, I, c, phi):
    """f[S][N] for constrained phi[S][5][K] (h, mu, w, r, alpha)."""
    lib = load()
    phi = np.asarray(phi, dtype=np.float64)
    if phi.ndim == 2:
        phi = phi[None]
    S, _, K = phi.shape
    f = np.empty((S, len(x)))
    keep = [_d(x), _d(B), _i(peak_off), _d(p), _d(I), _d(phi)]
    rc = lib.oracle_profile_asym(len(x), K, keep[0][1], keep[1][1], keep[2][1],
                                 keep[3][1], keep[4][1], float(c), S,
                                 keep[5][1], f.ctypes.data_as(_D))
    assert rc == 0, rc
    return f


def windows_asym(x, peak_off, p, c, phi):
    lib = load()
    phi = np.asarray(phi, dtype=np.float64)
    if phi.ndim == 2:
        phi = phi[None]
    S, _, K = phi.shape
    T = int(peak_off[-1])
    lo = np.empty((S, T), dtype=np.int32)
    hi = np.empty((S, T), dtype=np.int32)
    keep = [_d(x), _i(peak_off), _d(p), _d(phi)]
    lib.oracle_windows_asym(len(x), K, keep[0][1], keep[1][1], keep[2][1],
                            float(c), S, keep[3][1], lo.ctypes.data_as(_I),
                            hi.ctypes.data_as(_I))
    return lo, hi


def elbo_asym(prob, y, loc, logscale, eps, *, lam=0.0, mu_sd=0.03,
              w_shape=3.0, w_rate=100.0, alpha_mean=1.0, alpha_sd=0.2,
              grad=True, c=None):
    """Asymmetric model: loc, logscale [5][K], eps [S][5][K]."""
    lib = load()
    eps = np.ascontiguousarray(eps, dtype=np.float64)
    S, K = eps.shape[0], prob.K
    cut = prob.cutoff if c is None else c
    gl = np.empty((5, K)); gs = np.empty((5, K)); ll = np.empty(S)
    out = C.c_double(0.0)
    keep = [_d(prob.x), _d(y), _d(prob.bg), _i(prob.peak_off),
            _d(prob.peak_pos), _d(prob.peak_int), _d(loc), _d(logscale),
            _d(eps)]
    rc = lib.oracle_elbo_asym(prob.N, K, keep[0][1], keep[1][1], keep[2][1],
                              keep[3][1], keep[4][1], keep[5][1], float(cut),
                              float(lam), float(mu_sd), float(w_shape),
                              float(w_rate), float(alpha_mean),
                              float(alpha_sd), S, keep[6][1], keep[7][1],
                              keep[8][1], C.byref(out), ll.ctypes.data_as(_D),
                              gl.ctypes.data_as(_D) if grad else None,
                              gs.ctypes.data_as(_D) if grad else None)
    if rc != 0:
        raise ValueError(f"oracle_elbo_asym failed: {rc}")
    return out.value, ll, (gl if grad else None), (gs if grad else None)


def readout(peak_off, peak_int, m_h, logscale_h, threshold=0.01):
    """(mean_h, sd_h, area_ratio, selected indices) of the h latent."""
    lib = load()
    K = len(peak_off) - 1
    keep = [_i(peak_off), _d(peak_int if len(peak_int) else [0.0]), _d(m_h),
            _d(logscale_h)]
    mean, sd, ratio = np.empty(K), np.empty(K), np.empty(K)
    sel = np.empty(K, dtype=np.int32)
    rc = lib.oracle_readout(K, keep[0][1], keep[1][1], keep[2][1], keep[3][1],
                            float(threshold), mean.ctypes.data_as(_D),
                            sd.ctypes.data_as(_D), ratio.ctypes.data_as(_D),
                            sel.ctypes.data_as(_I))
    if rc != 0:
        raise ValueError("oracle_readout: total area not positive")
    return mean, sd, ratio, np.nonzero(sel)[0]


def num_threads():
    return load().oracle_num_threads()


def set_threads(n):
    """OpenMP threads of later oracle calls."""
    load().oracle_set_threads(int(n))


def profile_sec(x, B, peak_off, p, I, c, phi):
    """f[S][N] with the sec width law; phi[S][D][K], D = 4 or 5."""
    lib = load()
    phi = np.asarray(phi, dtype=np.float64)
    if phi.ndim == 2:
        phi = phi[None]
    S, D, K = phi.shape
    f = np.empty((S, len(x)))
    keep = [_d(x), _d(B), _i(peak_off), _d(p), _d(I), _d(phi)]
    rc = lib.oracle_profile_sec(len(x), K, keep[0][1], keep[1][1], keep[2][1],
                                keep[3][1], keep[4][1], float(c), D, S,
                                keep[5][1], f.ctypes.data_as(_D))
    assert rc == 0, rc
    return f


def windows_sec(x, peak_off, p, c, phi):
    """Window plan (lo, hi) [S][T] with the sec width law."""
    lib = load()
    phi = np.asarray(phi, dtype=np.float64)
    if phi.ndim == 2:
        phi = phi[None]
    S, D, K = phi.shape
    T = int(peak_off[-1])
    lo = np.empty((S, T), dtype=np.int32)
    hi = np.empty((S, T), dtype=np.int32)
    keep = [_d(x), _i(peak_off), _d(p), _d(phi)]
    rc = lib.oracle_windows_sec(len(x), K, keep[0][1], keep[1][1], keep[2][1],
                                float(c), D, S, keep[3][1],
                                lo.ctypes.data_as(_I), hi.ctypes.data_as(_I))
    assert rc == 0, rc
    return lo, hi


def elbo_sec(prob, y, loc, logscale, eps, *, lam=0.0, mu_sd=0.03,
             w_shape=3.0, w_rate=100.0, alpha_mean=1.0, alpha_sd=0.2,
             grad=True, c=None):
    """Sec width law: loc, logscale [D][K], eps [S][D][K], D = 4 or 5."""
    lib = load()
    eps = np.ascontiguousarray(eps, dtype=np.float64)
    S, D, K = eps.shape
    assert K == prob.K
    cut = prob.cutoff if c is None else c
    gl = np.empty((D, K)); gs = np.empty((D, K)); ll = np.empty(S)
    out = C.c_double(0.0)
    keep = [_d(prob.x), _d(y), _d(prob.bg), _i(prob.peak_off),
            _d(prob.peak_pos), _d(prob.peak_int), _d(loc), _d(logscale),
            _d(eps)]
    rc = lib.oracle_elbo_sec(prob.N, K, keep[0][1], keep[1][1], keep[2][1],
                             keep[3][1], keep[4][1], keep[5][1], float(cut),
                             float(lam), float(mu_sd), float(w_shape),
                             float(w_rate), float(alpha_mean),
                             float(alpha_sd), D, S, keep[6][1], keep[7][1],
                             keep[8][1], C.byref(out), ll.ctypes.data_as(_D),
                             gl.ctypes.data_as(_D) if grad else None,
                             gs.ctypes.data_as(_D) if grad else None)
    if rc != 0:
        raise ValueError(f"oracle_elbo_sec failed: {rc}")
    return out.value, ll, (gl if grad else None), (gs if grad else None)
