"""Brute-force selection: the exact MAP support over all 2^K phase subsets
at fixed profile parameters (test helper, CPU only)."""
import numpy as np
from scipy import special


def map_support(C, y, B, lam):
    """Exact MAP of h >= 0 for f = B + C^T h, objective
    sum(y ln f - f) - lam sum h (concave), by enumerating supports and
    solving each with damped Newton (step halving keeps f > 0 and the
    objective increasing)."""
    K = C.shape[0]

    def objective(CT, hT):
        f = B + CT.T @ hT
        if np.any(f <= 0):
            return -np.inf
        return np.sum(special.xlogy(y, f) - f) - lam * hT.sum()

    best = (-np.inf, None, None)
    for mask in range(1 << K):
        T = [k for k in range(K) if mask >> k & 1]
        h = np.zeros(K)
        if T:
            CT = C[T]
            hT = np.full(len(T), 100.0)
            cur = objective(CT, hT)
            for _ in range(500):
                f = B + CT.T @ hT
                g = CT @ (y / f - 1) - lam
                H = -(CT * (y / f ** 2)) @ CT.T
                step = np.linalg.solve(H, -g)
                t = 1.0
                while t > 1e-12:
                    new = objective(CT, hT + t * step)
                    if new >= cur:
                        break
                    t *= 0.5
                hT = hT + t * step
                cur = objective(CT, hT)
                if np.max(np.abs(t * step)) < 1e-11 * max(1.0, np.max(np.abs(hT))):
                    break
            if np.any(hT <= 0):
                continue
            h[T] = hT
        f = B + C.T @ h
        obj = np.sum(special.xlogy(y, f) - f) - lam * h.sum()
        if obj > best[0]:
            best = (obj, h, T)
    return best


def phase_basis(orc, prob, phi):
    """Unit-weight profile of every phase (rows), background excluded, at
    the profile parameters of phi [4][K]."""
    K = prob.K
    basis_phi = np.zeros((K, 4, K))
    for k in range(K):
        basis_phi[k] = phi
        basis_phi[k, 0] = 0.0
        basis_phi[k, 0, k] = 1.0
    return orc.profile(prob.x, np.zeros(prob.N), prob.peak_off, prob.peak_pos,
                       prob.peak_int, 0.0, basis_phi)


def area_ratios(prob, h):
    """Area ratio of each phase for weights h (unit-area peaks)."""
    isum = np.add.reduceat(prob.peak_int, prob.peak_off[:-1])
    isum[np.diff(prob.peak_off) == 0] = 0.0
    a = np.asarray(h) * isum
    return a / a.sum()
