"""Hamiltonian Monte Carlo in FP64 (TEST INFRASTRUCTURE ONLY, like the rest
of this package).

Leapfrog integration and the Metropolis correction (Neal, "MCMC using
Hamiltonian dynamics", 2011), step sizes adapted during warm-up by dual
averaging (Hoffman and Gelman, JMLR 2014, their Algorithm 5 with
mu = ln(10 eps0), gamma = 0.05, t0 = 10, kappa = 0.75), one chain at a time
in plain Python.  Momenta and Metropolis uniforms come from the oracle's
own Philox4x32-10: momenta of iteration i are the standard normals of
eps_philox keyed by (seed, i), the uniform of chain c is word 0 of the
block with counter (0, c, i) and key seed ^ 0x9E3779B97F4A7C15.
"""
from __future__ import annotations

import math

import numpy as np

from . import oracle as O

UNIFORM_KEY = 0x9E3779B97F4A7C15
LN_2PI = math.log(2.0 * math.pi)


def logpost(prob, y, z, lam=0.0, asymmetric=False, width_law=0, **prior):
    """ln p(Y|phi(z)) + ln p(phi(z)) + ln|J(z)| and its gradient in z, for
    one position z [D][K]: the ELBO estimate at zero noise and unit scale
    (mean z) minus its entropy term D K (1 + ln 2 pi) / 2.  width_law
    "sec" (or 1): the angle-dependent width (D taken from z)."""
    z = np.asarray(z, dtype=np.float64)
    zeros = np.zeros_like(z)
    eps = np.zeros((1,) + z.shape)
    if width_law in (1, "sec"):
        fn = O.elbo_sec
    else:
        fn = O.elbo_asym if asymmetric else O.elbo
    e, _, g, _ = fn(prob, y, z, zeros, eps, lam=lam, **prior)
    return e - 0.5 * z.size * (1.0 + LN_2PI), g


def uniform(seed, chain, it):
    key = (int(seed) ^ UNIFORM_KEY) & 0xFFFFFFFFFFFFFFFF
    v = O.philox4x32_10([0, chain, it & 0xFFFFFFFF, it >> 32],
                        [key & 0xFFFFFFFF, key >> 32])
    return (v[0] + 0.5) / 4294967296.0


def momenta(C, n, seed, it):
    """Standard normals [C][n] of iteration it (coordinate j of chain c is
    number j of sample c)."""
    return O.eps_philox(C, n, seed, it, D=1).reshape(C, n)


def leapfrog(fn, z, p, g, eps, L):
    """L leapfrog steps from (z, p) with gradient g at z; fn(z) -> (logp,
    grad).  Returns (z, p, logp, grad) at the end."""
    p = p + 0.5 * eps * g
    z = z + eps * p
    for l in range(1, L + 1):
        lp, g = fn(z)
        if l < L:
            p = p + eps * g
            z = z + eps * p
    p = p + 0.5 * eps * g
    return z, p, lp, g


def run(fn, z0, seed, n_warmup, n_draws, n_leapfrog, step_size,
        target_accept=0.8):
    """Chains from positions z0 [C][n]; fn(z [n]) -> (logp, grad [n]).
    Returns dict(z, draws [n_draws][C][n], logp [n_draws][C], accept [C],
    step [C], decisions [iterations][C] of (accepted, ln u - (H0 - H1)))."""
    z = np.array(z0, dtype=np.float64)
    C, n = z.shape
    lp = np.empty(C)
    g = np.empty((C, n))
    for c in range(C):
        lp[c], gc = fn(z[c])
        g[c] = np.asarray(gc).reshape(n)
    eps = np.full(C, float(step_size))
    leps_bar = np.zeros(C)
    hbar = np.zeros(C)
    mu = math.log(10.0 * step_size)
    gamma, t0, kappa, delta = 0.05, 10.0, 0.75, target_accept
    draws, logps, decisions = [], [], []
    accepted = np.zeros(C)
    for it in range(n_warmup + n_draws):
        p0 = momenta(C, n, seed, it)
        dec = []
        for c in range(C):
            h0 = -lp[c] + 0.5 * float(p0[c] @ p0[c])

            def f(x):
                v, gr = fn(x)
                return v, np.asarray(gr).reshape(n)

            z1, p1, lp1, g1 = leapfrog(f, z[c], p0[c], g[c], eps[c], n_leapfrog)
            h1 = -lp1 + 0.5 * float(p1 @ p1)
            dh = h0 - h1
            finite = math.isfinite(h1) and math.isfinite(dh)
            alpha = (1.0 if dh >= 0.0 else math.exp(dh)) if finite else 0.0
            lu = math.log(uniform(seed, c, it))
            acc = finite and lu < dh
            dec.append((acc, lu - dh if finite else math.inf))
            if acc:
                z[c], g[c], lp[c] = z1, g1, lp1
            if it < n_warmup:
                m = it + 1.0
                w = 1.0 / (m + t0)
                hbar[c] = (1.0 - w) * hbar[c] + w * (delta - alpha)
                leps = mu - math.sqrt(m) / gamma * hbar[c]
                eta = m ** -kappa
                leps_bar[c] = eta * leps + (1.0 - eta) * leps_bar[c]
                eps[c] = math.exp(leps)
            else:
                accepted[c] += acc
        decisions.append(dec)
        if it >= n_warmup:
            draws.append(z.copy())
            logps.append(lp.copy())
        if it + 1 == n_warmup:
            eps = np.exp(leps_bar)
    return dict(z=z, draws=np.array(draws), logp=np.array(logps),
                accept=accepted / max(n_draws, 1), step=eps,
                decisions=decisions)
