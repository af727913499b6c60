"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle runs.

This module holds no arithmetic of the phase-field method: it only draws
initial fields and parameters.  Draws follow one fixed convention so that
every consumer sees the same numbers: ``numpy.random.default_rng(seed)``
(PCG64), ``uniform(a, b, N)`` in node order (x fastest), generated in FP64;
FP32 runs cast to float32 and feed the CPU reference the same float32-rounded
values promoted back to FP64.
"""
from __future__ import annotations

import numpy as np


def uniform_field(n, lo, hi, seed=0, dtype=np.float64, base=0.0):
    """base + U(lo, hi) per node, node order x fastest."""
    N = int(np.prod(n))
    rng = np.random.default_rng(seed)
    a = base + rng.uniform(lo, hi, N)
    return a.astype(dtype)


# --- the paper-shaped workloads --------------------------------------------
# Allen-Cahn, 128x128 periodic, f = (c^2-1)^2/4, kappa = 1, L = 1, h = 1,
# c0 ~ U(-0.05, 0.05), forward Euler dt = 0.1, 1000 steps, FP64.
AC128 = dict(n=(128, 128), model=0, fe=0, W=1.0, kappa=1.0, mob=1.0, h=1.0, dt=0.1,
             steps=1000, lo=-0.05, hi=0.05, base=0.0)

# Cahn-Hilliard spinodal decomposition, 2048x2048 periodic (4 194 304 nodes),
# f = W c^2 (1-c)^2, W = 1, kappa = 2, M = 1, h = 1, c0 = 0.5 + U(-0.01, 0.01),
# explicit split step dt = 0.01, FP32 fields.
CH2048 = dict(n=(2048, 2048), model=1, fe=1, W=1.0, kappa=2.0, mob=1.0, h=1.0, dt=0.01,
              steps=10000, lo=-0.01, hi=0.01, base=0.5)

# Cahn-Hilliard 3-D, 128^3 periodic, two unknown fields (c, mu) = 4 194 304 DOF,
# c0 = 0.4 + U(-0.02, 0.02), backward Euler dt = 0.5, Newton rtol 1e-8,
# GMRES(30) with block-Jacobi, 200 steps.
CH3D128 = dict(n=(128, 128, 128), model=1, fe=1, W=1.0, kappa=2.0, mob=1.0, h=1.0, dt=0.5,
               steps=200, lo=-0.02, hi=0.02, base=0.4)


def initial_state(cfg, seed=0, dtype=np.float64, n=None):
    """Initial c (Allen-Cahn: eta) for a workload dict; Cahn-Hilliard states get
    a zero mu plane appended (callers fill mu as their scheme requires)."""
    n = tuple(n or cfg["n"])
    c = uniform_field(n, cfg["lo"], cfg["hi"], seed=seed, base=cfg["base"]).astype(dtype)
    if cfg["model"] == 1:
        return np.concatenate([c, np.zeros_like(c)])
    return c


def batch_samples(count=64, nmin=128, nmax=512, seed=0):
    """Ragged calibration batch: square sizes n_s ~ U{nmin..nmax}, then per-sample
    theta = (L, kappa, W) ~ logU(0.5, 2), then hidden theta* ~ logU(0.5, 2), then
    initial fields c0 ~ U(-0.05, 0.05), all from one generator in that order."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(nmin, nmax + 1, size=count)
    theta = np.exp(rng.uniform(np.log(0.5), np.log(2.0), size=(count, 3)))
    hidden = np.exp(rng.uniform(np.log(0.5), np.log(2.0), size=(count, 3)))
    fields = [rng.uniform(-0.05, 0.05, int(s) * int(s)) for s in sizes]
    return sizes, theta, hidden, fields


# Coupled Allen-Cahn / Cahn-Hilliard benchmark shape: the square [0, 100]^2 with
# n nodes per axis (h = 100 / (n - 1)), no-flux boundaries, M_c = 1, M_eta = 150,
# kappa_eta = 0.3.  Initial state: discs of the second phase (eta ~ 1) with a
# diffuse edge of width 2, in a matrix (eta ~ 0); c = 0.04 + 0.12 eta plus
# N(0, 0.005^2) noise; mu plane zero.  (The paper's own initial condition is a
# figure, not data; this is a stand-in of the same kind.)
COUPLED = dict(L=100.0, Mc=1.0, Meta=150.0, kappa=0.3, discs=((50.0, 50.0, 20.0),
                                                               (20.0, 25.0, 8.0),
                                                               (78.0, 70.0, 12.0)))


def coupled_state(n, seed=0, dtype=np.float64):
    """[c ; mu ; eta] on an n x n grid over [0, L]^2 (see COUPLED)."""
    L = COUPLED["L"]
    h = L / (n - 1)
    X, Y = np.meshgrid(np.arange(n) * h, np.arange(n) * h)
    eta = np.zeros((n, n))
    for (x0, y0, r0) in COUPLED["discs"]:
        eta = np.maximum(eta, 0.5 * (1.0 - np.tanh((np.hypot(X - x0, Y - y0) - r0) / 2.0)))
    rng = np.random.default_rng(seed)
    c = 0.04 + 0.12 * eta + 0.005 * rng.standard_normal((n, n))
    return np.concatenate([c.ravel(), np.zeros(n * n), eta.ravel()]).astype(dtype)


# Grain growth: p order parameters on an n x n grid (grid units, h = 1), grains from
# a seeded Voronoi partition (nearest of `grains` uniform seeds on the periodic
# square), grain g carried by order parameter g mod p; values 1 inside the
# grain's order parameter, 0 elsewhere, plus U(-0.01, 0.01) noise.
GRAIN = dict(p=20, grains=60, kappa=1.0, L=1.0, gamma=1.5, dt=0.1)


def grain_state(n, p, grains=None, seed=0, dtype=np.float64):
    """[eta_1 ; ... ; eta_p] on an n x n grid (see GRAIN)."""
    rng = np.random.default_rng(seed)
    grains = grains or 3 * p
    seeds = rng.uniform(0, n, size=(grains, 2))
    X, Y = np.meshgrid(np.arange(n) + 0.5, np.arange(n) + 0.5)
    best = np.full((n, n), np.inf)
    owner = np.zeros((n, n), dtype=np.int64)
    for g, (sx, sy) in enumerate(seeds):
        dx = np.abs(X - sx)
        dy = np.abs(Y - sy)
        d = np.minimum(dx, n - dx) ** 2 + np.minimum(dy, n - dy) ** 2
        closer = d < best
        best[closer] = d[closer]
        owner[closer] = g
    U = np.zeros((p, n, n))
    for k in range(p):
        U[k][owner % p == k] = 1.0
    U += rng.uniform(-0.01, 0.01, size=U.shape)
    return U.reshape(-1).astype(dtype)
