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
