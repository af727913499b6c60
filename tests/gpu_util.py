"""Shared helpers for the GPU parity tests (HIP library vs FP64 oracle)."""
import numpy as np
import torch

import oracle as O
from paper_2601_06079_amd import _abi as A
from paper_2601_06079_amd import solver as S

DEV = "cuda"


def pair(n, model, fe, dtype, h=1.0, W=1.0, kappa=1.0, mob=1.0, bc=O.PERIODIC):
    """The same problem for the GPU library and for the oracle."""
    g = S.Problem(n=tuple(n), model=model, fe=fe, dtype=dtype, h=h, W=W, kappa=kappa, mobility=mob,
                  bc=A.NOFLUX if bc == O.NOFLUX else A.PERIODIC)
    o = O.Problem(n=tuple(n), model=model, fe=fe, h=h, W=W, kappa=kappa, mob=mob, bc=bc)
    return g, o


def dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def host(t):
    return t.detach().to("cpu", torch.float64).numpy()


def rounded(a, dtype):
    """The values the GPU actually holds, promoted to float64 for the oracle."""
    np_dt = np.float32 if dtype == torch.float32 else np.float64
    return np.asarray(a).astype(np_dt).astype(np.float64)


def rel_l2(a, b):
    a = np.ravel(a)
    b = np.ravel(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def announce(*args):
    print("[gpu-case]", *args, flush=True)
