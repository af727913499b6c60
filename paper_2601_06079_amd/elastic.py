"""Eshelby inclusion (linear elasticity with an eigenstrain, Eqs. 3-4 and
Supplementary Note 3 Eq. III.1) on the GPU: ctypes binding of pf_el_*.

Argument marshalling only: the operator, the load, the conjugate-gradient
solve, the objective and the adjoint sensitivities all run in the library's
HIP kernels.  Displacements are device tensors of dim * N values,
component-major ([u_x ; u_y ; (u_z)], node index i + n0 (j + n1 k)).
"""
from __future__ import annotations

import ctypes as ct
from dataclasses import dataclass

import torch

from . import _abi as A


class pf_elastic(ct.Structure):
    _fields_ = [("dim", ct.c_int32), ("dtype", ct.c_int32), ("n", ct.c_int64 * 3),
                ("h", ct.c_double), ("E", ct.c_double), ("nu", ct.c_double),
                ("m", ct.c_double), ("a", ct.c_double), ("l", ct.c_double)]


class pf_el_report(ct.Structure):
    _fields_ = [("iterations", ct.c_int32), ("converged", ct.c_int32), ("status", ct.c_int32),
                ("levels", ct.c_int32), ("res_norm", ct.c_double), ("rhs_norm", ct.c_double)]


TUNE_EL_PLANES = 4
TUNE_EL_MG = 5  # 1: plain CG; 2: every multigrid level launched; v >= 3: one-block coarse grids up to v nodes
_L = None


def _lib():
    global _L
    if _L is None:
        L = A.lib()
        P = ct.POINTER(pf_elastic)
        R = ct.POINTER(pf_el_report)
        vp, i32, f64 = ct.c_void_p, ct.c_int32, ct.c_double
        for name, res, args in (("pf_el_workspace_size", i32, [vp, P, ct.POINTER(ct.c_size_t)]),
                                ("pf_el_apply", i32, [vp, P, vp, vp, vp]),
                                ("pf_el_rhs", i32, [vp, P, vp, vp]),
                                ("pf_el_solve", i32, [vp, P, vp, vp, f64, i32, R, vp, vp]),
                                ("pf_el_objective", i32, [vp, P, vp, vp, vp, vp, vp]),
                                ("pf_el_sensitivity", i32, [vp, P, vp, vp, ct.POINTER(ct.c_double), f64,
                                                            i32, R, vp, vp])):
            fn = getattr(L, name)
            fn.restype, fn.argtypes = res, args
        _L = L
    return _L


@dataclass
class ElasticProblem:
    """Grid, elastic constants and eigenstrain (see pf_elastic in include/pf.h).
    Defaults: the paper's E = 22.5 and nu = 0.3 on [0, 100]^dim; the misfit
    profile (m, a, l) is this library's choice (the paper does not print it)."""
    n: tuple
    h: float = 1.0
    E: float = 22.5
    nu: float = 0.3
    m: float = 0.01
    a: float = 20.0
    l: float = 0.5
    dtype: torch.dtype = torch.float32

    @property
    def dim(self):
        return len(self.n)

    @property
    def nnodes(self):
        N = 1
        for v in self.n:
            N *= int(v)
        return N

    @property
    def ndof(self):
        return self.dim * self.nnodes

    def c(self) -> pf_elastic:
        n3 = [int(v) for v in self.n] + [1] * (3 - len(self.n))
        return pf_elastic(self.dim, A.F64 if self.dtype == torch.float64 else A.F32,
                          (ct.c_int64 * 3)(*n3), float(self.h), float(self.E), float(self.nu),
                          float(self.m), float(self.a), float(self.l))


def _stream():
    return ct.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, p: ElasticProblem, name):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous device tensor")
    if t.dtype != p.dtype or t.numel() != p.ndof:
        raise ValueError(f"{name}: expected {p.ndof} values of {p.dtype}")
    return ct.c_void_p(t.data_ptr())


def workspace(p: ElasticProblem, device=None) -> torch.Tensor:
    nb = ct.c_size_t(0)
    A.check(_lib().pf_el_workspace_size(A.ctx(), ct.byref(p.c()), ct.byref(nb)))
    return torch.empty(int(nb.value) + 256, dtype=torch.uint8, device=device or torch.device("cuda"))


def _ws_ptr(ws: torch.Tensor):
    base = ws.data_ptr()
    return ct.c_void_p((base + 255) // 256 * 256)


def el_apply(p: ElasticProblem, u: torch.Tensor, out: torch.Tensor = None) -> torch.Tensor:
    y = torch.empty_like(u) if out is None else out
    A.check(_lib().pf_el_apply(A.ctx(), ct.byref(p.c()), _ptr(u, p, "u"), _ptr(y, p, "y"), _stream()))
    return y


def el_rhs(p: ElasticProblem, out: torch.Tensor = None, device=None) -> torch.Tensor:
    f = torch.empty(p.ndof, dtype=p.dtype, device=device or torch.device("cuda")) if out is None else out
    A.check(_lib().pf_el_rhs(A.ctx(), ct.byref(p.c()), _ptr(f, p, "f"), _stream()))
    return f


def el_solve(p: ElasticProblem, b: torch.Tensor = None, out: torch.Tensor = None, rtol=1e-6,
             maxit=20000, ws: torch.Tensor = None, allow_noconv=False):
    """Returns (u, report); b = None solves for the eigenstrain load."""
    dev = torch.device("cuda")
    u = torch.empty(p.ndof, dtype=p.dtype, device=dev) if out is None else out
    ws = workspace(p, dev) if ws is None else ws
    rep = pf_el_report()
    st = _lib().pf_el_solve(A.ctx(), ct.byref(p.c()), _ptr(b, p, "b"), _ptr(u, p, "u"), float(rtol), int(maxit),
                            ct.byref(rep), _ws_ptr(ws), _stream())
    A.check(st, allow=(A.PF_ENOCONV,) if allow_noconv else ())
    return u, rep


def el_objective(p: ElasticProblem, u: torch.Tensor, g: torch.Tensor = None,
                 ws: torch.Tensor = None) -> torch.Tensor:
    """Device float64 scalar g . u (g = None: the volume change)."""
    ws = workspace(p, u.device) if ws is None else ws
    out = torch.empty(1, dtype=torch.float64, device=u.device)
    A.check(_lib().pf_el_objective(A.ctx(), ct.byref(p.c()), _ptr(g, p, "g"), _ptr(u, p, "u"),
                                   ct.c_void_p(out.data_ptr()), _ws_ptr(ws), _stream()))
    return out


def el_sensitivity(p: ElasticProblem, u: torch.Tensor, g: torch.Tensor = None, rtol=1e-6,
                   maxit=20000, ws: torch.Tensor = None):
    """(O, dO/dE, dO/dnu) at the equilibrium u, and the adjoint solve's report."""
    ws = workspace(p, u.device) if ws is None else ws
    out = (ct.c_double * 3)()
    rep = pf_el_report()
    A.check(_lib().pf_el_sensitivity(A.ctx(), ct.byref(p.c()), _ptr(g, p, "g"), _ptr(u, p, "u"), out,
                                     float(rtol), int(maxit), ct.byref(rep), _ws_ptr(ws), _stream()))
    return (out[0], out[1], out[2]), rep
