"""Torch-facing wrappers of the C ABI: same names as include/pf.h, no arithmetic.

Tensors must be contiguous CUDA (HIP) tensors of the problem's dtype.  Every
call is enqueued on torch's current stream.
"""
from __future__ import annotations

import ctypes as ct
from dataclasses import dataclass, field, replace

import torch

from . import _abi as A


@dataclass
class Problem:
    """Problem statement (see pf_problem in include/pf.h)."""
    n: tuple
    model: int = A.ALLEN_CAHN
    fe: int = A.F_SYM
    dtype: torch.dtype = torch.float32
    h: float = 1.0
    W: float = 1.0
    kappa: float = 1.0
    mobility: float = 1.0
    bc: int = A.PERIODIC
    mobility_eta: float = 0.0  # coupled model: M_eta
    mass: int = A.MASS_LUMPED  # MASS_CONSISTENT: Gauss-integrated mass (implicit path)
    nfields: int = 1  # GRAIN: order parameters
    gamma: float = 1.5  # GRAIN: pair coupling
    quad: int = A.QUAD_GAUSS  # QUAD_LOBATTO: nodal quadrature

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
        if self.model == A.GRAIN:
            return int(self.nfields) * self.nnodes
        return {A.CAHN_HILLIARD: 2, A.COUPLED: 3}.get(self.model, 1) * self.nnodes

    def c(self) -> A.pf_problem:
        n3 = [int(v) for v in self.n] + [1] * (3 - len(self.n))
        return A.pf_problem(self.dim, self.bc, self.model, self.fe,
                            A.F64 if self.dtype == torch.float64 else A.F32, int(self.mass),
                            (ct.c_int64 * 3)(*n3), float(self.h), float(self.W),
                            float(self.kappa), float(self.mobility), float(self.mobility_eta),
                            int(self.nfields), int(self.quad), float(self.gamma))


def _stream():
    return ct.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor, p: Problem = None, n: int = None, name="tensor"):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if p is not None and t.dtype != p.dtype:
        raise ValueError(f"{name} has dtype {t.dtype}, problem says {p.dtype}")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
    return ct.c_void_p(t.data_ptr())


def workspace(p: Problem, op: int, device=None) -> torch.Tensor:
    nb = ct.c_size_t(0)
    A.check(A.lib().pf_workspace_size(A.ctx(device), ct.byref(p.c()), op, ct.byref(nb)))
    return torch.empty(max(int(nb.value), 8), dtype=torch.uint8,
                       device=device or torch.device("cuda"))


def residual(p: Problem, U: torch.Tensor, out: torch.Tensor = None) -> torch.Tensor:
    r = torch.empty_like(U) if out is None else out
    A.check(A.lib().pf_residual(A.ctx(), ct.byref(p.c()), _ptr(U, p, p.ndof, "U"),
                                _ptr(r, p, p.ndof, "r"), None, _stream()))
    return r


def step_explicit(p: Problem, U: torch.Tensor, dt: float, nsteps: int,
                  ws: torch.Tensor = None) -> torch.Tensor:
    """nsteps explicit steps in place on U; returns U."""
    if ws is None:
        ws = workspace(p, A.OP_STEP_EXPLICIT, U.device)
    A.check(A.lib().pf_step_explicit(A.ctx(), ct.byref(p.c()), float(dt), int(nsteps),
                                     _ptr(U, p, p.ndof, "U"), ct.c_void_p(ws.data_ptr()),
                                     _stream()))
    return U


def energy(p: Problem, U: torch.Tensor, ws: torch.Tensor = None,
           out: torch.Tensor = None) -> torch.Tensor:
    """Device tensor [E_h, sum m c] (float64)."""
    if ws is None:
        ws = workspace(p, A.OP_ENERGY, U.device)
    if out is None:
        out = torch.empty(2, dtype=torch.float64, device=U.device)
    A.check(A.lib().pf_energy(A.ctx(), ct.byref(p.c()), _ptr(U, p, p.ndof, "U"),
                              ct.c_void_p(out.data_ptr()), ct.c_void_p(ws.data_ptr()), _stream()))
    return out


def jvp(p: Problem, inv_dt: float, U: torch.Tensor, v: torch.Tensor,
        out: torch.Tensor = None) -> torch.Tensor:
    Jv = torch.empty_like(U) if out is None else out
    A.check(A.lib().pf_jvp(A.ctx(), ct.byref(p.c()), float(inv_dt), _ptr(U, p, p.ndof, "U"),
                           _ptr(v, p, p.ndof, "v"), _ptr(Jv, p, p.ndof, "Jv"), _stream()))
    return Jv


def newton_opts(**kw) -> A.pf_newton_opts:
    o = A.pf_newton_opts()
    A.lib().pf_newton_default_opts(ct.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


@dataclass
class NewtonReport:
    newton_its: int
    gmres_its: int
    converged: bool
    reason: int
    res_norm: list = field(default_factory=list)


def newton_step(p: Problem, dt: float, U_old: torch.Tensor, U: torch.Tensor, opts=None,
                ws: torch.Tensor = None, raise_on_noconv: bool = False) -> NewtonReport:
    """One backward-Euler step in place on U (initial guess on entry)."""
    if ws is None:
        ws = workspace(p, A.OP_NEWTON, U.device)
    o = opts if opts is not None else newton_opts()
    rep = A.pf_newton_report()
    st = A.lib().pf_newton_step(A.ctx(), ct.byref(p.c()), float(dt), _ptr(U_old, p, p.ndof, "U_old"),
                                _ptr(U, p, p.ndof, "U"), ct.byref(o), ct.byref(rep),
                                ct.c_void_p(ws.data_ptr()), _stream())
    allow = () if raise_on_noconv else (A.PF_ENOCONV, A.PF_ENONFINITE)
    A.check(st, allow=allow)
    k = rep.newton_its
    return NewtonReport(k, rep.gmres_its, bool(rep.converged), rep.reason,
                        [rep.res_norm[i] for i in range(min(k, 32) + 1)])


def vjp(p: Problem, kind: int, dt: float, U: torch.Tensor, vbar: torch.Tensor,
        Ubar: torch.Tensor, theta_bar: torch.Tensor, ws: torch.Tensor = None,
        U_old: torch.Tensor = None):
    """Accumulate vector-Jacobian products into Ubar and theta_bar (float64[3], on the
    device or, making the call host-synchronous, on the host).  U_old (VJP_RESIDUAL
    only) selects the backward-Euler residual M (U - U_old)/dt + r(U)."""
    if ws is None:
        ws = workspace(p, A.OP_VJP, U.device)
    if theta_bar.dtype != torch.float64 or theta_bar.numel() != 3 or not theta_bar.is_contiguous():
        raise ValueError("theta_bar must be a contiguous float64 tensor of 3 entries")
    flags = 0 if theta_bar.is_cuda else A.VJP_THETA_HOST
    uold = None if U_old is None else _ptr(U_old, p, p.ndof, "U_old")
    A.check(A.lib().pf_vjp(A.ctx(), ct.byref(p.c()), int(kind), float(dt), _ptr(U, p, p.ndof, "U"),
                           uold, _ptr(vbar, p, None, "vbar"), _ptr(Ubar, p, None, "Ubar"),
                           ct.c_void_p(theta_bar.data_ptr()), flags, ct.c_void_p(ws.data_ptr()),
                           _stream()))


def launch_shape(p: Problem):
    """(steps fused per launch, rows per wave, prefetch depth) that step_explicit
    uses for the 2-D problem p."""
    ks, ty, dp = ct.c_int(0), ct.c_int(0), ct.c_int(0)
    A.check(A.lib().pf_launch_shape(A.ctx(), ct.byref(p.c()), ct.byref(ks), ct.byref(ty), ct.byref(dp)))
    return int(ks.value), int(ty.value), int(dp.value)


def tune_set(key: int, value: int):
    A.check(A.lib().pf_tune_set(int(key), int(value)))


def tune_get(key: int) -> int:
    v = ct.c_int(0)
    A.check(A.lib().pf_tune_get(int(key), ct.byref(v)))
    return int(v.value)


# ---------------------------------------------------------------------------
class CheckpointedRun(torch.autograd.Function):
    """U_N = S^N(U_0; theta) for one problem, explicit (Eq. 12) or backward-Euler
    Newton steps (Eqs. 13-14), with a hand-written adjoint (Supp. Note 2,
    Eqs. II.5-II.6).

    theta = (mobility, kappa, W) as a float64 tensor of 3.  Forward keeps a
    snapshot every `every` steps; backward walks the segments in reverse,
    recomputes each segment's states from its snapshot (bitwise the forward's:
    every kernel is deterministic, and both passes advance with the same launches:
    fused launches are bitwise single steps on periodic grids, and no-flux grids,
    where a fused stage rounds the reflected rows differently, take single-step
    launches in the forward pass too) and applies the step adjoint of the library
    (pf_vjp: explicit-step VJP, or the transposed Newton solve at each root),
    accumulating the gradient of theta in FP64.  For Cahn-Hilliard explicit
    runs only the c plane of U_N is differentiated (mu is recomputed from c).
    """

    @staticmethod
    def forward(ctx, theta, U0, p, dt, nsteps, every, implicit, opts):
        if nsteps % every:
            raise ValueError("nsteps must be a multiple of the checkpoint interval")
        th = theta.detach().to("cpu", torch.float64).numpy()
        q = replace(p, mobility=float(th[0]), kappa=float(th[1]), W=float(th[2]))
        U = U0.detach().clone()
        ws = workspace(q, A.OP_NEWTON if implicit else A.OP_STEP_EXPLICIT, U.device)
        snaps = []
        single = q.bc == A.NOFLUX  # match the single-step recomputation bitwise
        for _ in range(nsteps // every):
            snaps.append(U.clone())
            if single:
                for _ in range(every):
                    _advance(q, U, dt, 1, implicit, opts, ws)
            else:
                _advance(q, U, dt, every, implicit, opts, ws)
        ctx.q, ctx.dt, ctx.every, ctx.implicit, ctx.opts = q, dt, every, implicit, opts
        ctx.snaps, ctx.theta_device = snaps, theta.device
        return U

    @staticmethod
    def backward(ctx, gU):
        q, dt, every, implicit = ctx.q, ctx.dt, ctx.every, ctx.implicit
        lam = gU.detach().to(q.dtype).contiguous().clone()
        N = q.nnodes
        if q.model == A.CAHN_HILLIARD and not implicit:
            lam[N:] = 0
        tb = torch.zeros(3, dtype=torch.float64, device=lam.device)
        ws = workspace(q, A.OP_NEWTON if implicit else A.OP_STEP_EXPLICIT, lam.device)
        vws = workspace(q, A.OP_VJP, lam.device)
        seg = torch.empty((every + 1, lam.numel()), dtype=q.dtype, device=lam.device)
        Ubar = torch.empty_like(lam)
        kind = A.VJP_NEWTON_STEP if implicit else A.VJP_EXPLICIT_STEP
        for snap in reversed(ctx.snaps):
            seg[0].copy_(snap)
            for k in range(every):  # seg[k + 1] = S(seg[k])
                seg[k + 1].copy_(seg[k])
                _advance(q, seg[k + 1], dt, 1, implicit, ctx.opts, ws)
            for k in reversed(range(every)):
                # explicit: VJP of the step taken from seg[k]; implicit: at its root seg[k + 1]
                Ubar.zero_()
                vjp(q, kind, dt, seg[k + 1] if implicit else seg[k], lam, Ubar, tb, vws)
                lam, Ubar = Ubar, lam
        return tb.to(ctx.theta_device), lam, None, None, None, None, None, None


def _advance(q, U, dt, nsteps, implicit, opts, ws):
    if not implicit:
        step_explicit(q, U, dt, nsteps, ws)
        return
    Uold = torch.empty_like(U)
    for _ in range(nsteps):
        Uold.copy_(U)
        newton_step(q, dt, Uold, U, opts, ws, raise_on_noconv=True)


def checkpointed_run(theta, U0, p, dt, nsteps, every=100, implicit=False, opts=None):
    """Differentiable run of nsteps steps of problem p (see CheckpointedRun)."""
    return CheckpointedRun.apply(theta, U0, p, dt, nsteps, every, implicit, opts)
