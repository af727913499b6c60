"""Ragged batches of 2-D problems (one launch for all samples) and the
checkpointed adjoint of a batched explicit trajectory.

Marshalling and bookkeeping only: every step and every adjoint step runs in
the HIP kernels behind pf_step_explicit_batched / pf_vjp_explicit_batched.
"""
from __future__ import annotations

import ctypes as ct

import numpy as np
import torch

from . import _abi as A


def _bind():
    L = A.lib()
    P = ct.POINTER(A.pf_problem)
    S = ct.POINTER(A.pf_batch_sample)
    I = ct.POINTER(A.pf_batch_info)
    vp, i32, i64, f64 = ct.c_void_p, ct.c_int, ct.c_int64, ct.c_double
    sig = {
        "pf_batch_plan_size": (i32, [P, S, i32, i32, i32, ct.POINTER(ct.c_size_t)]),
        "pf_batch_plan": (i32, [vp, P, S, i32, f64, i32, i32, i32, vp, ct.c_size_t, I, vp]),
        "pf_batch_workspace_size": (i32, [I, i32, ct.POINTER(ct.c_size_t)]),
        "pf_step_explicit_batched": (i32, [vp, I, vp, i64, vp, vp, vp, vp]),
        "pf_vjp_explicit_batched": (i32, [vp, I, vp, i64, vp, vp, vp, vp, i32, vp]),
        "pf_batch_autotune": (i32, [vp, P, S, i32, f64, vp, vp, vp, ct.c_size_t, I,
                                    ct.POINTER(ct.c_double), vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    return L


def _stream():
    return ct.c_void_p(torch.cuda.current_stream().cuda_stream)


class Batch:
    """A packed batch of square-or-rectangular periodic 2-D problems.

    sizes: list of (nx, ny); theta: (count, 3) array of (mobility, kappa, W).
    Sample fields are packed back to back, each starting on a 64-element
    boundary.
    """

    def __init__(self, sizes, theta, dt, model=A.ALLEN_CAHN, fe=A.F_SYM, dtype=torch.float32,
                 h=1.0, ks=0, ty=0, depth=0, device="cuda"):
        self.L = _bind()
        self.sizes = [(int(a), int(b)) for a, b in sizes]
        self.count = len(self.sizes)
        self.dtype = dtype
        self.device = torch.device(device)
        self.dt = float(dt)
        self.base = A.pf_problem(2, A.PERIODIC, model, fe, A.F64 if dtype == torch.float64 else A.F32,
                                 0, (ct.c_int64 * 3)(2, 2, 1), h, 1.0, 1.0, 1.0)
        self.offsets = []
        off = 0
        for nx, ny in self.sizes:
            self.offsets.append(off)
            off += (nx * ny + 63) // 64 * 64
        self.total_alloc = off
        self.h = float(h)
        self.set_theta(theta, ks=ks, ty=ty, depth=depth)

    def _samples(self, theta):
        th = np.asarray(theta, dtype=np.float64).reshape(self.count, 3)
        arr = (A.pf_batch_sample * self.count)()
        for i, ((nx, ny), o) in enumerate(zip(self.sizes, self.offsets)):
            arr[i] = A.pf_batch_sample(o, (ct.c_int64 * 3)(nx, ny, 1), self.h, th[i, 2], th[i, 1],
                                       th[i, 0])
        return arr

    def set_theta(self, theta, ks=0, ty=0, depth=0):
        """(Re)build the device plan for parameters theta (count x 3: mobility, kappa, W)."""
        self.theta = np.asarray(theta, dtype=np.float64).reshape(self.count, 3).copy()
        self.samples = self._samples(self.theta)
        nb = ct.c_size_t(0)
        A.check(self.L.pf_batch_plan_size(ct.byref(self.base), self.samples, self.count, 4, 8,
                                          ct.byref(nb)))
        self.plan = torch.empty(int(nb.value), dtype=torch.uint8, device=self.device)
        self.info = A.pf_batch_info()
        A.check(self.L.pf_batch_plan(A.ctx(self.device), ct.byref(self.base), self.samples, self.count, self.dt, ks, ty,
                                     depth, ct.c_void_p(self.plan.data_ptr()), self.plan.numel(),
                                     ct.byref(self.info), _stream()))
        # a single-step plan for trajectory mode and step counts that are not a multiple of ks
        self.info1 = A.pf_batch_info()
        self.plan1 = torch.empty_like(self.plan)
        A.check(self.L.pf_batch_plan(A.ctx(self.device), ct.byref(self.base), self.samples, self.count, self.dt, 1,
                                     self.info.ty, self.info.depth,
                                     ct.c_void_p(self.plan1.data_ptr()), self.plan1.numel(),
                                     ct.byref(self.info1), _stream()))

    @property
    def total(self):
        return int(self.info.total)

    def empty(self):
        return torch.zeros(self.total, dtype=self.dtype, device=self.device)

    def pack(self, fields):
        U = self.empty()
        for (nx, ny), o, f in zip(self.sizes, self.offsets, fields):
            U[o:o + nx * ny] = torch.as_tensor(np.asarray(f).ravel(), dtype=self.dtype)
        return U

    def views(self, U):
        return [U[o:o + nx * ny] for (nx, ny), o in zip(self.sizes, self.offsets)]

    def mse_weights(self):
        """FP64 weights of the packed layout: 1 / (nx ny) on sample s's nodes, 0 on the
        padding between samples (built once)."""
        if getattr(self, "_mse_w", None) is None:
            w = torch.zeros(self.total, dtype=torch.float64, device=self.device)
            for (nx, ny), o in zip(self.sizes, self.offsets):
                w[o:o + nx * ny] = 1.0 / (nx * ny)
            self._mse_w = w
        return self._mse_w

    def side_stream(self):
        """A second stream (default priority) for work that overlaps the caller's."""
        if getattr(self, "_side", None) is None:
            self._side = torch.cuda.Stream(device=self.device)
        return self._side

    def workspace(self, op):
        """Workspace of step or vjp on the fused plan."""
        info = self.info
        nb = ct.c_size_t(0)
        A.check(self.L.pf_batch_workspace_size(ct.byref(info), op, ct.byref(nb)))
        return torch.empty(int(nb.value), dtype=torch.uint8, device=self.device)

    def step(self, U, nsteps, ws=None, traj=None):
        """nsteps explicit steps of every sample in place on U (or into traj)."""
        if ws is None:
            ws = self.workspace(A.OP_STEP_EXPLICIT)
        if traj is not None:  # the fused plan: two states per launch when ks >= 2
            A.check(self.L.pf_step_explicit_batched(A.ctx(self.device), ct.byref(self.info),
                                                    ct.c_void_p(self.plan.data_ptr()), int(nsteps),
                                                    ct.c_void_p(U.data_ptr()), None,
                                                    ct.c_void_p(traj.data_ptr()), _stream()))
            return traj
        ks = int(self.info.ks)
        main = (int(nsteps) // ks) * ks
        if main:
            A.check(self.L.pf_step_explicit_batched(A.ctx(self.device), ct.byref(self.info), ct.c_void_p(self.plan.data_ptr()),
                                                    main, ct.c_void_p(U.data_ptr()),
                                                    ct.c_void_p(ws.data_ptr()), None, _stream()))
        if nsteps - main:
            A.check(self.L.pf_step_explicit_batched(A.ctx(self.device), ct.byref(self.info1),
                                                    ct.c_void_p(self.plan1.data_ptr()), int(nsteps - main),
                                                    ct.c_void_p(U.data_ptr()), ct.c_void_p(ws.data_ptr()),
                                                    None, _stream()))
        return U

    def vjp(self, states, lam, theta_bar, nsteps, ws=None, begin=True, end=True):
        """Adjoint of nsteps steps whose inputs are states[k]; lam in/out, theta_bar +=
        (begin: zero the FP64 partials in ws first; end: reduce them into theta_bar).
        Segments of one trajectory give bitwise the one-call gradient when each
        has an even number of steps."""
        if ws is None:
            ws = self.workspace(A.OP_VJP)
        flags = (A.VJP_BEGIN if begin else 0) | (A.VJP_END if end else 0)
        # the fused plan: two adjoint steps per launch when it was built for ks >= 2
        A.check(self.L.pf_vjp_explicit_batched(A.ctx(self.device), ct.byref(self.info), ct.c_void_p(self.plan.data_ptr()),
                                               int(nsteps), ct.c_void_p(states.data_ptr()),
                                               ct.c_void_p(lam.data_ptr()),
                                               ct.c_void_p(theta_bar.data_ptr()),
                                               ct.c_void_p(ws.data_ptr()), flags, _stream()))

    def autotune(self, U_scratch):
        """Time every launch shape on U_scratch (overwritten); keep the fastest."""
        ws = self.workspace(A.OP_STEP_EXPLICIT)
        us = ct.c_double(0.0)
        info = A.pf_batch_info()
        A.check(self.L.pf_batch_autotune(A.ctx(self.device), ct.byref(self.base), self.samples, self.count, self.dt,
                                         ct.c_void_p(U_scratch.data_ptr()), ct.c_void_p(ws.data_ptr()),
                                         ct.c_void_p(self.plan.data_ptr()), self.plan.numel(),
                                         ct.byref(info), ct.byref(us), _stream()))
        self.info = info
        self.set_theta(self.theta, ks=info.ks, ty=info.ty, depth=info.depth)
        return dict(ks=info.ks, ty=info.ty, depth=info.depth, us_per_step=us.value)


class BatchedExplicitRun(torch.autograd.Function):
    """U_N = S^N(U_0; theta) for a batch, with a hand-written adjoint.

    every = k: forward keeps a snapshot every k steps and the last segment's states;
    backward walks the segments in reverse, applies the batched step adjoint to
    each, and meanwhile recomputes the next one's states from its snapshot
    (trajectory mode) on a second stream.
    every = None: forward writes the whole trajectory (N states) in device memory
    as it runs (trajectory mode), and backward applies the adjoint to it directly,
    with no recomputation; on a 288 GB device this holds, e.g., 2000 states of a
    7.6 M-node batch (61 GB in FP32).
    Either way the per-sample gradient of theta = (mobility, kappa, W) accumulates
    in FP64 (Supp. Note 2, Eqs. II.5-II.6, one constraint per step), and both give
    bitwise the same gradient for even checkpoint intervals.
    """

    @staticmethod
    def forward(ctx, theta, U0, batch, nsteps, every):
        if every is not None and nsteps % every:
            raise ValueError("nsteps must be a multiple of the checkpoint interval")
        batch.set_theta(theta.detach().cpu().numpy(), ks=batch.info.ks, ty=batch.info.ty,
                        depth=batch.info.depth)
        ctx.batch, ctx.every, ctx.nsteps = batch, every, nsteps
        if every is None:
            traj = torch.empty((nsteps + 1, batch.total), dtype=batch.dtype, device=U0.device)
            traj[0].copy_(U0.detach())
            if nsteps:
                batch.step(traj[0], nsteps, traj=traj[1])
            ctx.traj = traj
            return traj[nsteps].clone()
        ws = batch.workspace(A.OP_STEP_EXPLICIT)
        U = U0.detach().clone()
        snaps = []
        nseg = nsteps // every
        ctx.snaps, ctx.last = [], None
        if nseg == 0:
            return U
        for _ in range(nseg - 1):
            snaps.append(U.clone())
            batch.step(U, every, ws)
        ctx.snaps = snaps
        # the last segment runs in trajectory mode: the backward pass starts on
        # its states without recomputing them
        last = torch.empty((every + 1, batch.total), dtype=batch.dtype, device=U0.device)
        last[0].copy_(U)
        batch.step(last[0], every, traj=last[1])
        ctx.last = last
        return last[every].clone()

    @staticmethod
    def backward(ctx, gU):
        b, every = ctx.batch, ctx.every
        lam = gU.detach().to(b.dtype).contiguous().clone()
        tb = torch.zeros(b.count * 3, dtype=torch.float64, device=b.device)
        ws = b.workspace(A.OP_VJP)
        if every is None:
            if ctx.traj is None:
                raise RuntimeError("the batched adjoint's states were released by an earlier backward")
            if ctx.nsteps:
                b.vjp(ctx.traj, lam, tb, ctx.nsteps, ws, begin=True, end=True)
            ctx.traj = None
            return tb.view(b.count, 3), lam, None, None, None
        if ctx.last is None:
            if ctx.snaps is None:
                raise RuntimeError("the batched adjoint's states were released by an earlier backward")
            return tb.view(b.count, 3), lam, None, None, None  # no steps
        # segments in reverse; the last one's states were kept by the forward pass
        snaps = [None] + ctx.snaps[::-1]
        nseg = len(snaps)
        # two segment buffers: while the adjoint walks segment i on the caller's
        # stream, a second stream recomputes segment i + 1 from its snapshot, so
        # each launch's tail is filled by the other kernel
        seg = [ctx.last]
        if nseg > 1:
            seg.append(torch.empty((every, b.total), dtype=b.dtype, device=b.device))
        ctx.last = ctx.snaps = None
        main = torch.cuda.current_stream(b.device)
        side = b.side_stream()

        def recompute(j):
            buf = seg[j % 2]
            buf[0].copy_(snaps[j])
            if every > 1:
                b.step(buf[0], every - 1, traj=buf[1])

        for i in range(nseg):
            if i + 1 < nseg:
                side.wait_stream(main)  # the adjoint of segment i - 1 has released its buffer
                with torch.cuda.stream(side):
                    recompute(i + 1)
            b.vjp(seg[i % 2], lam, tb, every, ws, begin=(i == 0), end=(i == nseg - 1))
            if i + 1 < nseg:
                main.wait_stream(side)
        return tb.view(b.count, 3), lam, None, None, None


def trajectory_fits(batch, nsteps, reserve=0.8):
    """True when nsteps + 1 states of the batch fit in `reserve` of the free device memory."""
    free, _ = torch.cuda.mem_get_info(batch.device)
    es = torch.empty((), dtype=batch.dtype).element_size()
    return (nsteps + 1) * batch.total * es <= reserve * free


def explicit_run(theta, U0, batch, nsteps, every="auto"):
    """Differentiable batched explicit trajectory (see BatchedExplicitRun).
    every: checkpoint interval, None to keep the whole trajectory, or "auto" (the
    whole trajectory when it fits in device memory, else a snapshot every 100)."""
    if every == "auto":
        every = None if trajectory_fits(batch, nsteps) else 100
    return BatchedExplicitRun.apply(theta, U0, batch, nsteps, every)


def per_sample_mse(batch, U, targets):
    """sum over samples of mean over nodes (U_s - target_s)^2 (FP64 accumulation), as
    one weighted sum over the packed batch (a handful of launches, not several per
    sample); the padding between samples has weight 0 and is masked, whatever it holds."""
    w = batch.mse_weights()
    d = torch.where(w > 0, U.double() - targets.double(), 0.0)
    return (w * d * d).sum()
