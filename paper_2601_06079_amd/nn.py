"""Convolutional surrogate (learned K-step jump for Cahn-Hilliard) on the GPU:
ctypes binding of pf_nn_* plus the training loop and the checked rollout.

Every forward, backward, optimiser and check step runs in the library's HIP
kernels (BF16 matrix cores for the hidden convolutions); this module only
allocates buffers, draws synthetic training data with the plain batched
solver and strings the calls together.
"""
from __future__ import annotations

import ctypes as ct
import time

import numpy as np
import torch

from . import _abi as A
from . import batch as B


def _bind():
    L = A.lib()
    vp, i32, f64 = ct.c_void_p, ct.c_int, ct.c_double
    sig = {
        "pf_nn_param_count": (i32, []),
        "pf_nn_workspace_size": (i32, [i32, i32, i32, ct.POINTER(ct.c_size_t)]),
        "pf_nn_forward": (i32, [vp, i32, i32, i32, vp, vp, vp, vp, vp, vp]),
        "pf_nn_backward": (i32, [vp, i32, i32, i32, vp, vp, vp, vp, vp, vp, vp, vp]),
        "pf_nn_check": (i32, [i32, i32, i32, vp, vp, vp, f64, f64, vp, vp, vp]),
        "pf_nn_adam": (i32, [vp, vp, vp, vp, i32, f64, f64, f64, f64, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    return L


def _p(t):
    return ct.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return ct.c_void_p(torch.cuda.current_stream().cuda_stream)


LAYOUT = [("W1", (3, 3, 3, 32)), ("b1", (32,)), ("W2", (3, 3, 32, 32)), ("b2", (32,)),
          ("W3", (3, 3, 32, 32)), ("b3", (32,)), ("W4", (3, 3, 32, 1)), ("b4", (1,))]


def init_params(seed=0, out_scale=0.05):
    """He-normal weights for the hidden layers, small output layer, zero biases (FP64 host)."""
    rng = np.random.default_rng(seed)
    out = []
    for name, shape in LAYOUT:
        n = int(np.prod(shape))
        if name[0] == "b":
            out.append(np.zeros(n))
        else:
            fan_in = 9 * shape[2]
            s = np.sqrt(2.0 / fan_in) * (out_scale if name == "W4" else 1.0)
            out.append(rng.standard_normal(n) * s)
    return np.concatenate(out)


class Surrogate:
    """The 4-layer, width-32, 3x3 periodic conv operator with FP32 masters + Adam."""

    def __init__(self, params=None, seed=0, device="cuda"):
        self.L = _bind()
        self.n = int(self.L.pf_nn_param_count())
        p = init_params(seed) if params is None else np.asarray(params, dtype=np.float64)
        assert p.size == self.n
        self.device = torch.device(device)
        self.params = torch.as_tensor(p, dtype=torch.float32, device=self.device).contiguous()
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.t = 0
        self._ws = {}

    def workspace(self, Bn, H, W):
        key = (Bn, H, W)
        if key not in self._ws:
            nb = ct.c_size_t(0)
            A.check(self.L.pf_nn_workspace_size(Bn, H, W, ct.byref(nb)))
            self._ws = {key: torch.empty(int(nb.value), dtype=torch.uint8, device=self.device)}
        return self._ws[key]

    def forward(self, c, M, kappa):
        """c: [B, H, W] float32 device; M, kappa: [B] float32 device -> c_hat [B, H, W]."""
        Bn, H, W = c.shape
        out = torch.empty_like(c)
        A.check(self.L.pf_nn_forward(_p(self.params), Bn, H, W, _p(c), _p(M), _p(kappa), _p(out),
                                     _p(self.workspace(Bn, H, W)), _stream()))
        return out

    def loss_and_grad(self, c, M, kappa, target):
        Bn, H, W = c.shape
        loss = torch.empty(Bn, dtype=torch.float64, device=self.device)
        grad = torch.empty_like(self.params)
        A.check(self.L.pf_nn_backward(_p(self.params), Bn, H, W, _p(c), _p(M), _p(kappa), _p(target),
                                      _p(loss), _p(grad), _p(self.workspace(Bn, H, W)), _stream()))
        return loss, grad

    def train_step(self, c, M, kappa, target, lr=1e-3):
        loss, grad = self.loss_and_grad(c, M, kappa, target)
        self.t += 1
        A.check(self.L.pf_nn_adam(_p(self.params), _p(self.m), _p(self.v), _p(grad), self.t, lr,
                                  0.9, 0.999, 1e-8, _stream()))
        return loss

    def check(self, chat, c_prev, c_step, K_dt, dt):
        """Per-sample (rho, sum(c_hat - c_prev), ||c_hat - c_prev||/(K dt)) as a [B, 3] tensor."""
        Bn, H, W = chat.shape
        out = torch.empty((Bn, 3), dtype=torch.float64, device=self.device)
        A.check(self.L.pf_nn_check(Bn, H, W, _p(chat), _p(c_prev), _p(c_step), K_dt, dt, _p(out),
                                   _p(self.workspace(Bn, H, W)), _stream()))
        return out


# ---------------------------------------------------------------------------
# Cahn-Hilliard trajectories from the plain solver (batched FP32 explicit steps)
class CHEnsemble:
    """Bn independent 2-D Cahn-Hilliard runs of one size with per-sample (M, kappa)."""

    def __init__(self, Bn, n, M, kappa, dt=0.01, W=1.0, seed=0, device="cuda"):
        self.Bn, self.n, self.dt = Bn, n, dt
        self.M = np.asarray(M, dtype=np.float64)
        self.kappa = np.asarray(kappa, dtype=np.float64)
        theta = np.stack([self.M, self.kappa, np.full(Bn, W)], axis=1)
        self.batch = B.Batch([(n, n)] * Bn, theta, dt, model=A.CAHN_HILLIARD, fe=A.F_01,
                             dtype=torch.float32, device=device)
        assert self.batch.total == Bn * n * n  # n*n is a multiple of 64: samples are contiguous
        rng = np.random.default_rng(seed)
        self.U = torch.as_tensor(0.5 + rng.uniform(-0.01, 0.01, Bn * n * n), dtype=torch.float32,
                                 device=device)
        self.ws = self.batch.workspace(A.OP_STEP_EXPLICIT)
        self.Mt = torch.as_tensor(self.M, dtype=torch.float32, device=device)
        self.kt = torch.as_tensor(self.kappa, dtype=torch.float32, device=device)

    def field(self):
        return self.U.view(self.Bn, self.n, self.n)

    def advance(self, nsteps, U=None):
        U = self.U if U is None else U
        self.batch.step(U, nsteps, self.ws)
        return U


def train(model, n=512, Bn=16, iters=300, K=20, dt=0.01, lr=2e-3, lr_min=None, burn=(1500, 6000),
          seed=0, log=None):
    """Train on (c_t, c_{t+K}) pairs drawn along fresh plain-solver trajectories with
    M, kappa ~ U(0.5, 2).  With lr_min the step size follows a cosine decay from lr
    to lr_min over the run.  Returns the per-iteration mean loss."""
    import math
    rng = np.random.default_rng(seed)
    hist = []
    ens = None
    for it in range(iters):
        if it % 25 == 0:  # a new ensemble of trajectories every 25 iterations
            M = rng.uniform(0.5, 2.0, Bn)
            kap = rng.uniform(0.5, 2.0, Bn)
            ens = CHEnsemble(Bn, n, M, kap, dt=dt, seed=int(rng.integers(1 << 30)))
            ens.advance(int(rng.integers(burn[0] // K, burn[1] // K)) * K)
        c0 = ens.field().clone()
        ens.advance(K)
        tgt = ens.field().clone()
        lr_t = lr if lr_min is None else lr_min + 0.5 * (lr - lr_min) * (1 + math.cos(math.pi * it / iters))
        loss = model.train_step(c0, ens.Mt, ens.kt, tgt, lr=lr_t)
        hist.append(float(loss.mean()))
        if log and (it % 100 == 0 or it == iters - 1):
            log(f"iter {it} loss {hist[-1]:.3e}")
    return hist


def rollout(model, ens, jumps, K, tau, energy_check=True):
    """Advance ens by `jumps` surrogate jumps of K steps.  Each jump is checked per
    sample: (i) mass |mean(c_hat) - mean(c)| <= 1e-6, (ii) discrete energy not
    increased beyond 1e-7 relative, (iii) normalised backward-Euler residual of
    the jump rho <= tau.  Samples that fail take K plain solver steps instead
    (the plain solver runs only when some sample fails).  Returns the number of
    fallbacks."""
    from . import solver as S
    Bn, n, dt = ens.Bn, ens.n, ens.dt
    fallbacks = 0
    egeom = [S.Problem(n=(n, n), model=A.ALLEN_CAHN, fe=A.F_01, dtype=torch.float32, W=1.0,
                       kappa=float(k)) for k in ens.kappa]
    ews = S.workspace(egeom[0], A.OP_ENERGY)
    for _ in range(jumps):
        c = ens.field().clone()
        chat = model.forward(c, ens.Mt, ens.kt)
        step = chat.reshape(-1).clone()
        ens.batch.step(step, 1, ens.ws)  # one explicit step of c_hat feeds the residual check
        out = model.check(chat, c, step.view_as(chat), K * dt, dt)
        ok = (out[:, 0] <= tau) & (out[:, 1].abs() <= 1e-6 * n * n)
        if energy_check:
            e = torch.stack([torch.stack([S.energy(g, c[i].reshape(-1), ews)[0],
                                          S.energy(g, chat[i].reshape(-1), ews)[0]])
                             for i, g in enumerate(egeom)])
            ok = ok & (e[:, 1] <= e[:, 0] + 1e-7 * e[:, 0].abs())
        nfail = int((~ok).sum())
        if nfail:
            ens.advance(K)  # plain steps from c for the fallback
            merged = torch.where(ok.view(-1, 1, 1), chat, ens.field())
            ens.U.copy_(merged.reshape(-1))
        else:
            ens.U.copy_(chat.reshape(-1))
        fallbacks += nfail
    return fallbacks


# ---------------------------------------------------------------------------
def _ch_batch(Bn, n, M, kappa, dt, dtype):
    theta = np.stack([np.asarray(M, float), np.asarray(kappa, float), np.ones(Bn)], axis=1)
    return B.Batch([(n, n)] * Bn, theta, dt, model=A.CAHN_HILLIARD, fe=A.F_01, dtype=dtype)


def _timed(fn):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, time.perf_counter() - t0


def gain_experiment(model=None, train_iters=2000, n=512, Bn=16, K=20, dt=0.01, jumps=10,
                    dts=(0.01, 0.0125, 0.02, 0.025), burn=2000, seed=0, log=None):
    """What the surrogate gains over the plain solver at matched error.

    1. Train (train_iters iterations, cosine-decayed Adam, 512^2 pairs).
    2. tau = 99th percentile of rho over plain-solver K-step jumps on held-out
       trajectories (the threshold a correct jump passes 99% of the time).
    3. On fresh held-out samples, advance `jumps` x K steps of dt three ways from
       the same state: (a) the FP64 plain solver at dt (the reference); (b) the
       checked surrogate rollout with plain-solver fallback; (c) the plain FP32
       solver at each dt' in dts (same end time).  Errors are relative L2 against
       (a) over the batch; wall times include every host synchronisation.
    4. The gain is T(cheapest plain dt' whose error <= the rollout's error) / T(rollout)."""
    say = log or (lambda m: None)
    rng = np.random.default_rng(seed)
    if model is None:
        model = Surrogate(seed=int(rng.integers(1 << 30)))
    t_train = 0.0
    if train_iters:
        hist, t_train = _timed(lambda: train(model, n=n, Bn=Bn, iters=train_iters, K=K, dt=dt, lr=1e-3,
                                             lr_min=1e-5, burn=(1000, 6000), seed=seed + 1, log=log))
        say(f"trained {train_iters} iterations in {t_train:.1f} s, final loss {np.mean(hist[-20:]):.3e}")
    # 2. threshold from plain jumps
    cal = CHEnsemble(Bn, n, rng.uniform(0.5, 2, Bn), rng.uniform(0.5, 2, Bn), dt=dt,
                     seed=int(rng.integers(1 << 30)))
    cal.advance(burn)
    rhos = []
    for _ in range(4):
        c0 = cal.field().clone()
        cal.advance(K)
        c1 = cal.field().clone()
        step = c1.reshape(-1).clone()
        cal.batch.step(step, 1, cal.ws)
        rhos.append(model.check(c1, c0, step.view_as(c1), K * dt, dt)[:, 0].cpu().numpy())
        cal.advance(5 * K)
    tau = float(np.percentile(np.concatenate(rhos), 99))
    # 3. held-out rollout
    M, kap = rng.uniform(0.5, 2, Bn), rng.uniform(0.5, 2, Bn)
    test = CHEnsemble(Bn, n, M, kap, dt=dt, seed=int(rng.integers(1 << 30)))
    test.advance(burn)
    U0 = test.U.clone()
    steps = jumps * K
    ref_b = _ch_batch(Bn, n, M, kap, dt, torch.float64)
    ref = U0.double()
    ref_b.step(ref, steps)
    refn = float(ref.norm())
    # surrogate rollout (warm-up jump first, on a copy)
    warm = CHEnsemble(Bn, n, M, kap, dt=dt, seed=0)
    warm.U.copy_(U0)
    rollout(model, warm, 1, K, tau)
    fb, t_sur = _timed(lambda: rollout(model, test, jumps, K, tau))
    err_sur = float((test.U.double() - ref).norm()) / refn
    net_only = CHEnsemble(Bn, n, M, kap, dt=dt, seed=0)
    net_only.U.copy_(U0)
    rollout(model, net_only, jumps, K, tau=float("inf"), energy_check=False)
    err_net = float((net_only.U.double() - ref).norm()) / refn
    plain = []
    for d in dts:
        m = int(round(steps * dt / d))
        b = _ch_batch(Bn, n, M, kap, d, torch.float32)
        ws = b.workspace(A.OP_STEP_EXPLICIT)
        U = U0.clone()
        b.step(U, 10, ws)
        U.copy_(U0)
        _, t = _timed(lambda: b.step(U, m, ws))
        e = float((U.double() - ref).norm()) / refn
        plain.append({"dt": d, "steps": m, "seconds": t, "rel_err": e if np.isfinite(e) else None})
        say(f"plain dt={d}: {m} steps, {t * 1e3:.3f} ms, rel err {e:.3e}")
    ok = [r for r in plain if r["rel_err"] is not None and r["rel_err"] <= err_sur]
    best = min(ok, key=lambda r: r["seconds"]) if ok else plain[0]
    rec = {"workload": f"{Bn} x {n}^2 Cahn-Hilliard, M, kappa ~ U(0.5, 2), {jumps} jumps of K = {K} "
                       f"steps of dt = {dt} after {burn} burn-in steps",
           "train_iters": train_iters, "train_seconds": t_train, "tau": tau,
           "rollout_seconds": t_sur, "rollout_rel_err": err_sur, "fallbacks": int(fb),
           "jumps_total": jumps * Bn, "network_only_rel_err": err_net, "plain": plain,
           "matched_plain_dt": best["dt"] if ok else None,
           "gain": best["seconds"] / t_sur}
    say(f"rollout: {t_sur * 1e3:.3f} ms, rel err {err_sur:.3e}, fallbacks {fb}/{jumps * Bn}, "
        f"tau {tau:.3e}, network-only err {err_net:.3e}, gain {rec['gain']:.3f}")
    return rec
