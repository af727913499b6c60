"""Checkpointed single-problem runs behind torch.autograd (explicit and
backward-Euler Newton steps): gradients vs the FP64 oracle's discrete adjoints,
vs central differences, and independence of the checkpoint interval."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2601_06079_amd import _abi as A
from paper_2601_06079_amd import solver as S
from tests.gpu_util import announce, dev, host, pair, rel_l2

pytestmark = pytest.mark.gpu
F32, F64 = torch.float32, torch.float64


def _grads(g, theta, U0, dt, nsteps, every, w, implicit=False, opts=None):
    th = torch.tensor(theta, dtype=F64, device="cuda", requires_grad=True)
    u0 = dev(U0, g.dtype).requires_grad_(True)
    UN = S.checkpointed_run(th, u0, g, dt, nsteps, every=every, implicit=implicit, opts=opts)
    (UN * dev(w, g.dtype)).sum().backward()
    return th.grad.detach().clone(), u0.grad.detach().clone(), UN.detach()


@pytest.mark.parametrize("model", [O.AC, O.CH])
def test_explicit_run_gradient_matches_oracle_adjoint(model):
    announce("checkpointed explicit run vs oracle", model)
    fe = O.F_SYM if model == O.AC else O.F_01
    theta = np.array([1.2, 0.8, 1.3])  # mobility, kappa, W
    g, o = pair((12, 10), model, fe, F64, W=theta[2], kappa=theta[1], mob=theta[0])
    rng = np.random.default_rng(4)
    N = o.nnodes
    c0 = rng.uniform(0.2, 0.8, N) if model == O.CH else rng.uniform(-0.5, 0.5, N)
    U0 = np.concatenate([c0, np.zeros(N)]) if model == O.CH else c0
    w = rng.standard_normal(o.ndof)
    if model == O.CH:
        w[N:] = 0.0  # only the c plane of an explicit run is differentiated
    dt, nsteps = (0.01, 20) if model == O.CH else (0.05, 20)
    tb, ub, UN = _grads(g, theta, U0, dt, nsteps, 5, w)
    assert rel_l2(host(UN)[:N], O.explicit(o, U0, dt, nsteps)[:N]) < 1e-12
    tref, uref = O.explicit_adjoint(o, dt, nsteps, U0, w[:N])
    np.testing.assert_allclose(host(tb), tref, rtol=1e-9, atol=1e-13)
    assert rel_l2(host(ub)[:N], uref) < 1e-10


@pytest.mark.parametrize("model", [O.AC, O.CH])
def test_explicit_run_noflux_gradient_matches_oracle_adjoint(model):
    """No-flux grid (the paper's benchmark boundary): the checkpointed explicit run's
    gradient against the oracle's discrete adjoint, and independent of the checkpoint
    interval bitwise (both passes advance with single-step launches there)."""
    announce("checkpointed explicit run, no-flux, vs oracle", model)
    fe = O.F_SYM if model == O.AC else O.F_01
    theta = np.array([1.1, 0.9, 1.2])
    g, o = pair((14, 11), model, fe, F64, W=theta[2], kappa=theta[1], mob=theta[0], bc=O.NOFLUX)
    rng = np.random.default_rng(17)
    N = o.nnodes
    c0 = rng.uniform(0.2, 0.8, N) if model == O.CH else rng.uniform(-0.5, 0.5, N)
    U0 = np.concatenate([c0, np.zeros(N)]) if model == O.CH else c0
    w = rng.standard_normal(o.ndof)
    if model == O.CH:
        w[N:] = 0.0
    dt, nsteps = (0.01, 12) if model == O.CH else (0.05, 12)
    tb, ub, UN = _grads(g, theta, U0, dt, nsteps, 4, w)
    assert rel_l2(host(UN)[:N], O.explicit(o, U0, dt, nsteps)[:N]) < 1e-12
    tref, uref = O.explicit_adjoint(o, dt, nsteps, U0, w[:N])
    np.testing.assert_allclose(host(tb), tref, rtol=1e-9, atol=1e-13)
    assert rel_l2(host(ub)[:N], uref) < 1e-10
    tb2, ub2, _ = _grads(g, theta, U0, dt, nsteps, 12, w)
    assert torch.equal(tb, tb2) and torch.equal(ub, ub2)


def _oracle_implicit_adjoint(o, dt, nsteps, U0, w):
    """Chain of the oracle's one-step BE adjoints along its own roots."""
    states = [np.asarray(U0, float)]
    for _ in range(nsteps):
        U, conv, _, _ = O.newton_be(o, dt, states[-1], rtol=1e-13, maxit=40, solver=0)
        assert conv
        states.append(U)
    lam, tb = np.asarray(w, float).copy(), np.zeros(3)
    for k in reversed(range(nsteps)):
        t, lam = O.newton_adjoint(o, dt, states[k + 1], lam, solver=0)
        tb += t
    return tb, lam, states[-1]


@pytest.mark.parametrize("model", [O.AC, O.CH])
def test_implicit_run_gradient_matches_oracle_adjoint(model):
    announce("checkpointed implicit run vs oracle", model)
    fe = O.F_SYM if model == O.AC else O.F_01
    theta = np.array([0.9, 1.4, 1.1])
    g, o = pair((10, 8), model, fe, F64, W=theta[2], kappa=theta[1], mob=theta[0])
    rng = np.random.default_rng(7)
    N = o.nnodes
    U0 = (np.concatenate([rng.uniform(0.3, 0.7, N), np.zeros(N)]) if model == O.CH
          else rng.uniform(-0.6, 0.6, N))
    w = rng.standard_normal(o.ndof)
    dt, nsteps = (0.5, 4) if model == O.CH else (0.2, 4)
    opts = S.newton_opts(rtol=1e-13, lin_rtol_min=1e-13, lin_rtol_max=1e-13, max_newton=40)
    tb, ub, UN = _grads(g, theta, U0, dt, nsteps, 2, w, implicit=True, opts=opts)
    tref, uref, Uref = _oracle_implicit_adjoint(o, dt, nsteps, U0, w)
    assert rel_l2(host(UN), Uref) < 1e-10
    np.testing.assert_allclose(host(tb), tref, rtol=1e-7, atol=1e-10)
    assert rel_l2(host(ub), uref) < 1e-7


def test_checkpoint_interval_does_not_change_gradients():
    """Recomputed segments are bitwise the forward's states, so the gradient is
    the same for every checkpoint interval."""
    announce("checkpoint interval invariance")
    g, o = pair((40, 36), O.CH, O.F_01, F32, W=1.0, kappa=1.7, mob=0.8)
    rng = np.random.default_rng(11)
    U0 = np.concatenate([rng.uniform(0.45, 0.55, o.nnodes), np.zeros(o.nnodes)])
    w = np.concatenate([rng.standard_normal(o.nnodes), np.zeros(o.nnodes)])
    th = [0.8, 1.7, 1.0]
    a = _grads(g, th, U0, 0.01, 24, 4, w)
    b = _grads(g, th, U0, 0.01, 24, 24, w)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    gi, _ = pair((12, 12), O.AC, O.F_SYM, F64, W=1.0, kappa=1.0, mob=1.0)
    U0 = rng.uniform(-0.5, 0.5, 144)
    w = rng.standard_normal(144)
    a = _grads(gi, [1.0, 1.0, 1.0], U0, 0.3, 4, 1, w, implicit=True)
    b = _grads(gi, [1.0, 1.0, 1.0], U0, 0.3, 4, 4, w, implicit=True)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


def test_implicit_run_gradient_vs_central_differences():
    announce("implicit run vs central FD")
    theta = np.array([1.1, 0.9, 1.2])
    g, _ = pair((16, 16), O.AC, O.F_SYM, F64)
    rng = np.random.default_rng(13)
    U0 = rng.uniform(-0.5, 0.5, 256)
    w = rng.standard_normal(256)
    opts = S.newton_opts(rtol=1e-13, lin_rtol_min=1e-13, lin_rtol_max=1e-13, max_newton=40)
    tb, _, _ = _grads(g, theta, U0, 0.4, 3, 3, w, implicit=True, opts=opts)

    def loss(th):
        with torch.no_grad():
            UN = S.checkpointed_run(torch.tensor(th, dtype=F64), dev(U0, F64), g, 0.4, 3, every=3,
                                    implicit=True, opts=opts)
        return float((host(UN) * w).sum())

    for k in range(3):
        e = 1e-6 * theta[k]
        tp, tm = theta.copy(), theta.copy()
        tp[k] += e
        tm[k] -= e
        fd = (loss(tp) - loss(tm)) / (2 * e)
        assert abs(host(tb)[k] - fd) <= 1e-6 * max(abs(fd), 1e-3), (k, host(tb)[k], fd)
