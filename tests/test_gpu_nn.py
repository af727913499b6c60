"""Convolutional surrogate: BF16-MFMA kernels vs the FP64 oracle on identical
bf16 operands and rounding points, the residual check vs the oracle's
backward-Euler residual, training, and the checked rollout's fallback."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2601_06079_amd import _abi as A
from paper_2601_06079_amd import nn as NN
from tests.gpu_util import announce, host, rel_l2

pytestmark = pytest.mark.gpu
F32 = torch.float32


def _inputs(Bn, H, W, seed):
    r = np.random.default_rng(seed)
    c = (0.5 + 0.3 * np.tanh(r.standard_normal((Bn, H, W)))).astype(np.float32)
    M = r.uniform(0.5, 2.0, Bn).astype(np.float32)
    k = r.uniform(0.5, 2.0, Bn).astype(np.float32)
    t = (c + 0.05 * r.standard_normal((Bn, H, W))).astype(np.float32)
    return c, M, k, t


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


def _params(seed):
    return NN.init_params(seed, out_scale=1.0).astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("shape", [(2, 8, 32), (1, 13, 64), (3, 4, 96)])
def test_forward_matches_oracle(shape):
    announce("nn forward", shape)
    Bn, H, W = shape
    c, M, k, _ = _inputs(Bn, H, W, 1)
    p = _params(2)
    model = NN.Surrogate(params=p)
    got = host(model.forward(_dev(c), _dev(M), _dev(k)))
    ref, _, _ = O.nn(c.astype(np.float64), M[:, None, None].astype(np.float64),
                     k[:, None, None].astype(np.float64), p, round_bf16=True)
    assert rel_l2(got - c, ref - c) < 1e-3
    # exact mass per sample (the projection), to FP32 rounding of the field
    assert np.max(np.abs(got.mean(axis=(1, 2)) - c.astype(np.float64).mean(axis=(1, 2)))) < 1e-6


@pytest.mark.parametrize("shape", [(2, 8, 32), (2, 12, 64)])
def test_backward_matches_oracle(shape):
    announce("nn backward", shape)
    Bn, H, W = shape
    c, M, k, t = _inputs(Bn, H, W, 3)
    p = _params(4)
    model = NN.Surrogate(params=p)
    loss, grad = model.loss_and_grad(_dev(c), _dev(M), _dev(k), _dev(t))
    _, lref, gref = O.nn(c.astype(np.float64), M[:, None, None].astype(np.float64),
                         k[:, None, None].astype(np.float64), p, target=t.astype(np.float64),
                         round_bf16=True, grad=True)
    assert float(host(loss).sum()) == pytest.approx(lref, rel=1e-3)
    g = host(grad)
    off = 0
    for name, shp in NN.LAYOUT:
        n = int(np.prod(shp))
        err = rel_l2(g[off:off + n], gref[off:off + n])
        assert err < 5e-3, (name, err)
        off += n


def test_adam_matches_oracle():
    model = NN.Surrogate(seed=5)
    p0 = host(model.params).astype(np.float64)
    m, v, p = np.zeros_like(p0), np.zeros_like(p0), p0.copy()
    r = np.random.default_rng(6)
    for t in range(1, 4):
        g = r.standard_normal(p0.size).astype(np.float32)
        model.t += 1
        A.check(model.L.pf_nn_adam(NN._p(model.params), NN._p(model.m), NN._p(model.v),
                                   NN._p(_dev(g)), model.t, 1e-2, 0.9, 0.999, 1e-8, NN._stream()))
        O.adam(p, m, v, g.astype(np.float64), 1e-2, 0.9, 0.999, 1e-8, t)
    np.testing.assert_allclose(host(model.params), p, rtol=2e-5, atol=2e-6)


def test_residual_check_matches_oracle_be_residual():
    """rho = ||R_BE(c_hat; c, K dt)|| / ||m (c_hat - c)/(K dt)|| for the c-row, with
    R_BE evaluated by the oracle's own residual (Eqs. 13-14)."""
    Bn, n, K, dt = 2, 32, 20, 0.01
    M = np.array([1.2, 0.7])
    kap = np.array([0.9, 1.6])
    ens = NN.CHEnsemble(Bn, n, M, kap, dt=dt, seed=3)
    ens.advance(400)
    c = ens.field().clone()
    ens.advance(K)
    chat = ens.field().clone() + 1e-4 * torch.sin(torch.arange(n, device="cuda", dtype=F32))[None, None, :]
    chat = chat - chat.mean(dim=(1, 2), keepdim=True) + c.mean(dim=(1, 2), keepdim=True)
    step = chat.reshape(-1).clone()
    ens.batch.step(step, 1, ens.ws)
    model = NN.Surrogate(seed=0)
    out = host(model.check(chat, c, step.view_as(chat), K * dt, dt))
    for b in range(Bn):
        o = O.Problem(n=(n, n), model=O.CH, fe=O.F_01, W=1.0, kappa=kap[b], mob=M[b])
        cb = host(c[b]).ravel()
        hb = host(chat[b]).ravel()
        U = O.explicit(o, np.concatenate([hb, 0 * hb]), dt, 0)  # mu = g(c_hat)/m
        R = O.be_residual(o, K * dt, np.concatenate([cb, 0 * cb]), U)[: n * n]
        rho = np.linalg.norm(R) / np.linalg.norm((hb - cb) / (K * dt))
        assert out[b, 0] == pytest.approx(rho, rel=2e-3)


def test_training_reduces_loss():
    announce("nn training")
    model = NN.Surrogate(seed=1)
    hist = NN.train(model, n=64, Bn=8, iters=120, K=20, burn=(600, 2000), lr=2e-3, seed=2)
    assert np.mean(hist[-20:]) < 0.5 * np.mean(hist[:5])


def test_forced_fallback_equals_plain_solver_bitwise():
    """tau = 0 rejects every jump: the rollout is then exactly the plain solver."""
    Bn, n, K = 3, 64, 20
    M, kap = np.array([1.0, 1.5, 0.6]), np.array([1.2, 0.8, 1.9])
    a = NN.CHEnsemble(Bn, n, M, kap, seed=9)
    b = NN.CHEnsemble(Bn, n, M, kap, seed=9)
    a.advance(200)
    b.advance(200)
    model = NN.Surrogate(seed=4)
    fb = NN.rollout(model, a, jumps=3, K=K, tau=0.0)
    b.advance(3 * K)
    assert fb == 3 * Bn
    assert torch.equal(a.U, b.U)
