"""Convolutional surrogate: BF16-MFMA kernels vs the FP64 oracle on identical
bf16 operands and rounding points, the residual check vs the oracle's
backward-Euler residual, training, and the checked rollout's fallback."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2601_06079_amd import _abi as A
from paper_2601_06079_amd import nn as NN
from paper_2601_06079_amd import solver as S
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


def _dyadic(seed, Bn, H, W):
    """Inputs and weights on coarse power-of-two grids, so that every sum either side
    forms is exact in FP32 whatever its order (checked by _exact_bound), and every
    hidden activation is a multiple of 1/16 that bf16 rounds the same way on both
    sides.  c in {0, 1/4, ..., 1}; M, kappa in {1/2, 1, 3/2, 2}; W1 in {0, +-1/4};
    W2, W3 sparse in {0, +-1}; W4 sparse in {0, +-2^-10}; biases in (1/16) Z."""
    r = np.random.default_rng(seed)
    c = r.integers(0, 5, (Bn, H, W)) / 4.0
    M = r.integers(1, 5, Bn) / 2.0
    k = r.integers(1, 5, Bn) / 2.0
    parts = []
    for name, shp in NN.LAYOUT:
        n = int(np.prod(shp))
        if name == "W1":
            v = r.integers(-1, 2, n) / 4.0
        elif name in ("W2", "W3"):
            v = r.choice([-1.0, 0.0, 1.0], n, p=[1 / 32, 15 / 16, 1 / 32])
        elif name == "W4":
            v = r.choice([-1.0, 0.0, 1.0], n, p=[1 / 16, 7 / 8, 1 / 16]) * 2.0 ** -10
        elif name == "b4":
            v = np.zeros(n)
        else:
            v = r.integers(-8, 9, n) / 16.0
        parts.append(v)
    return c, M, k, np.concatenate(parts)


def _exact_bound(p):
    """Largest (sum of |terms|) / (grid of the terms) over the four layers: below 2^24
    every partial sum is a multiple of the grid that FP32 holds exactly."""
    off, blocks = 0, {}
    for name, shp in NN.LAYOUT:
        n = int(np.prod(shp))
        blocks[name] = p[off:off + n].reshape(shp)
        off += n
    amax = np.array([1.0, 2.0, 2.0])  # max |a0| per input channel (c, M, kappa)
    grid, worst = 0.25, 0.0           # grid of a0 (c: 1/4; M, kappa: 1/2)
    for l, wgrid in ((1, 0.25), (2, 1.0), (3, 1.0), (4, 2.0 ** -10)):
        w = np.abs(blocks[f"W{l}"]).reshape(9, -1, blocks[f"W{l}"].shape[-1])
        b = np.abs(blocks[f"b{l}"])
        s = np.einsum("tic,i->c", w, amax) + b
        grid = min(grid * wgrid, 1.0 / 16 if l < 4 else grid * wgrid)
        worst = max(worst, float(s.max()) / grid)
        amax = np.full(32, float(s.max()) * (1 + 2.0 ** -8))  # bf16 rounding may round up
    return worst


@pytest.mark.parametrize("shape", [(2, 8, 64), (1, 5, 32), (3, 4, 96), (1, 13, 160), (2, 1, 32), (3, 2, 64)])
def test_forward_exact_dyadic(shape):
    """Exact arithmetic on both sides: the GPU forward equals the oracle's up to the
    final FP32 rounding of c_hat (pins every tap, channel and tile index)."""
    announce("nn forward exact", shape)
    Bn, H, W = shape
    c, M, k, p = _dyadic(11 + H, Bn, H, W)
    assert _exact_bound(p) < 2.0 ** 24
    model = NN.Surrogate(params=p)
    got = host(model.forward(_dev(c.astype(np.float32)), _dev(M.astype(np.float32)),
                             _dev(k.astype(np.float32))))
    ref, _, _ = O.nn(c, M[:, None, None] * np.ones_like(c), k[:, None, None] * np.ones_like(c),
                     p, round_bf16=True)
    d_ref = ref - c
    assert np.std(d_ref) > 1e-3  # the network is not trivially zero
    assert np.max(np.abs((got - c) - d_ref)) <= 4e-7 * max(1.0, np.max(np.abs(ref)))


def test_forward_exact_dyadic_full_size():
    """One sample of the surrogate workload's full size (512 x 512) in exact
    arithmetic: every tile of the launch the benchmark uses, against the oracle."""
    announce("nn forward exact 512^2")
    c, M, k, p = _dyadic(5, 1, 512, 512)
    assert _exact_bound(p) < 2.0 ** 24
    model = NN.Surrogate(params=p)
    got = host(model.forward(_dev(c.astype(np.float32)), _dev(M.astype(np.float32)),
                             _dev(k.astype(np.float32))))
    ref, _, _ = O.nn(c, M[:, None, None] * np.ones_like(c), k[:, None, None] * np.ones_like(c),
                     p, round_bf16=True)
    assert np.std(ref - c) > 1e-3
    assert np.max(np.abs((got - c) - (ref - c))) <= 4e-7 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("shape", [(2, 8, 32), (1, 13, 64), (3, 4, 96), (2, 64, 128), (3, 1, 32), (2, 2, 96)])
def test_forward_matches_oracle(shape):
    """Random weights: the two sides sum in different orders, so an activation that
    lies within FP32 noise of a bf16 rounding boundary can round one ulp apart (one
    such flip moves d by ~|W4| 2^-8 |a| over up to 7x7 pixels).  The tolerance
    covers a few flips on a small grid; the exact test above pins the indexing."""
    announce("nn forward", shape)
    Bn, H, W = shape
    c, M, k, _ = _inputs(Bn, H, W, 1)
    p = _params(2)
    model = NN.Surrogate(params=p)
    got = host(model.forward(_dev(c), _dev(M), _dev(k)))
    ref, _, _ = O.nn(c.astype(np.float64), M[:, None, None].astype(np.float64),
                     k[:, None, None].astype(np.float64), p, round_bf16=True)
    assert rel_l2(got - c, ref - c) < (1e-3 if Bn * H * W >= 8192 else 5e-3)
    # exact mass per sample (the projection), to FP32 rounding of the field
    assert np.max(np.abs(got.mean(axis=(1, 2)) - c.astype(np.float64).mean(axis=(1, 2)))) < 1e-6


@pytest.mark.parametrize("group", [1, 2, 3])
def test_forward_sample_groups_bitwise(group):
    """The forward pass runs in groups of samples (each with its own M, kappa): every
    grouping gives the bits of the single-group pass, and the single-group pass
    matches the oracle."""
    announce("nn forward groups", group)
    Bn, H, W = 5, 8, 64
    c, M, k, _ = _inputs(Bn, H, W, 7)
    p = _params(3)
    model = NN.Surrogate(params=p)
    try:
        S.tune_set(A.TUNE_NN_GROUP, Bn)
        ref = model.forward(_dev(c), _dev(M), _dev(k)).clone()
        S.tune_set(A.TUNE_NN_GROUP, group)
        got = model.forward(_dev(c), _dev(M), _dev(k))
    finally:
        S.tune_set(A.TUNE_NN_GROUP, 0)
    assert torch.equal(got, ref)
    o, _, _ = O.nn(c.astype(np.float64), M[:, None, None].astype(np.float64),
                   k[:, None, None].astype(np.float64), p, round_bf16=True)
    assert rel_l2(host(ref) - c, o - c) < 5e-3


def test_forward_unaligned_buffers_bitwise():
    """c and c_hat at a 4-byte offset take the projection's scalar path; it gives the
    bits of the vectorised one (the same mean and the same per-pixel formula)."""
    announce("nn forward unaligned")
    Bn, H, W = 3, 8, 64
    c, M, k, _ = _inputs(Bn, H, W, 17)
    p = _params(18)
    model = NN.Surrogate(params=p)
    Md, kd = _dev(M), _dev(k)  # kept alive until the asynchronous call has read them
    ref = model.forward(_dev(c), Md, kd).clone()
    n = Bn * H * W
    cbuf = torch.zeros(n + 1, dtype=F32, device="cuda")
    cbuf[1:] = _dev(c).reshape(-1)
    obuf = torch.zeros(n + 1, dtype=F32, device="cuda")
    cu, ou = cbuf[1:].view(Bn, H, W), obuf[1:].view(Bn, H, W)
    A.check(model.L.pf_nn_forward(NN._p(model.params), Bn, H, W, NN._p(cu), NN._p(Md), NN._p(kd),
                                  NN._p(ou), NN._p(model.workspace(Bn, H, W)), NN._stream()))
    torch.cuda.synchronize()
    assert torch.equal(ou, ref)


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
        if name == "b4":
            # c_hat does not depend on the output bias (the mean is subtracted): the
            # exact gradient is 0 and both sides return rounding noise
            assert abs(g[off]) <= 1e-6 * np.linalg.norm(gref[off - 288:off])
            assert abs(gref[off]) <= 1e-12 * np.linalg.norm(gref[off - 288:off])
        else:
            err = rel_l2(g[off:off + n], gref[off:off + n])
            assert err < 5e-3, (name, err)
        off += n


@pytest.mark.parametrize("shape", [(2, 8, 64), (1, 16, 32)])
def test_backward_exact_dyadic(shape):
    """Exact arithmetic through the whole backward pass (pins every index of the
    weight and data gradients).  The forward is exact (dyadic weights and inputs, see
    _dyadic); with H W = 512 every c_hat is a multiple of 2^-23 below 2 in magnitude,
    so FP32 holds it exactly on both sides.  The target is c_hat minus a zero-mean
    offset delta of +-2^-6 on a few pixels, so dL/dc_hat = 2 delta / (H W) = +-2^-14,
    its mean is exactly 0 and the data gradients stay multiples of 2^-24 whose sums
    fit FP32's 24 bits (9 x 2^-24 after the output layer, below 2^-12 after layer 3,
    below 2^-3.8 after layer 2): each side rounds the same exact values to bf16.
    The weight gradients are FP32 sums over pixels in different orders on the two
    sides, so they agree to accumulation rounding (held to 1e-6); the output bias
    has an exactly zero gradient on both sides."""
    announce("nn backward exact", shape)
    Bn, H, W = shape
    HW = H * W
    assert HW == 512
    c, M, k, p = _dyadic(31 + H, Bn, H, W)
    assert _exact_bound(p) < 2.0 ** 24
    Mb, kb = M[:, None, None] * np.ones_like(c), k[:, None, None] * np.ones_like(c)
    ref, _, _ = O.nn(c, Mb, kb, p, round_bf16=True)
    r = np.random.default_rng(7 + H)
    delta = np.zeros((Bn, H, W))
    for b in range(Bn):
        idx = r.choice(HW, 12, replace=False)
        delta[b].flat[idx[:6]] = 2.0 ** -6
        delta[b].flat[idx[6:]] = -2.0 ** -6
    t = ref - delta
    assert np.array_equal(t.astype(np.float32).astype(np.float64), t)
    model = NN.Surrogate(params=p)
    cd, Md, kd = _dev(c.astype(np.float32)), _dev(M.astype(np.float32)), _dev(k.astype(np.float32))
    got = host(model.forward(cd, Md, kd))
    assert np.array_equal(got, ref)  # the forward is exact
    loss, grad = model.loss_and_grad(cd, Md, kd, _dev(t.astype(np.float32)))
    _, lref, gref = O.nn(c, Mb, kb, p, target=t, round_bf16=True, grad=True)
    assert lref == Bn * 12 * 2.0 ** -12 / HW
    assert float(host(loss).sum()) == lref
    g = host(grad)
    off = 0
    for name, shp in NN.LAYOUT:
        n = int(np.prod(shp))
        if name == "b4":
            assert g[off] == 0.0 and gref[off] == 0.0
        else:
            assert np.linalg.norm(gref[off:off + n]) > 0, name
            err = rel_l2(g[off:off + n], gref[off:off + n])
            assert err < 1e-6, (name, err)
        off += n


def test_backward_matches_oracle_8192_pixels():
    """Random weights on 2 x 64 x 64 = 8192 pixels: the rounding flips of single
    activations (see test_forward_matches_oracle) average out over this many pixels,
    so every layer's gradient is held to 1e-3 relative L2."""
    announce("nn backward 8192 px")
    Bn, H, W = 2, 64, 64
    c, M, k, t = _inputs(Bn, H, W, 13)
    p = _params(14)
    model = NN.Surrogate(params=p)
    loss, grad = model.loss_and_grad(_dev(c), _dev(M), _dev(k), _dev(t))
    _, lref, gref = O.nn(c.astype(np.float64), M[:, None, None].astype(np.float64),
                         k[:, None, None].astype(np.float64), p, target=t.astype(np.float64),
                         round_bf16=True, grad=True)
    assert float(host(loss).sum()) == pytest.approx(lref, rel=1e-4)
    g = host(grad)
    off = 0
    for name, shp in NN.LAYOUT:
        n = int(np.prod(shp))
        if name != "b4":
            err = rel_l2(g[off:off + n], gref[off:off + n])
            assert err < 1e-3, (name, err)
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


def test_gain_protocol_small():
    """The matched-error gain protocol on a small case: its invariants, not its
    outcome (the full 512^2 figure is a benchmark record)."""
    announce("nn gain protocol")
    rec = NN.gain_experiment(train_iters=60, n=128, Bn=4, jumps=3, burn=400, seed=3)
    assert 0 <= rec["fallbacks"] <= rec["jumps_total"] == 12
    assert rec["tau"] > 0 and np.isfinite(rec["rollout_rel_err"]) and rec["gain"] > 0
    p0 = rec["plain"][0]
    assert p0["dt"] == 0.01 and p0["rel_err"] < 1e-4  # FP32 vs the FP64 reference, same dt
    if rec["fallbacks"] == rec["jumps_total"]:
        # every jump rejected: the rollout is the plain FP32 solver at dt, bit for bit
        assert rec["rollout_rel_err"] == p0["rel_err"]
    assert all(r["rel_err"] is None or r["rel_err"] < 1e-2 for r in rec["plain"])
