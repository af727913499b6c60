"""Pins of the surrogate's FP64 oracle: bfloat16 rounding against torch's own
conversion, the forward pass against torch.nn.functional.conv2d with circular
padding, the backward pass against torch autograd and finite differences, and
Adam against torch.optim.Adam."""
import numpy as np
import pytest
import torch
import torch.nn.functional as Fn

import oracle as O

rng = np.random.default_rng(7)


def test_bf16_rounding_matches_torch_and_ties_to_even(orc):
    assert O.bf16(1.0) == 1.0
    assert O.bf16(1 + 2 ** -8) == 1.0                 # tie -> even (k = 0)
    assert O.bf16(1 + 3 * 2 ** -8) == 1 + 2 ** -6      # tie -> even (k = 2)
    assert O.bf16(-(1 + 3 * 2 ** -8)) == -(1 + 2 ** -6)
    x = rng.standard_normal(4000).astype(np.float32) * np.exp(rng.uniform(-20, 20, 4000)).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    got = np.array([O.bf16(float(v)) for v in x])
    assert np.array_equal(got, ref)


def _params(scale=0.2, seed=0):
    r = np.random.default_rng(seed)
    out = []
    for name, shape in O.NN_LAYOUT:
        out.append((r.standard_normal(int(np.prod(shape))) * (scale if name[0] == "W" else 0.05)))
    return np.concatenate(out)


def _torch_net(c, M, kap, params):
    """The same network in torch float64 (NCHW, circular padding)."""
    ct_ = torch.as_tensor(c, dtype=torch.float64)
    x = torch.stack([ct_, torch.full_like(ct_, float(M)), torch.full_like(ct_, float(kap))], dim=1)
    p = torch.as_tensor(params)
    off = 0
    layers = []
    for name, shape in O.NN_LAYOUT:
        n = int(np.prod(shape))
        layers.append(p[off:off + n].reshape(shape))
        off += n
    h = x
    for i in range(4):
        w = layers[2 * i].permute(3, 2, 0, 1)  # [ky,kx,ci,co] -> [co,ci,ky,kx]
        b = layers[2 * i + 1]
        h = Fn.conv2d(Fn.pad(h, (1, 1, 1, 1), mode="circular"), w, b)
        if i < 3:
            h = torch.relu(h)
    d = h[:, 0]
    return torch.as_tensor(c) + d - d.mean(dim=(1, 2), keepdim=True)


def test_forward_matches_torch_conv2d(orc):
    B, H, W = 2, 7, 9
    c = rng.uniform(0.3, 0.7, (B, H, W))
    M, kap = 1.3, 0.7
    p = _params()
    chat, _, _ = O.nn(c, M, kap, p, round_bf16=False)
    ref = _torch_net(c, M, kap, p).numpy()
    np.testing.assert_allclose(chat, ref, rtol=1e-12, atol=1e-13)


def test_backward_matches_torch_autograd_and_fd(orc):
    B, H, W = 2, 5, 6
    c = rng.uniform(0.3, 0.7, (B, H, W))
    tgt = rng.uniform(0.3, 0.7, (B, H, W))
    M, kap = 0.9, 1.6
    p = _params(seed=3)
    _, loss, g = O.nn(c, M, kap, p, target=tgt, round_bf16=False, grad=True)
    pt = torch.as_tensor(p).clone().requires_grad_(True)
    chat = _torch_net(c, M, kap, pt)
    L = ((chat - torch.as_tensor(tgt)) ** 2).mean(dim=(1, 2)).sum()
    L.backward()
    assert loss == pytest.approx(L.item(), rel=1e-12)
    np.testing.assert_allclose(g, pt.grad.numpy(), rtol=1e-9, atol=1e-12)
    for i in rng.choice(p.size, 12, replace=False):
        e = np.zeros_like(p)
        e[i] = 1e-6
        fd = (O.nn(c, M, kap, p + e, target=tgt, round_bf16=False)[1] -
              O.nn(c, M, kap, p - e, target=tgt, round_bf16=False)[1]) / 2e-6
        assert g[i] == pytest.approx(fd, rel=1e-5, abs=1e-9)


def test_mean_projection_conserves_mass(orc):
    c = rng.uniform(0.3, 0.7, (3, 8, 8))
    chat, _, _ = O.nn(c, 1.0, 1.0, _params(seed=5), round_bf16=True)
    np.testing.assert_allclose(chat.mean(axis=(1, 2)), c.mean(axis=(1, 2)), atol=1e-14)


def test_adam_matches_torch(orc):
    n = 50
    p = rng.standard_normal(n)
    pt = torch.tensor(p.copy(), requires_grad=True)
    opt = torch.optim.Adam([pt], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    m, v = np.zeros(n), np.zeros(n)
    for t in range(1, 6):
        g = rng.standard_normal(n)
        O.adam(p, m, v, g, 1e-2, 0.9, 0.999, 1e-8, t)
        pt.grad = torch.tensor(g)
        opt.step()
    np.testing.assert_allclose(p, pt.detach().numpy(), rtol=1e-12, atol=1e-14)
