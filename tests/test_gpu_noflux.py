"""No-flux (natural boundary) grids: the HIP library against the FP64 oracle,
element by element, for every single-problem entry point."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2601_06079_amd import _abi as A
from paper_2601_06079_amd import inputs as I
from paper_2601_06079_amd import solver as S
from tests.gpu_util import announce, dev, host, pair, rel_l2, rounded

pytestmark = pytest.mark.gpu

F32, F64 = torch.float32, torch.float64
NF = O.NOFLUX
TOL = {F32: 1e-5, F64: 1e-12}

# 2-D shapes reach the streaming kernel with one and several strips and chunks;
# 3-D shapes reach the node kernels and the tiled Jacobian product (n < tile and
# n > tile, partial tiles)
SHAPES_2D = [(2, 2), (3, 5), (64, 48), (130, 97), (61, 200)]
SHAPES_3D = [(2, 2, 2), (3, 4, 5), (17, 9, 12), (33, 17, 29)]


def _state(o, lo, hi, seed, base=0.0):
    c = I.uniform_field(o.n, lo, hi, seed=seed, base=base)
    if o.model == O.CH:
        return np.concatenate([c, I.uniform_field(o.n, -0.5, 0.5, seed=seed + 1)])
    return c


@pytest.mark.parametrize("dtype", [F32, F64])
@pytest.mark.parametrize("model", [O.AC, O.CH])
@pytest.mark.parametrize("n", SHAPES_2D + SHAPES_3D)
def test_residual_noflux(n, model, dtype):
    announce("noflux residual", n, model, dtype)
    g, o = pair(n, model, O.F_01 if model == O.CH else O.F_SYM, dtype, h=0.7, W=1.3, kappa=0.9,
                mob=1.1, bc=NF)
    U = rounded(_state(o, -1.0, 1.0, seed=3), dtype)
    assert rel_l2(host(S.residual(g, dev(U, dtype))), O.residual(o, U)) < TOL[dtype]


@pytest.mark.parametrize("dtype", [F32, F64])
@pytest.mark.parametrize("model", [O.AC, O.CH])
@pytest.mark.parametrize("n", [(5, 7), (96, 70), (3, 4, 5), (12, 10, 9), (33, 17, 29)])
def test_jvp_noflux(n, model, dtype):
    announce("noflux jvp", n, model, dtype)
    g, o = pair(n, model, O.F_01, dtype, h=1.0, W=1.0, kappa=2.0, mob=0.8, bc=NF)
    U = rounded(_state(o, 0.2, 0.8, seed=5), dtype)
    v = rounded(np.random.default_rng(9).standard_normal(o.ndof), dtype)
    for inv_dt in (0.0, 2.0):
        Jv = host(S.jvp(g, inv_dt, dev(U, dtype), dev(v, dtype)))
        assert rel_l2(Jv, O.jvp(o, inv_dt, U, v)) < TOL[dtype]


@pytest.mark.parametrize("dtype", [F32, F64])
@pytest.mark.parametrize("n,fe", [((7, 5), O.F_SYM), ((128, 96), O.F_01), ((4, 5, 6), O.F_01),
                                  ((2, 3, 2), O.F_SYM), ((20, 16, 12), O.F_SYM)])
def test_energy_and_mass_noflux(n, fe, dtype):
    announce("noflux energy", n, fe, dtype)
    g, o = pair(n, O.AC, fe, dtype, h=0.8, W=1.2, kappa=1.7, bc=NF)
    U = rounded(I.uniform_field(n, -1, 1, seed=11), dtype)
    out = host(S.energy(g, dev(U, dtype)))
    assert out[0] == pytest.approx(O.energy(o, U), rel=1e-12)
    assert out[1] == pytest.approx(O.total_mass(o, U), rel=1e-12, abs=1e-12)


@pytest.mark.parametrize("dtype", [F32, F64])
@pytest.mark.parametrize("model", [O.AC, O.CH])
@pytest.mark.parametrize("n", SHAPES_2D + SHAPES_3D)
def test_explicit_noflux(n, model, dtype):
    announce("noflux explicit", n, model, dtype)
    if model == O.AC:
        g, o = pair(n, O.AC, O.F_SYM, dtype, W=1.0, kappa=1.0, mob=1.0, bc=NF)
        U0, dt = rounded(_state(o, -0.05, 0.05, 1), dtype), 0.1
    else:
        g, o = pair(n, O.CH, O.F_01, dtype, W=1.0, kappa=2.0, mob=1.0, bc=NF)
        U0, dt = rounded(_state(o, -0.01, 0.01, 2, base=0.5), dtype), 0.01
    N = o.nnodes
    for steps in (1, 5):
        Ug = dev(U0, dtype)
        S.step_explicit(g, Ug, dt, steps)
        ug, uo = host(Ug), O.explicit(o, U0, dt, steps)
        assert rel_l2(ug[:N], uo[:N]) < TOL[dtype] * steps
        tol_upd = 2e-3 if dtype == F32 else 1e-9
        assert rel_l2(ug[:N] - U0[:N], uo[:N] - U0[:N]) < tol_upd
        if model == O.CH:
            assert rel_l2(ug[N:], uo[N:]) < (1e-4 if dtype == F32 else 1e-11)


@pytest.mark.parametrize("ks", [2, 3, 4])
@pytest.mark.parametrize("model,n", [(O.AC, (128, 128)), (O.CH, (200, 150)), (O.CH, (61, 37)),
                                     (O.AC, (5, 7)), (O.CH, (3, 4))])
def test_explicit_noflux_fused_matches_single_steps(ks, model, n):
    """ks fused no-flux steps per launch agree with ks single-step launches to
    rounding.  (Not bitwise, unlike periodic grids: a fused stage evaluates the
    reflected ghost rows, whose stencil sums run in mirrored order.)"""
    announce("noflux fused", ks, model, n)
    fe = O.F_01 if model == O.CH else O.F_SYM
    g, o = pair(n, model, fe, F32, W=1.0, kappa=2.0 if model == O.CH else 1.0, mob=1.0, bc=NF)
    U0 = _state(o, -0.05, 0.05, 12, base=0.5 if model == O.CH else 0.0)
    dt = 0.01 if model == O.CH else 0.1
    out = []
    for fuse in (1, ks):  # single-step launches, then ks fused steps per launch
        try:
            S.tune_set(A.TUNE_STREAM2D_FUSE, fuse)
            t = dev(U0, F32)
            S.step_explicit(g, t, dt, 2 * ks + 1)
        finally:
            S.tune_set(A.TUNE_STREAM2D_FUSE, 0)
        out.append(t)
    ref, t = out
    N = o.nnodes
    assert rel_l2(host(t)[:N] - U0[:N], host(ref)[:N] - U0[:N]) < 1e-5
    assert rel_l2(host(t)[:N], O.explicit(o, rounded(U0, F32), dt, 2 * ks + 1)[:N]) < 1e-5


def test_cahn_hilliard_noflux_conserves_mass_and_decays_energy():
    """Paper-shaped 2-D run: [0, 100]^2 with h = 100/n, no-flux, f' = 4c(c-1)(c-1/2)."""
    n = (256, 256)
    g, o = pair(n, O.CH, O.F_01, F32, h=100.0 / 256, W=1.0, kappa=1.5, mob=1.0, bc=NF)
    U0 = I.initial_state(dict(I.CH2048, n=n), seed=0, dtype=np.float32)
    U = dev(U0, F32)
    gE, _ = pair(n, O.AC, O.F_01, F32, h=100.0 / 256, W=1.0, kappa=1.5, bc=NF)
    e0 = host(S.energy(gE, U[: o.nnodes].contiguous()))
    S.step_explicit(g, U, 1e-4, 500)
    e1 = host(S.energy(gE, U[: o.nnodes].contiguous()))
    assert abs(e1[1] - e0[1]) < 1e-6 * abs(e0[1])
    assert e1[0] <= e0[0]


@pytest.mark.parametrize("dtype", [F64, F32])
@pytest.mark.parametrize("model,n", [(O.AC, (12, 10)), (O.CH, (9, 8)), (O.CH, (6, 5, 4)),
                                     (O.AC, (5, 6, 4)), (O.CH, (17, 16, 18))])
def test_newton_noflux(model, n, dtype):
    announce("noflux newton", model, n, dtype)
    if model == O.AC:
        g, o = pair(n, O.AC, O.F_SYM, dtype, W=1.0, kappa=1.0, mob=1.0, bc=NF)
        Uold = I.uniform_field(n, -0.5, 0.5, seed=3)
    else:
        g, o = pair(n, O.CH, O.F_01, dtype, W=1.0, kappa=2.0, mob=1.0, bc=NF)
        c = I.uniform_field(n, -0.05, 0.05, seed=4, base=0.4)
        Uold = O.explicit(o, np.concatenate([c, np.zeros_like(c)]), 1.0, 0)
    Uold = rounded(Uold, dtype)
    dt = 0.5
    Ug, Uog = dev(Uold, dtype), dev(Uold, dtype)
    rtol = 1e-11 if dtype == F64 else 1e-8
    rep = S.newton_step(g, dt, Uog, Ug, S.newton_opts(rtol=rtol, lin_rtol_min=1e-8))
    assert rep.converged, rep
    big = o.ndof > 2000  # dense LU for the small cases, FP64 GMRES at 1e-13 beyond
    Uo, conv, _, _ = O.newton_be(o, dt, Uold, rtol=1e-13 if not big else 1e-11, maxit=30,
                                 solver=1 if big else 0, lin_rtol=1e-13)
    assert conv
    assert rel_l2(host(Ug), Uo) < (1e-9 if dtype == F64 else 1e-5)
    if model == O.CH:  # the lumped mass sum_a m_a c_a is conserved
        N = o.nnodes
        m0 = O.total_mass(o, Uold[:N])
        assert abs(O.total_mass(o, host(Ug)[:N]) - m0) < (1e-10 if dtype == F64 else 1e-4) * abs(m0)


@pytest.mark.parametrize("dtype", [F64, F32])
@pytest.mark.parametrize("model,n", [(O.AC, (20, 17)), (O.CH, (16, 13)), (O.CH, (5, 6, 7)),
                                     (O.AC, (6, 5, 4))])
def test_vjp_residual_noflux(model, n, dtype):
    announce("noflux vjp residual", model, n, dtype)
    g, o = pair(n, model, O.F_01, dtype, W=1.2, kappa=0.8, mob=1.3, bc=NF)
    U = rounded(np.random.default_rng(2).uniform(0.2, 0.8, o.ndof), dtype)
    w = rounded(np.random.default_rng(3).standard_normal(o.ndof), dtype)
    Ub = torch.zeros(o.ndof, dtype=dtype, device="cuda")
    tb = torch.zeros(3, dtype=F64, device="cuda")
    S.vjp(g, A.VJP_RESIDUAL, 1.0, dev(U, dtype), dev(w, dtype), Ub, tb)
    tol = 1e-11 if dtype == F64 else 1e-5
    assert rel_l2(host(Ub), O.jvp_t(o, 0.0, U, w)) < tol
    np.testing.assert_allclose(host(tb), O.dr_dtheta(o, U, w), rtol=tol * 10)


@pytest.mark.parametrize("dtype", [F64, F32])
@pytest.mark.parametrize("model,n", [(O.AC, (24, 19)), (O.CH, (18, 15)), (O.AC, (7, 6, 5)),
                                     (O.CH, (6, 5, 4)), (O.CH, (2, 3))])
def test_vjp_explicit_step_noflux(model, n, dtype):
    announce("noflux vjp explicit", model, n, dtype)
    g, o = pair(n, model, O.F_01 if model == O.CH else O.F_SYM, dtype, W=1.2, kappa=0.8, mob=1.3,
                bc=NF)
    N = o.nnodes
    U = rounded(I.uniform_field(n, -0.3, 0.3, seed=5, base=0.5 if model == O.CH else 0.0), dtype)
    if model == O.CH:
        U = np.concatenate([U, np.zeros(N)])
    vb = rounded(np.random.default_rng(6).standard_normal(N), dtype)
    dt = 0.05
    Ub = torch.zeros(o.ndof if model == O.AC else N, dtype=dtype, device="cuda")
    tb = torch.zeros(3, dtype=F64, device="cuda")
    S.vjp(g, A.VJP_EXPLICIT_STEP, dt, dev(U, dtype), dev(vb, dtype), Ub, tb)
    tref, uref = O.explicit_adjoint(o, dt, 1, U, vb)
    tol = 1e-11 if dtype == F64 else 1e-5
    assert rel_l2(host(Ub)[:N], uref) < tol
    np.testing.assert_allclose(host(tb), tref, rtol=tol * 100, atol=1e-12 * np.abs(tref).max())


@pytest.mark.parametrize("model,n", [(O.AC, (6, 5)), (O.CH, (5, 4)), (O.CH, (3, 3, 4))])
def test_vjp_newton_step_noflux(model, n):
    announce("noflux vjp newton", model, n)
    g, o = pair(n, model, O.F_01, F64, W=1.0, kappa=2.0, mob=1.0, bc=NF)
    if model == O.CH:
        c = I.uniform_field(n, -0.1, 0.1, seed=7, base=0.4)
        Uold = O.explicit(o, np.concatenate([c, np.zeros_like(c)]), 1.0, 0)
    else:
        Uold = I.uniform_field(n, 0.2, 0.8, seed=7)
    dt = 0.5
    U, conv, _, _ = O.newton_be(o, dt, Uold, rtol=1e-14, maxit=30, solver=0)
    assert conv
    w = np.random.default_rng(8).standard_normal(o.ndof)
    Ub = torch.zeros(o.ndof, dtype=F64, device="cuda")
    tb = torch.zeros(3, dtype=F64, device="cuda")
    S.vjp(g, A.VJP_NEWTON_STEP, dt, dev(U, F64), dev(w, F64), Ub, tb)
    tref, uref = O.newton_adjoint(o, dt, U, w, solver=0)
    assert rel_l2(host(Ub), uref) < 1e-9
    np.testing.assert_allclose(host(tb), tref, rtol=1e-8)
