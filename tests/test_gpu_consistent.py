"""Consistent-mass implicit path (every term of the weak form Gauss-integrated:
the backward-Euler time term and the Cahn-Hilliard mu-row carry the Q1 mass
matrix instead of the lumped one): HIP vs the FP64 oracle, through the C ABI."""
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


def pair_cm(n, model, fe, dtype, bc=O.PERIODIC, **kw):
    g, o = pair(n, model, fe, dtype, bc=bc, **kw)
    g.mass = A.MASS_CONSISTENT
    o.mass = O.CONSISTENT
    return g, o


CASES = [(O.AC, (14, 11), O.PERIODIC), (O.CH, (12, 9), O.NOFLUX), (O.CH, (6, 5, 7), O.PERIODIC),
         (O.AC, (5, 6, 4), O.NOFLUX), (O.CH, (70, 3), O.PERIODIC)]


@pytest.mark.parametrize("dtype", [F64, F32])
@pytest.mark.parametrize("model,n,bc", CASES)
def test_residual_and_jvp(model, n, bc, dtype):
    announce("consistent residual/jvp", model, n, bc, dtype)
    g, o = pair_cm(n, model, O.F_01, dtype, bc=bc, W=1.1, kappa=0.9, mob=1.3, h=0.7)
    rng = np.random.default_rng(sum(n))
    U = rounded(rng.uniform(0.2, 0.8, o.ndof), dtype)
    v = rounded(rng.standard_normal(o.ndof), dtype)
    tol = 1e-12 if dtype == F64 else 2e-6
    r = host(S.residual(g, dev(U, dtype)))
    ref = O.residual(o, U)
    assert np.abs(r - ref).max() <= tol * np.abs(ref).max()
    Jv = host(S.jvp(g, 3.0, dev(U, dtype), dev(v, dtype)))
    ref = O.jvp(o, 3.0, U, v)
    assert np.abs(Jv - ref).max() <= tol * np.abs(ref).max()


def _ch_state(o, base, amp, seed):
    c = I.uniform_field(o.n, -amp, amp, seed=seed, base=base)
    lo = O.Problem(**{**o.__dict__, "mass": O.LUMPED})
    return O.explicit(lo, np.concatenate([c, np.zeros_like(c)]), 1.0, 0)


@pytest.mark.parametrize("dtype", [F64, F32])
@pytest.mark.parametrize("model,n,bc", [(O.AC, (12, 10), O.NOFLUX), (O.CH, (9, 8), O.PERIODIC),
                                        (O.CH, (6, 5, 4), O.NOFLUX), (O.AC, (5, 6, 4), O.PERIODIC)])
def test_newton_step_matches_oracle(model, n, bc, dtype):
    announce("consistent newton", model, n, bc, dtype)
    if model == O.AC:
        g, o = pair_cm(n, O.AC, O.F_SYM, dtype, bc=bc, W=1.0, kappa=1.0, mob=1.0)
        Uold = I.uniform_field(n, -0.5, 0.5, seed=3)
    else:
        g, o = pair_cm(n, O.CH, O.F_01, dtype, bc=bc, W=1.0, kappa=2.0, mob=1.0)
        Uold = _ch_state(o, 0.4, 0.05, 4)
    dt = 0.5
    Uold = rounded(Uold, dtype)
    Ug, Uog = dev(Uold, dtype), dev(Uold, dtype)
    rtol = 1e-11 if dtype == F64 else 1e-8
    rep = S.newton_step(g, dt, Uog, Ug, S.newton_opts(rtol=rtol, lin_rtol_min=1e-8))
    assert rep.converged, rep
    Uo, conv, its, _ = O.newton_be(o, dt, Uold, rtol=1e-13, maxit=30, solver=0)
    assert conv
    tol = 1e-9 if dtype == F64 else 1e-5
    assert rel_l2(host(Ug), Uo) < tol
    if model == O.CH:
        assert O.total_mass(o, host(Ug)) == pytest.approx(O.total_mass(o, Uold),
                                                         rel=1e-11 if dtype == F64 else 1e-5)


def test_linear_mode_closed_form():
    """f == 0 Allen-Cahn with the consistent mass: a Fourier mode is damped by
    lm / (lm + dt L kappa lk) (stiffness and mass symbols of the Q1 stencils)."""
    n, k, h, dt = (16, 12), (3, 2), 1.0, 0.7
    th = [2 * np.pi * k[a] / n[a] for a in range(2)]
    c0, c1 = np.cos(th[0]), np.cos(th[1])
    lk = (8 - 2 * c0 - 2 * c1 - 4 * c0 * c1) / 3
    lm = (2 + c0) * (2 + c1) / 9
    X, Y = np.meshgrid(np.arange(n[0]), np.arange(n[1]))
    mode = np.cos(th[0] * X + th[1] * Y).ravel()
    g = S.Problem(n=n, model=A.ALLEN_CAHN, fe=A.F_SYM, dtype=F64, W=0.0, kappa=1.5, mobility=0.9,
                  mass=A.MASS_CONSISTENT)
    Uo, U = dev(mode, F64), dev(mode, F64)
    rep = S.newton_step(g, dt, Uo, U, S.newton_opts(rtol=1e-13, lin_rtol_min=1e-12, lin_rtol_max=1e-12))
    assert rep.converged
    assert rel_l2(host(U), mode * lm / (lm + dt * 0.9 * 1.5 * lk)) < 1e-11


@pytest.mark.parametrize("dtype", [F64, F32])
@pytest.mark.parametrize("model,n", [(O.AC, (20, 17)), (O.CH, (16, 13)), (O.CH, (5, 6, 7))])
def test_vjp_residual(model, n, dtype):
    announce("consistent vjp residual", model, n, dtype)
    g, o = pair_cm(n, model, O.F_01, dtype, W=1.2, kappa=0.8, mob=1.3)
    U = rounded(np.random.default_rng(2).uniform(0.2, 0.8, o.ndof), dtype)
    w = rounded(np.random.default_rng(3).standard_normal(o.ndof), dtype)
    Ub = torch.zeros(o.ndof, dtype=dtype, device="cuda")
    tb = torch.zeros(3, dtype=F64, device="cuda")
    S.vjp(g, A.VJP_RESIDUAL, 1.0, dev(U, dtype), dev(w, dtype), Ub, tb)
    tol = 1e-11 if dtype == F64 else 1e-5
    assert rel_l2(host(Ub), O.jvp_t(o, 0.0, U, w)) < tol
    np.testing.assert_allclose(host(tb), O.dr_dtheta(o, U, w), rtol=tol * 10)


@pytest.mark.parametrize("model,n,bc", [(O.AC, (6, 5), O.PERIODIC), (O.CH, (5, 4), O.NOFLUX),
                                        (O.CH, (3, 3, 4), O.PERIODIC)])
def test_vjp_newton_step(model, n, bc):
    announce("consistent vjp newton", model, n, bc)
    g, o = pair_cm(n, model, O.F_01, F64, bc=bc, W=1.0, kappa=2.0, mob=1.0)
    Uold = _ch_state(o, 0.4, 0.1, 7) if model == O.CH else I.uniform_field(n, 0.2, 0.8, seed=7)
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


def test_explicit_paths_reject_consistent_mass():
    g = S.Problem(n=(16, 16), model=A.CAHN_HILLIARD, fe=A.F_01, dtype=F32, mass=A.MASS_CONSISTENT)
    U = torch.zeros(g.ndof, dtype=F32, device="cuda")
    ws = torch.empty(4 * g.ndof + 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(A.PFError) as e:
        S.step_explicit(g, U, 0.01, 1, ws)
    assert e.value.status == A.PF_EUNSUPPORTED
    Ub = torch.zeros(g.nnodes, dtype=F32, device="cuda")
    tb = torch.zeros(3, dtype=F64, device="cuda")
    with pytest.raises(A.PFError) as e:
        S.vjp(g, A.VJP_EXPLICIT_STEP, 0.01, U, Ub.clone(), Ub, tb)
    assert e.value.status == A.PF_EUNSUPPORTED


def test_paper_shape_ch512_noflux():
    """The paper's 2-D Cahn-Hilliard implicit shape with every term Gauss-integrated:
    [0, 100]^2 on 512^2 nodes, no-flux, dt = 0.05, three steps.  Each step converges,
    conserves sum m c, and stays within the time-discretisation difference of the
    lumped-mass step (the two schemes differ at O(h^2) per step)."""
    announce("consistent ch512")
    n = (512, 512)
    kw = dict(model=A.CAHN_HILLIARD, fe=A.F_01, dtype=F32, W=1.0, kappa=1.5, mobility=1.0,
              h=100.0 / 511, bc=A.NOFLUX)
    gc = S.Problem(n=n, mass=A.MASS_CONSISTENT, **kw)
    gl = S.Problem(n=n, **kw)
    c0 = I.uniform_field(n, -0.05, 0.05, seed=0, base=0.5).astype(np.float32)
    U = torch.as_tensor(np.concatenate([c0, np.zeros_like(c0)]), device="cuda")
    S.step_explicit(gl, U, 1e-30, 0)  # mu0 from c0 (lumped split-step row)
    Ul = U.clone()
    ws = S.workspace(gc, A.OP_NEWTON)
    for _ in range(3):
        Uold = U.clone()
        rep = S.newton_step(gc, 0.05, Uold, U, ws=ws)
        assert rep.converged, rep
        Ulold = Ul.clone()
        rl = S.newton_step(gl, 0.05, Ulold, Ul, ws=ws)
        assert rl.converged
    # sum m c (the second entry of the library's energy reduction) is conserved
    e = host(S.energy(gc, U))
    el = host(S.energy(gl, Ul))
    e0 = host(S.energy(gl, torch.as_tensor(np.concatenate([c0, np.zeros_like(c0)]), device="cuda")))
    assert e[1] == pytest.approx(e0[1], rel=1e-5)
    assert el[1] == pytest.approx(e0[1], rel=1e-5)
    d = rel_l2(host(U)[: gc.nnodes] - 0.5, host(Ul)[: gc.nnodes] - 0.5)
    assert 1e-6 < d < 0.2, d
