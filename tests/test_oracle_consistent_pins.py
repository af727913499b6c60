"""Pins of the oracle's consistent-mass implicit path (every term of the weak
form Gauss-integrated, so the time term and the Cahn-Hilliard mu-row carry
M_ab = int phi_a phi_b instead of the row-sum lumped mass).

Independent references: the closed-form Q1 consistent-mass stencil
(tests/golden/q1_stencils.txt), the row sums of that stencil (the lumped mass),
the Fourier symbols of the backward-Euler step of the linear Allen-Cahn and
Cahn-Hilliard equations, conservation of sum m c, central differences of the
Newton-step adjoint, and GMRES against dense LU.
"""
import numpy as np
import pytest

import oracle as O
from tests import stencils as S
from tests.test_oracle_pins import _mode, _rel, _symbols

rng = np.random.default_rng(77)


@pytest.mark.parametrize("n,h", [((5, 6), 1.0), ((4, 3), 0.41), ((3, 4, 5), 1.0), ((4, 4, 3), 0.7)])
def test_time_term_is_the_consistent_mass_stencil(orc, n, h):
    """With zero mobility the Jacobian is inv_dt M; M is the closed-form stencil."""
    p = O.Problem(n=n, model=O.AC, fe=O.F_SYM, W=1.3, kappa=0.7, mob=0.0, h=h, mass=O.CONSISTENT)
    v = rng.standard_normal(p.nnodes)
    Jv = O.jvp(p, 2.5, np.zeros(p.nnodes), v)
    name = "mass2d" if len(n) == 2 else "mass3d"
    assert _rel(Jv, 2.5 * S.apply(name, v, n, h)) < 1e-13


@pytest.mark.parametrize("n,h", [((6, 5), 0.8), ((4, 5, 3), 1.1)])
def test_mu_row_is_the_consistent_mass(orc, n, h):
    """Cahn-Hilliard r_mu = M mu - [N(c) + kappa K c]; at c = 0 with f_01
    (f'(0) = 0) it is M mu."""
    p = O.Problem(n=n, model=O.CH, fe=O.F_01, W=1.0, kappa=1.5, mob=1.0, h=h, mass=O.CONSISTENT)
    mu = rng.standard_normal(p.nnodes)
    r = O.residual(p, np.concatenate([np.zeros(p.nnodes), mu]))
    name = "mass2d" if len(n) == 2 else "mass3d"
    assert _rel(r[p.nnodes:], S.apply(name, mu, n, h)) < 1e-13


@pytest.mark.parametrize("n", [(5, 6), (4, 3, 5)])
def test_noflux_rows_sum_to_the_lumped_mass(orc, n):
    """Row sums of the consistent mass are the lumped mass, boundary rows included."""
    p = O.Problem(n=n, model=O.AC, fe=O.F_SYM, W=1.0, kappa=1.0, mob=0.0, h=0.6, bc=O.NOFLUX,
                  mass=O.CONSISTENT)
    Jv = O.jvp(p, 1.0, np.zeros(p.nnodes), np.ones(p.nnodes))
    assert _rel(Jv, O.lumped_mass(p)) < 1e-14


@pytest.mark.parametrize("n,k", [((8, 6), (3, 1)), ((6, 6, 4), (1, 2, 1))])
def test_backward_euler_modes(orc, n, k):
    """Linear Allen-Cahn (f = 0): a mode is damped by lm / (lm + dt L kappa lk);
    linear Cahn-Hilliard (W = 0): by lm^2 / (lm^2 + dt M kappa lk^2), with lk, lm
    the stiffness and consistent-mass symbols (lumped: lm -> 1)."""
    h, dt = 0.9, 0.7
    th, lk, lm = _symbols(n, k, h)
    mode = _mode(n, th, h)
    p = O.Problem(n=n, model=O.AC, fe=O.F_SYM, W=0.0, kappa=1.5, mob=0.9, h=h, mass=O.CONSISTENT)
    U, conv, _, _ = O.newton_be(p, dt, mode, solver=0)
    assert conv
    assert _rel(U, mode * lm / (lm + dt * p.mob * p.kappa * lk)) < 1e-12
    Uc = U
    q = O.Problem(n=n, model=O.CH, fe=O.F_01, W=0.0, kappa=1.2, mob=0.8, h=h, mass=O.CONSISTENT)
    U0 = np.concatenate([mode, np.zeros(q.nnodes)])
    U, conv, _, _ = O.newton_be(q, dt, U0, solver=0)
    assert conv
    g = lm * lm / (lm * lm + dt * q.mob * q.kappa * lk * lk)
    assert _rel(U[: q.nnodes], g * mode) < 1e-11
    # and the lumped variant keeps its own symbol: the two differ
    pl = O.Problem(**{**p.__dict__, "mass": O.LUMPED})
    Ul, conv, _, _ = O.newton_be(pl, dt, mode, solver=0)
    assert _rel(Ul, mode / (1 + dt * p.mob * p.kappa * lk)) < 1e-12
    assert _rel(Ul, Uc) > 1e-3


def test_cahn_hilliard_step_conserves_mass(orc):
    p = O.Problem(n=(7, 6), model=O.CH, fe=O.F_01, W=1.0, kappa=1.5, mob=1.0, h=1.3, bc=O.NOFLUX,
                  mass=O.CONSISTENT)
    c = 0.45 + 0.05 * rng.standard_normal(p.nnodes)
    U0 = np.concatenate([c, np.zeros(p.nnodes)])
    U, conv, _, _ = O.newton_be(p, 0.3, U0, rtol=1e-13, solver=0)
    assert conv
    assert O.total_mass(p, U) == pytest.approx(O.total_mass(p, U0), rel=1e-13)


def test_explicit_path_rejects_consistent_mass(orc):
    p = O.Problem(n=(4, 4), model=O.AC, mass=O.CONSISTENT)
    with pytest.raises(ValueError):
        O.explicit(p, np.zeros(p.nnodes), 0.1, 1)


def test_newton_adjoint_vs_fd(orc):
    p = O.Problem(n=(4, 5), model=O.CH, fe=O.F_01, W=1.0, kappa=2.0, mob=1.0, mass=O.CONSISTENT)
    c = 0.4 + rng.uniform(-0.1, 0.1, p.nnodes)
    Uold = np.concatenate([c, np.zeros_like(c)])
    dt = 0.5
    w = rng.standard_normal(p.ndof)

    def obj(q, uold):
        U, conv, _, _ = O.newton_be(q, dt, uold, rtol=1e-14, maxit=30, solver=0)
        return w @ U

    U, conv, _, _ = O.newton_be(p, dt, Uold, rtol=1e-14, maxit=30, solver=0)
    tb, ub = O.newton_adjoint(p, dt, U, w, solver=0)
    for kk, name in enumerate(["mob", "kappa", "W"]):
        eps = 1e-6
        hp = O.Problem(**{**p.__dict__, name: getattr(p, name) + eps})
        hm = O.Problem(**{**p.__dict__, name: getattr(p, name) - eps})
        assert tb[kk] == pytest.approx((obj(hp, Uold) - obj(hm, Uold)) / (2 * eps), rel=1e-6)
    for i in (0, 6, 11):
        e = np.zeros(p.ndof)
        e[i] = 1e-6
        assert ub[i] == pytest.approx((obj(p, Uold + e) - obj(p, Uold - e)) / 2e-6, rel=1e-6, abs=1e-10)


def test_gmres_matches_dense(orc):
    p = O.Problem(n=(5, 4, 3), model=O.CH, fe=O.F_01, W=1.0, kappa=2.0, mob=1.0, mass=O.CONSISTENT)
    U = 0.4 + 0.05 * rng.standard_normal(p.ndof)
    b = rng.standard_normal(p.ndof)
    for tr in (False, True):
        x0 = O.linear_solve(p, 2.0, U, b, transpose=tr, solver=0)
        x1 = O.linear_solve(p, 2.0, U, b, transpose=tr, solver=1, lin_rtol=1e-13)
        assert _rel(x1, x0) < 1e-10
