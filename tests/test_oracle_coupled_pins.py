"""Pins of the coupled Allen-Cahn / Cahn-Hilliard oracle (Eq. 7, Supp. Note 3)
against what the mathematics fixes: properties of the interpolation function,
derivatives of the free energies, the rows of the residual as gradients of the
discrete energy, a closed-form Fourier-mode step, and conservation."""
import numpy as np
import pytest

import oracle as O

BCS = [O.PERIODIC, O.NOFLUX]


def test_interpolation_function_is_a_monotone_step_from_0_to_1():
    """h rises monotonically from 0 to 1 with zero slope at both ends (Sec. 2.1)."""
    assert O.cp_poly("h", 0.0) == 0.0 and O.cp_poly("h", 1.0) == pytest.approx(1.0, abs=1e-15)
    assert O.cp_poly("dh", 0.0) == 0.0 and O.cp_poly("dh", 1.0) == pytest.approx(0.0, abs=1e-13)
    assert O.cp_poly("h", 0.5) == pytest.approx(0.5, abs=1e-15)
    xs = np.linspace(0.0, 1.0, 101)
    assert all(O.cp_poly("dh", x) >= 0.0 for x in xs)
    hs = [O.cp_poly("h", x) for x in xs]
    assert all(b >= a for a, b in zip(hs, hs[1:]))


@pytest.mark.parametrize("f", ["fa", "fb", "h"])
def test_polynomial_derivatives(f):
    """f_a', f_b', h' are the derivatives of f_a, f_b, h (central differences)."""
    for x in np.linspace(-0.3, 1.3, 17):
        e = 1e-5
        fd = (O.cp_poly(f, x + e) - O.cp_poly(f, x - e)) / (2 * e)
        assert O.cp_poly("d" + f, x) == pytest.approx(fd, rel=1e-8, abs=1e-8)


def _rand_state(p, seed):
    rng = np.random.default_rng(seed)
    N = p.nnodes
    return np.concatenate([rng.uniform(0.0, 1.0, N), rng.uniform(-1, 1, N), rng.uniform(0.0, 1.0, N)])


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("n", [(4, 3), (3, 2, 3)])
def test_mu_and_eta_rows_are_energy_gradients(n, bc):
    """With mu = 0 the mu-row is -dE_h/dc and the eta-row is M_eta dE_h/d eta:
    both rows are the first variation of the discrete energy (Eq. 7)."""
    p = O.CoupledProblem(n=n, bc=bc, h=0.7, Mc=1.3, Meta=2.5, kappa=0.4)
    N = p.nnodes
    U = _rand_state(p, 1)
    U[N:2 * N] = 0.0
    r = O.cp_residual(p, U)
    e = 1e-6
    for a in range(N):
        for plane, row, scale in ((0, N, -1.0), (2 * N, 2 * N, 1.0 / p.Meta)):
            Up, Um = U.copy(), U.copy()
            Up[plane + a] += e
            Um[plane + a] -= e
            fd = (O.cp_energy(p, Up) - O.cp_energy(p, Um)) / (2 * e)
            assert scale * r[row + a] == pytest.approx(fd, rel=1e-6, abs=1e-8)


def test_c_row_closed_form_mode():
    """r_c = M_c K mu: on a periodic 2-D grid a Fourier mode of mu is an eigenvector
    of the Q1 stiffness with eigenvalue (8 - 2cx - 2cy - 4cx cy)/3 (h-free in 2-D)."""
    n, k = (12, 10), (2, 3)
    p = O.CoupledProblem(n=n, h=1.7, Mc=0.8)
    th = [2 * np.pi * k[i] / n[i] for i in range(2)]
    X, Y = np.meshgrid(np.arange(n[0]), np.arange(n[1]))
    mode = np.cos(th[0] * X + th[1] * Y).ravel()
    lam = (8 - 2 * np.cos(th[0]) - 2 * np.cos(th[1]) - 4 * np.cos(th[0]) * np.cos(th[1])) / 3
    N = p.nnodes
    U = np.concatenate([np.full(N, 0.3), mode, np.zeros(N)])
    r = O.cp_residual(p, U)
    np.testing.assert_allclose(r[:N], p.Mc * lam * mode, atol=1e-12)


@pytest.mark.parametrize("bc", BCS)
def test_uniform_state(bc):
    """Uniform c, eta: the quadrature of constants gives the lumped mass, so
    mu = f_a'(c)(1 - h) + f_b'(c) h and r_eta = M_eta m (f_b - f_a)(c) h'(eta)."""
    p = O.CoupledProblem(n=(5, 4), bc=bc, h=0.9, Meta=3.0)
    N = p.nnodes
    c, eta = 0.37, 0.61
    U = np.concatenate([np.full(N, c), np.zeros(N), np.full(N, eta)])
    m = O.cp_lumped_mass(p)
    r = O.cp_residual(p, U)
    h, dh = O.cp_poly("h", eta), O.cp_poly("dh", eta)
    mu = O.cp_poly("dfa", c) * (1 - h) + O.cp_poly("dfb", c) * h
    np.testing.assert_allclose(r[:N], 0.0, atol=1e-13)
    np.testing.assert_allclose(r[N:2 * N], -m * mu, rtol=1e-13)
    np.testing.assert_allclose(r[2 * N:], p.Meta * m * (O.cp_poly("fb", c) - O.cp_poly("fa", c)) * dh,
                               rtol=1e-12)


def test_explicit_mode_decay_closed_form():
    """eta = 1 everywhere: mu = f_b'(c) = 10c - 5.9746 is linear, so a composition mode
    decays by 1 - dt M_c lam_K 10 s_M / m per step, s_M = (2 + cx)(2 + cy)/9 the
    Gauss-quadrature (consistent) mass symbol relative to the lumped mass m = h^2."""
    n, k, h, dt = (16, 12), (3, 2), 1.3, 1e-3
    p = O.CoupledProblem(n=n, h=h, Mc=0.9, Meta=5.0, kappa=0.3)
    th = [2 * np.pi * k[i] / n[i] for i in range(2)]
    X, Y = np.meshgrid(np.arange(n[0]), np.arange(n[1]))
    mode = np.cos(th[0] * X + th[1] * Y).ravel()
    N = p.nnodes
    cbar, A = 0.4, 0.01
    U0 = np.concatenate([cbar + A * mode, np.zeros(N), np.ones(N)])
    U1 = O.cp_explicit(p, U0, dt, 1)
    lam = (8 - 2 * np.cos(th[0]) - 2 * np.cos(th[1]) - 4 * np.cos(th[0]) * np.cos(th[1])) / 3
    sM = (2 + np.cos(th[0])) * (2 + np.cos(th[1])) / 9
    A1 = A * (1 - dt * p.Mc * lam * 10.0 * sM / h ** 2)
    np.testing.assert_allclose(U1[:N], cbar + A1 * mode, atol=1e-14)
    np.testing.assert_allclose(U1[2 * N:], 1.0, atol=1e-14)  # eta = 1 is an equilibrium
    # the final mu plane is f_b' of the new composition through the same quadrature
    np.testing.assert_allclose(U1[N:2 * N], 10.0 * (cbar + A1 * sM * mode) - 5.9746, atol=1e-12)


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("n", [(9, 7), (4, 5, 3)])
def test_explicit_conserves_composition_and_decreases_energy(n, bc):
    """Forward Euler with a small step: sum m c is conserved exactly (rows of K sum
    to zero) and the discrete energy decreases (gradient flow)."""
    p = O.CoupledProblem(n=n, bc=bc, h=1.0, Mc=1.0, Meta=1.0, kappa=0.3)
    rng = np.random.default_rng(4)
    N = p.nnodes
    U = np.concatenate([0.5 + 0.05 * rng.standard_normal(N), np.zeros(N),
                        0.5 + 0.2 * rng.standard_normal(N)])
    m0, e0 = O.cp_total_mass(p, U), O.cp_energy(p, U)
    V = O.cp_explicit(p, U, 2e-3, 20)
    assert O.cp_total_mass(p, V) == pytest.approx(m0, rel=1e-13)
    assert O.cp_energy(p, V) < e0


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("n", [(4, 3), (2, 3, 2)])
def test_coupled_jvp_is_the_residual_derivative(n, bc):
    """Brute force: J v equals the central difference of the backward-Euler residual."""
    p = O.CoupledProblem(n=n, bc=bc, h=0.8, Mc=1.2, Meta=2.0, kappa=0.4)
    U = _rand_state(p, 6)
    Uold = _rand_state(p, 7)
    v = np.random.default_rng(8).standard_normal(p.ndof)
    dt, e = 0.3, 1e-6
    fd = (O.cp_be_residual(p, dt, Uold, U + e * v) - O.cp_be_residual(p, dt, Uold, U - e * v)) / (2 * e)
    np.testing.assert_allclose(O.cp_jvp(p, 1.0 / dt, U, v), fd, rtol=1e-7, atol=1e-7)


def test_coupled_jacobian_mixed_blocks_are_transposes():
    """d r_mu / d eta = -(1/M_eta) (d r_eta / d c)^T: both are the mixed second
    derivative of the discrete energy."""
    p = O.CoupledProblem(n=(5, 4), bc=O.NOFLUX, h=0.9, Meta=3.0)
    N = p.nnodes
    U = _rand_state(p, 9)
    rng = np.random.default_rng(10)
    a, b = rng.standard_normal(N), rng.standard_normal(N)
    z = np.zeros(N)
    # w_mu^T (dr_mu/deta) v_eta  and  w_eta^T (dr_eta/dc) v_c  with w, v swapped
    left = a @ O.cp_jvp(p, 0.0, U, np.concatenate([z, z, b]))[N:2 * N]
    right = b @ O.cp_jvp(p, 0.0, U, np.concatenate([a, z, z]))[2 * N:]
    assert left == pytest.approx(-right / p.Meta, rel=1e-12)


def test_coupled_backward_euler_mode_closed_form():
    """eta = 1: the backward-Euler step damps a composition mode by
    1 / (1 + dt M_c lam_K 10 s_M / m) (the explicit factor's implicit counterpart)."""
    n, k, h, dt = (8, 6), (1, 2), 1.1, 0.05
    p = O.CoupledProblem(n=n, h=h, Mc=0.7, Meta=2.0, kappa=0.3)
    th = [2 * np.pi * k[i] / n[i] for i in range(2)]
    X, Y = np.meshgrid(np.arange(n[0]), np.arange(n[1]))
    mode = np.cos(th[0] * X + th[1] * Y).ravel()
    N = p.nnodes
    cbar, A = 0.3, 0.02
    Uold = np.concatenate([cbar + A * mode, np.zeros(N), np.ones(N)])
    U, conv, _ = O.cp_newton_be(p, dt, Uold, rtol=1e-13)
    assert conv
    lam = (8 - 2 * np.cos(th[0]) - 2 * np.cos(th[1]) - 4 * np.cos(th[0]) * np.cos(th[1])) / 3
    sM = (2 + np.cos(th[0])) * (2 + np.cos(th[1])) / 9
    A1 = A / (1 + dt * p.Mc * lam * 10.0 * sM / h ** 2)
    np.testing.assert_allclose(U[:N], cbar + A1 * mode, atol=1e-12)
    np.testing.assert_allclose(U[2 * N:], 1.0, atol=1e-12)


@pytest.mark.parametrize("bc", BCS)
def test_coupled_newton_root_conserves_composition(bc):
    p = O.CoupledProblem(n=(6, 5), bc=bc, h=1.0, Mc=1.0, Meta=150.0, kappa=0.3)
    rng = np.random.default_rng(0)
    N = p.nnodes
    eta = rng.uniform(0, 1, N)
    c = 0.04 + 0.12 * eta + 0.005 * rng.standard_normal(N)
    Uold = O.cp_explicit(p, np.concatenate([c, np.zeros(N), eta]), 1e-3, 0)
    U, conv, its = O.cp_newton_be(p, 0.01, Uold, rtol=1e-12)
    assert conv and its <= 8
    assert np.abs(O.cp_be_residual(p, 0.01, Uold, U)).max() < 1e-11
    assert O.cp_total_mass(p, U) == pytest.approx(O.cp_total_mass(p, Uold), rel=1e-13)
    assert O.cp_energy(p, U) < O.cp_energy(p, Uold)
