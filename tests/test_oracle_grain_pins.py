"""Pins of the multi-order-parameter (grain-growth) oracle against facts that do
not come from it: the single-order-parameter limit (the already-pinned Allen-Cahn
oracle with f = (eta^2 - 1)^2/4), the residual as the gradient of the discrete
energy (central differences), the closed-form two-grain boundary profile for
gamma = 3/2, stationary single-grain states, permutation symmetry, and energy
decay of small explicit steps.
"""
import numpy as np
import pytest

import oracle as O

rng = np.random.default_rng(2024)


def _rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


@pytest.mark.parametrize("n,bc", [((7, 6), O.PERIODIC), ((5, 4, 6), O.NOFLUX)])
def test_single_grain_is_allen_cahn(orc, n, bc):
    """p = 1: f = eta^4/4 - eta^2/2 + 1/4 = (eta^2 - 1)^2/4, the Allen-Cahn f_sym at W = 1."""
    g = O.GrainProblem(n, p=1, bc=bc, h=0.8, L=1.3, kappa=0.7, gamma=1.5)
    a = O.Problem(n=n, model=O.AC, fe=O.F_SYM, bc=bc, h=0.8, W=1.0, kappa=0.7, mob=1.3)
    U = rng.uniform(-1, 1, g.nnodes)
    assert _rel(O.gg_residual(g, U), O.residual(a, U)) < 1e-14
    assert O.gg_energy(g, U) == pytest.approx(O.energy(a, U), rel=1e-14)
    assert _rel(O.gg_explicit(g, U, 0.03, 4), O.explicit(a, U, 0.03, 4)) < 1e-14


def test_local_energy_gradient(orc):
    g = O.GrainProblem((2, 2), p=5, gamma=1.3)
    for _ in range(4):
        eta = rng.uniform(-1, 1.2, 5)
        df = O.gg_df(g, eta)
        for i in range(5):
            e = np.zeros(5)
            e[i] = 1e-6
            fd = (O.gg_f(g, eta + e) - O.gg_f(g, eta - e)) / 2e-6
            assert df[i] == pytest.approx(fd, rel=1e-7, abs=1e-9)


@pytest.mark.parametrize("n,bc,p", [((6, 5), O.PERIODIC, 3), ((5, 6), O.NOFLUX, 4), ((4, 3, 4), O.NOFLUX, 2)])
def test_residual_is_energy_gradient(orc, n, bc, p):
    """r_i / L = dE_h / d eta_i (the weak form is the first variation of F)."""
    g = O.GrainProblem(n, p=p, bc=bc, h=0.9, L=1.7, kappa=0.8, gamma=1.5)
    U = rng.uniform(0, 1, g.ndof)
    r = O.gg_residual(g, U) / g.L
    for k in rng.choice(g.ndof, 8, replace=False):
        e = np.zeros(g.ndof)
        e[k] = 1e-6
        fd = (O.gg_energy(g, U + e) - O.gg_energy(g, U - e)) / 2e-6
        assert r[k] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def _two_grain_error(h, kappa=1.0, X=10.0):
    nx = int(round(2 * X / h)) + 1
    x = -X + h * np.arange(nx)
    t = np.tanh(x / np.sqrt(2 * kappa))
    e1, e2 = 0.5 * (1 - t), 0.5 * (1 + t)
    g = O.GrainProblem((nx, 2), p=2, bc=O.NOFLUX, h=h, L=1.0, kappa=kappa, gamma=1.5)
    U = np.concatenate([np.tile(e1, 2), np.tile(e2, 2)])
    # relax towards the discrete equilibrium with stable explicit steps
    m = O.gg_lumped_mass(g)
    dt = 0.2 * h * h / kappa
    V = U.copy()
    for _ in range(6):
        V = O.gg_explicit(g, V, dt, 400)
    return np.max(np.abs(V - U)), np.max(np.abs(O.gg_residual(g, V) / np.tile(m, 2)))


def test_two_grain_boundary_profile(orc):
    """gamma = 3/2: the flat boundary between two grains is exactly
    eta_1 = (1 - tanh(x / sqrt(2 kappa)))/2, eta_2 = 1 - eta_1 (substitute into
    kappa eta'' = df/deta); the discrete equilibrium converges to it at second order."""
    errs = []
    for h in (0.5, 0.25):
        e, res = _two_grain_error(h)
        assert res < 1e-4 * (1 / h)
        errs.append(e)
    assert errs[0] / errs[1] > 3.3, errs
    assert errs[1] < 5e-3


def test_single_grain_states_are_stationary(orc):
    g = O.GrainProblem((5, 4), p=4, h=1.0)
    N = g.nnodes
    for i in range(4):
        U = np.zeros(g.ndof)
        U[i * N:(i + 1) * N] = 1.0
        assert np.max(np.abs(O.gg_residual(g, U))) < 1e-14
        assert O.gg_energy(g, U) == pytest.approx(0.0, abs=1e-14)
    assert np.max(np.abs(O.gg_residual(g, np.zeros(g.ndof)))) < 1e-14


def test_permutation_symmetry(orc):
    g = O.GrainProblem((6, 5), p=4, h=0.7, gamma=1.2)
    N = g.nnodes
    U = rng.uniform(0, 1, g.ndof).reshape(4, N)
    perm = [2, 0, 3, 1]
    r = O.gg_residual(g, U.ravel()).reshape(4, N)
    rp = O.gg_residual(g, U[perm].ravel()).reshape(4, N)
    assert _rel(rp, r[perm]) < 1e-14
    assert O.gg_energy(g, U[perm].ravel()) == pytest.approx(O.gg_energy(g, U.ravel()), rel=1e-14)


def test_explicit_steps_decrease_energy(orc):
    g = O.GrainProblem((16, 12), p=5, h=1.0, kappa=1.0, gamma=1.5)
    U = rng.uniform(0, 1, g.ndof)
    E = [O.gg_energy(g, U)]
    for _ in range(10):
        U = O.gg_explicit(g, U, 0.05, 5)
        E.append(O.gg_energy(g, U))
    assert all(b < a for a, b in zip(E, E[1:]))


@pytest.mark.parametrize("n,bc,p", [((5, 4), O.PERIODIC, 3), ((4, 5), O.NOFLUX, 2), ((3, 4, 3), O.NOFLUX, 2)])
def test_jvp_is_derivative_of_residual(orc, n, bc, p):
    """The Jacobian product against central differences of the backward-Euler
    residual, and its symmetry (the Hessian of the discrete energy plus a mass)."""
    g = O.GrainProblem(n, p=p, bc=bc, h=0.8, L=1.3, kappa=0.9, gamma=1.5)
    U = rng.uniform(0, 1, g.ndof)
    Uold = rng.uniform(0, 1, g.ndof)
    v = rng.standard_normal(g.ndof)
    w = rng.standard_normal(g.ndof)
    dt = 0.4
    eps = 1e-6
    fd = (O.gg_be_residual(g, dt, Uold, U + eps * v) - O.gg_be_residual(g, dt, Uold, U - eps * v)) / (2 * eps)
    Jv = O.gg_jvp(g, 1 / dt, U, v)
    assert _rel(Jv, fd) < 1e-8
    assert w @ Jv == pytest.approx(v @ O.gg_jvp(g, 1 / dt, U, w), rel=1e-12)


def test_backward_euler_single_grain_is_allen_cahn(orc):
    g = O.GrainProblem((6, 5), p=1, h=1.0, L=1.1, kappa=0.8)
    a = O.Problem(n=(6, 5), model=O.AC, fe=O.F_SYM, W=1.0, kappa=0.8, mob=1.1)
    Uold = rng.uniform(-0.8, 0.8, g.nnodes)
    U1, ok1, _ = O.gg_newton_be(g, 0.5, Uold)
    U2, ok2, _, _ = O.newton_be(a, 0.5, Uold, rtol=1e-12, solver=0)
    assert ok1 and ok2
    assert _rel(U1, U2) < 1e-12


def test_backward_euler_step_solves_the_residual(orc):
    g = O.GrainProblem((5, 6), p=3, bc=O.NOFLUX, h=1.0, L=1.0, kappa=1.0)
    Uold = rng.uniform(0, 1, g.ndof)
    U, ok, its = O.gg_newton_be(g, 1.0, Uold, rtol=1e-13)
    assert ok and its >= 2
    R = O.gg_be_residual(g, 1.0, Uold, U)
    assert np.max(np.abs(R)) < 1e-12 * max(1.0, np.max(np.abs(O.gg_residual(g, Uold))))
    assert O.gg_energy(g, U) < O.gg_energy(g, Uold)
