"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed-form
stencils, brute-force integrals, finite differences of the discrete energy,
Fourier multipliers, exact equilibrium profiles, conservation laws, symmetries
and closed-form adjoints.
"""
import numpy as np
import pytest

import oracle as O
from tests import stencils as S

rng = np.random.default_rng(1234)


def _rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


# ---------------------------------------------------------------- PIN1 ------
# Gradient term: with f == 0 the Allen-Cahn residual is L kappa K eta, and K is
# the closed-form Q1 stiffness stencil (Sec. 2.1 Eq. 5, weak form).
@pytest.mark.parametrize("n,h", [((6, 5), 1.0), ((7, 4), 0.37), ((4, 5, 3), 1.0), ((3, 4, 5), 0.6)])
def test_pin1_stiffness_stencil(orc, n, h):
    p = O.Problem(n=n, model=O.AC, fe=O.F_SYM, W=0.0, kappa=1.7, mob=0.8, h=h)
    eta = rng.standard_normal(p.nnodes)
    r = O.residual(p, eta)
    name = "stiff2d" if len(n) == 2 else "stiff3d"
    ref = p.mob * p.kappa * S.apply(name, eta, n, h)
    assert _rel(r, ref) < 1e-13


def test_pin1_noflux_rows_sum_to_zero(orc):
    p = O.Problem(n=(5, 6), model=O.AC, W=0.0, kappa=1.0, bc=O.NOFLUX, h=0.5)
    r = O.residual(p, np.full(p.nnodes, 3.0))
    assert np.max(np.abs(r)) < 1e-13


# ---------------------------------------------------------------- PIN2 ------
# Interpolation and scatter: the linear part of f' assembles the consistent
# mass matrix.  For f_sym, N(c) = W(N3(c) - Mc c) with N3 cubic-homogeneous,
# so Mc c = (N(2c) - 8 N(c)) / (6 W) exactly.
@pytest.mark.parametrize("n,h", [((5, 6), 1.0), ((4, 3), 0.41), ((3, 4, 5), 1.0), ((4, 4, 3), 0.7)])
def test_pin2_consistent_mass(orc, n, h):
    p = O.Problem(n=n, model=O.AC, fe=O.F_SYM, W=1.3, kappa=0.0, mob=1.0, h=h)
    c = rng.standard_normal(p.nnodes)
    mc = (O.residual(p, 2 * c) - 8 * O.residual(p, c)) / (6 * p.W)
    name = "mass2d" if len(n) == 2 else "mass3d"
    assert _rel(mc, S.apply(name, c, n, h)) < 1e-12


def _exact_quadratic_moment_2d(c, n, h):
    """int c_h^2 phi_a over a periodic Q1 grid by 4-point Gauss per axis
    (exact: the integrand is degree <= 4 per axis), written independently."""
    x, w = np.polynomial.legendre.leggauss(4)
    nx, ny = n
    C = c.reshape(ny, nx)
    out = np.zeros_like(C)
    for ey in range(ny):
        for ex in range(nx):
            xs = [ex, (ex + 1) % nx]
            ys = [ey, (ey + 1) % ny]
            for qi, xi in enumerate(x):
                for qj, yj in enumerate(x):
                    px = [(1 - xi) / 2, (1 + xi) / 2]
                    py = [(1 - yj) / 2, (1 + yj) / 2]
                    ch = sum(px[a] * py[b] * C[ys[b], xs[a]] for a in range(2) for b in range(2))
                    for a in range(2):
                        for b in range(2):
                            out[ys[b], xs[a]] += w[qi] * w[qj] * (h / 2) ** 2 * ch * ch * px[a] * py[b]
    return out.ravel()


def test_pin2b_quadratic_term_exact(orc):
    # f_01' = 2W(c - 3c^2 + 2c^3): the even part of N gives the quadratic term,
    # which 2-point Gauss integrates exactly (degree 3 per axis).
    n, h = (4, 5), 0.8
    p = O.Problem(n=n, model=O.AC, fe=O.F_01, W=0.9, kappa=0.0, mob=1.0, h=h)
    c = rng.standard_normal(p.nnodes)
    even = 0.5 * (O.residual(p, c) + O.residual(p, -c))
    ref = 2 * p.W * (-3.0) * _exact_quadratic_moment_2d(c, n, h)
    assert _rel(even, ref) < 1e-13


# ---------------------------------------------------------------- PIN3 ------
# Pointwise f' and the update: on a uniform state r = L f'(c) m, and one
# explicit step is the scalar recurrence c <- c - dt L f'(c).  The f_01
# derivative is checked against the paper's printed form 4c(c-1)(c-1/2)
# (Supplementary Note 3), the f_sym one against W(c^3 - c).
@pytest.mark.parametrize("fe", [O.F_SYM, O.F_01])
def test_pin3_uniform_state(orc, fe):
    p = O.Problem(n=(5, 4), model=O.AC, fe=fe, W=1.0, kappa=2.0, mob=0.7, h=0.5)
    cbar, dt = 0.3, 0.05
    fprime = (4 * cbar * (cbar - 1) * (cbar - 0.5)) if fe == O.F_01 else (cbar ** 3 - cbar)
    r = O.residual(p, np.full(p.nnodes, cbar))
    np.testing.assert_allclose(r, p.mob * fprime * p.h ** 2, rtol=1e-13)
    c = cbar
    for _ in range(3):
        fp = (4 * c * (c - 1) * (c - 0.5)) if fe == O.F_01 else (c ** 3 - c)
        c = c - dt * p.mob * fp
    U = O.explicit(p, np.full(p.nnodes, cbar), dt, 3)
    np.testing.assert_allclose(U, c, rtol=1e-14)


def test_pin3_lumped_mass(orc):
    p = O.Problem(n=(5, 4, 3), h=0.5)
    np.testing.assert_allclose(O.lumped_mass(p), 0.125, rtol=1e-14)
    q = O.Problem(n=(4, 3), bc=O.NOFLUX, h=2.0)
    m = O.lumped_mass(q).reshape(3, 4)
    assert m[1, 1] == pytest.approx(4.0) and m[0, 1] == pytest.approx(2.0) and m[0, 0] == pytest.approx(1.0)


# ---------------------------------------------------------------- PIN4 ------
# r = grad E_h exactly (Allen-Cahn, L = 1) and g = grad_c E_h (Cahn-Hilliard
# mu-row source), because both come from the same quadrature.
@pytest.mark.parametrize("n,fe,bc", [((2, 2), O.F_SYM, O.PERIODIC), ((3, 4), O.F_01, O.PERIODIC),
                                     ((4, 3), O.F_SYM, O.NOFLUX), ((2, 3, 2), O.F_01, O.PERIODIC),
                                     ((3, 3, 3), O.F_SYM, O.NOFLUX)])
def test_pin4_residual_is_energy_gradient(orc, n, fe, bc):
    p = O.Problem(n=n, model=O.AC, fe=fe, bc=bc, W=1.1, kappa=0.9, mob=1.0, h=0.7)
    u = 0.5 + 0.4 * rng.standard_normal(p.nnodes)
    r = O.residual(p, u)
    g = np.zeros(p.nnodes)
    eps = 1e-5
    for i in range(p.nnodes):
        e = np.zeros(p.nnodes)
        e[i] = eps
        g[i] = (O.energy(p, u + e) - O.energy(p, u - e)) / (2 * eps)
    assert _rel(r, g) < 1e-8
    # Cahn-Hilliard: mu-row = m mu - grad_c E_h
    q = O.Problem(n=n, model=O.CH, fe=fe, bc=bc, W=1.1, kappa=0.9, mob=1.3, h=0.7)
    mu = rng.standard_normal(p.nnodes)
    rq = O.residual(q, np.concatenate([u, mu]))
    assert _rel(O.lumped_mass(q) * mu - rq[p.nnodes:], g) < 1e-8


# ---------------------------------------------------------------- PIN5 ------
@pytest.mark.parametrize("model,n", [(O.AC, (3, 4)), (O.CH, (3, 3)), (O.AC, (2, 3, 2)), (O.CH, (2, 2, 3))])
def test_pin5_jvp_matches_fd_and_dot_test(orc, model, n):
    p = O.Problem(n=n, model=model, fe=O.F_01, W=1.0, kappa=2.0, mob=0.8, h=1.0)
    U = 0.4 + 0.2 * rng.standard_normal(p.ndof)
    Uold = U + 0.01 * rng.standard_normal(p.ndof)
    v = rng.standard_normal(p.ndof)
    w = rng.standard_normal(p.ndof)
    dt = 0.3
    Jv = O.jvp(p, 1.0 / dt, U, v)
    eps = 1e-6
    fd = (O.be_residual(p, dt, Uold, U + eps * v) - O.be_residual(p, dt, Uold, U - eps * v)) / (2 * eps)
    assert _rel(Jv, fd) < 1e-7
    Jtw = O.jvp_t(p, 1.0 / dt, U, w)
    assert abs(Jv @ w - v @ Jtw) < 1e-12 * np.linalg.norm(Jv) * np.linalg.norm(w)
    # parameter derivatives by central differences of r
    g = O.dr_dtheta(p, U, w)
    for k, name in enumerate(["mob", "kappa", "W"]):
        hp = O.Problem(**{**p.__dict__, name: getattr(p, name) + eps})
        hm = O.Problem(**{**p.__dict__, name: getattr(p, name) - eps})
        fdk = w @ (O.residual(hp, U) - O.residual(hm, U)) / (2 * eps)
        assert g[k] == pytest.approx(fdk, rel=1e-7, abs=1e-9)


def test_pin5_ac_jacobian_symmetric(orc):
    p = O.Problem(n=(3, 3), model=O.AC, fe=O.F_SYM, W=1.0, kappa=1.0, mob=1.0)
    U = rng.standard_normal(p.ndof)
    J = np.stack([O.jvp(p, 2.0, U, e) for e in np.eye(p.ndof)], axis=1)
    assert np.max(np.abs(J - J.T)) < 1e-14


# ---------------------------------------------------------------- PIN6 ------
def _symbols(n, k, h):
    th = [2 * np.pi * k[a] / n[a] for a in range(len(n))]
    cs = [np.cos(t) for t in th]
    if len(n) == 2:
        lk = (8 - 2 * cs[0] - 2 * cs[1] - 4 * cs[0] * cs[1]) / (3 * h * h)
        lm = (2 + cs[0]) * (2 + cs[1]) / 9
    else:
        lk = sum((2 - 2 * cs[a]) * (2 + cs[(a + 1) % 3]) * (2 + cs[(a + 2) % 3]) for a in range(3)) / (9 * h * h)
        lm = (2 + cs[0]) * (2 + cs[1]) * (2 + cs[2]) / 27
    return th, lk, lm


def _mode(n, th, h):
    grids = np.meshgrid(*[np.arange(m) for m in reversed(n)], indexing="ij")
    ph = sum(th[a] * grids[len(n) - 1 - a] for a in range(len(n)))
    return np.cos(ph).ravel()


@pytest.mark.parametrize("n,k", [((16, 12), (3, 2)), ((8, 8), (4, 1)), ((8, 6, 4), (1, 2, 1))])
def test_pin6_fourier_multipliers(orc, n, k):
    h, dt, eps = 0.8, 0.02, 1e-6
    th, lk, lm = _symbols(n, k, h)
    mode = _mode(n, th, h)
    # Allen-Cahn about 0 with f_sym: f''(0) = -W
    p = O.Problem(n=n, model=O.AC, fe=O.F_SYM, W=1.2, kappa=0.9, mob=1.1, h=h)
    g = 1 - dt * p.mob * (p.kappa * lk - p.W * lm)
    out = O.explicit(p, eps * mode, dt, 1)
    assert _rel(out, g * eps * mode) < 1e-10
    # Cahn-Hilliard about 1/2 with f_01: f''(1/2) = -W
    q = O.Problem(n=n, model=O.CH, fe=O.F_01, W=1.2, kappa=0.9, mob=1.1, h=h)
    gq = 1 - dt * q.mob * lk * (-q.W * lm + q.kappa * lk)
    U = np.concatenate([0.5 + eps * mode, np.zeros(q.nnodes)])
    out = O.explicit(q, U, dt, 1)[: q.nnodes]
    assert _rel(out - 0.5, gq * eps * mode) < 1e-9


def test_pin6_backward_euler_mode(orc):
    # linear Allen-Cahn (f == 0): BE damps each mode by exactly 1/(1 + dt L kappa lambda_K)
    n, k, h, dt = (8, 6), (3, 1), 1.0, 0.7
    th, lk, lm = _symbols(n, k, h)
    mode = _mode(n, th, h)
    p = O.Problem(n=n, model=O.AC, fe=O.F_SYM, W=0.0, kappa=1.5, mob=0.9, h=h)
    U, conv, its, _ = O.newton_be(p, dt, mode, solver=0)
    assert conv
    assert _rel(U, mode / (1 + dt * p.mob * p.kappa * lk)) < 1e-12


# ---------------------------------------------------------------- PIN7 ------
def _strip_equilibrium(model, h, kappa=1.0, W=1.0, X=10.0):
    nx = int(round(2 * X / h)) + 1
    x = -X + h * np.arange(nx)
    if model == O.AC:
        prof = np.tanh(x / np.sqrt(2 * kappa / W))
        p = O.Problem(n=(nx, 2), model=O.AC, fe=O.F_SYM, bc=O.NOFLUX, W=W, kappa=kappa, mob=1.0, h=h)
        U0 = np.tile(prof, 2)
    else:
        prof = 0.5 * (1 + np.tanh(x / np.sqrt(2 * kappa / W)))
        p = O.Problem(n=(nx, 2), model=O.CH, fe=O.F_01, bc=O.NOFLUX, W=W, kappa=kappa, mob=1.0, h=h)
        U0 = np.concatenate([np.tile(prof, 2), np.zeros(2 * nx)])
    # steady state: backward Euler with a very large step (Newton on r = 0 up to
    # the conserved mass for Cahn-Hilliard)
    U, conv, its, hist = O.newton_be(p, 1e8, U0, rtol=1e-13, maxit=40, solver=0)
    err = np.max(np.abs(U[:nx] - prof))
    return err


@pytest.mark.parametrize("model", [O.AC, O.CH])
def test_pin7_tanh_equilibrium_second_order(orc, model):
    e = [_strip_equilibrium(model, h) for h in (0.5, 0.25, 0.125)]
    assert e[0] / e[1] > 3.5 and e[1] / e[2] > 3.5, e
    assert e[2] < 2e-3


# ---------------------------------------------------------------- PIN8/9 ----
def test_pin8_ch_explicit_conserves_mass(orc):
    p = O.Problem(n=(16, 16), model=O.CH, fe=O.F_01, W=1.0, kappa=2.0, mob=1.0, h=1.0)
    c = 0.5 + rng.uniform(-0.01, 0.01, p.nnodes)
    U = O.explicit(p, np.concatenate([c, 0 * c]), 0.01, 200)
    assert abs(O.total_mass(p, U) - O.total_mass(p, c)) < 1e-12 * O.total_mass(p, c)
    assert np.max(np.abs(U[: p.nnodes] - c)) > 1e-6  # it did move


def test_pin8_ch_backward_euler_conserves_mass(orc):
    p = O.Problem(n=(6, 5, 4), model=O.CH, fe=O.F_01, W=1.0, kappa=2.0, mob=1.0, h=1.0)
    c = 0.4 + rng.uniform(-0.02, 0.02, p.nnodes)
    U0 = np.concatenate([c, np.zeros_like(c)])
    U, conv, its, hist = O.newton_be(p, 0.5, U0, rtol=1e-10, solver=1, lin_rtol=1e-13)
    assert conv
    assert abs(O.total_mass(p, U) - O.total_mass(p, c)) < 1e-11 * O.total_mass(p, c)


def test_pin9_energy_decay(orc):
    # Allen-Cahn explicit within dt L (4 kappa / h^2 + max f'') <= 2
    p = O.Problem(n=(24, 24), model=O.AC, fe=O.F_SYM, W=1.0, kappa=1.0, mob=1.0, h=1.0)
    U = rng.uniform(-0.05, 0.05, p.nnodes)
    E = [O.energy(p, U)]
    for _ in range(40):
        U = O.explicit(p, U, 0.1, 5)
        E.append(O.energy(p, U))
    assert all(E[i + 1] <= E[i] + 1e-12 * abs(E[i]) for i in range(len(E) - 1))
    # Cahn-Hilliard backward Euler at dt < 4 kappa / (M gamma^2)
    q = O.Problem(n=(10, 10), model=O.CH, fe=O.F_01, W=1.0, kappa=2.0, mob=1.0, h=1.0)
    c = 0.4 + rng.uniform(-0.05, 0.05, q.nnodes)
    U = np.concatenate([c, np.zeros_like(c)])
    E = [O.energy(q, U)]
    for _ in range(6):
        U, conv, _, _ = O.newton_be(q, 2.0, U, rtol=1e-11, solver=0)
        assert conv
        E.append(O.energy(q, U))
    assert all(E[i + 1] <= E[i] + 1e-12 * abs(E[i]) for i in range(len(E) - 1))


# ---------------------------------------------------------------- PIN10 -----
def test_pin10_symmetries(orc):
    n = (6, 5)
    p = O.Problem(n=n, model=O.AC, fe=O.F_SYM, W=1.0, kappa=1.3, mob=0.9, h=0.6)
    u = rng.standard_normal(p.nnodes)
    r = O.residual(p, u).reshape(5, 6)
    U = u.reshape(5, 6)
    # translation
    rt = O.residual(p, np.roll(U, (2, 3), axis=(0, 1)).ravel()).reshape(5, 6)
    assert np.max(np.abs(rt - np.roll(r, (2, 3), axis=(0, 1)))) < 1e-13
    # reflection
    rf = O.residual(p, U[:, ::-1].ravel()).reshape(5, 6)
    assert np.max(np.abs(rf - r[:, ::-1])) < 1e-13
    # axis permutation
    pT = O.Problem(n=(5, 6), model=O.AC, fe=O.F_SYM, W=1.0, kappa=1.3, mob=0.9, h=0.6)
    rT = O.residual(pT, U.T.ravel()).reshape(6, 5)
    assert np.max(np.abs(rT - r.T)) < 1e-13
    # c -> -c (f_sym is even)
    assert np.max(np.abs(O.residual(p, -u) + O.residual(p, u))) < 1e-13
    # c -> 1 - c (f_01 symmetric about 1/2)
    q = O.Problem(n=n, model=O.AC, fe=O.F_01, W=1.0, kappa=1.3, mob=0.9, h=0.6)
    assert np.max(np.abs(O.residual(q, 1 - u) + O.residual(q, u))) < 1e-12


# ---------------------------------------------------------------- PIN11/12 --
def test_pin11_adjoint_closed_form_heat(orc):
    # f == 0: each mode evolves as g^N with g = 1 - dt L kappa lambda_K
    n, k, h, dt, N = (12, 10), (2, 3), 1.0, 0.05, 30
    th, lk, lm = _symbols(n, k, h)
    mode = _mode(n, th, h)
    p = O.Problem(n=n, model=O.AC, fe=O.F_SYM, W=0.0, kappa=1.4, mob=0.8, h=h)
    A = 0.3
    # O = (1/N) sum_i eta_i^N mode_i = A g^N <mode^2>
    m2 = np.mean(mode * mode)
    gU = mode / p.nnodes
    tb, ub = O.explicit_adjoint(p, dt, N, A * mode, gU)
    g = 1 - dt * p.mob * p.kappa * lk
    dO_dg = A * m2 * N * g ** (N - 1)
    assert tb[0] == pytest.approx(dO_dg * (-dt * p.kappa * lk), rel=1e-10)
    assert tb[1] == pytest.approx(dO_dg * (-dt * p.mob * lk), rel=1e-10)
    # (the W-sensitivity at W = 0 is not zero, dr/dW = L N_1(eta); it is
    # covered by the finite-difference test below)
    np.testing.assert_allclose(ub, g ** N * mode / p.nnodes, rtol=1e-10, atol=1e-16)


@pytest.mark.parametrize("model", [O.AC, O.CH])
def test_pin11_adjoint_vs_central_fd(orc, model):
    n, dt, N = (8, 8), 0.05, 25
    if model == O.AC:
        p = O.Problem(n=n, model=O.AC, fe=O.F_SYM, W=1.3, kappa=0.8, mob=1.2)
        U0 = rng.uniform(-0.5, 0.5, p.nnodes)
    else:
        p = O.Problem(n=n, model=O.CH, fe=O.F_01, W=1.3, kappa=0.8, mob=1.2)
        U0 = np.concatenate([0.5 + rng.uniform(-0.2, 0.2, p.nnodes), np.zeros(p.nnodes)])
    target = rng.uniform(-0.5, 0.5, p.nnodes)

    def loss(q, u0):
        u = O.explicit(q, u0, dt, N)[: q.nnodes]
        return np.mean((u - target) ** 2)

    uN = O.explicit(p, U0, dt, N)[: p.nnodes]
    gU = 2 * (uN - target) / p.nnodes
    tb, ub = O.explicit_adjoint(p, dt, N, U0, gU)
    for k, name in enumerate(["mob", "kappa", "W"]):
        eps = 1e-6 * getattr(p, name)
        hp = O.Problem(**{**p.__dict__, name: getattr(p, name) + eps})
        hm = O.Problem(**{**p.__dict__, name: getattr(p, name) - eps})
        fd = (loss(hp, U0) - loss(hm, U0)) / (2 * eps)
        assert tb[k] == pytest.approx(fd, rel=1e-6)
    # initial-condition gradient, a few entries
    for i in (0, 17, 40):
        e = np.zeros(p.ndof)
        e[i] = 1e-6
        fd = (loss(p, U0 + e) - loss(p, U0 - e)) / 2e-6
        assert ub[i] == pytest.approx(fd, rel=1e-5, abs=1e-12)


def test_pin12_conserved_objective_has_zero_gradient(orc):
    # d/dtheta of mean(c) = 0 for Cahn-Hilliard (paper Eq. 20 objective)
    p = O.Problem(n=(8, 8), model=O.CH, fe=O.F_01, W=1.0, kappa=1.5, mob=1.0)
    U0 = np.concatenate([0.5 + rng.uniform(-0.1, 0.1, p.nnodes), np.zeros(p.nnodes)])
    tb, ub = O.explicit_adjoint(p, 0.02, 20, U0, np.full(p.nnodes, 1.0 / p.nnodes))
    assert np.max(np.abs(tb)) < 1e-13
    np.testing.assert_allclose(ub, 1.0 / p.nnodes, rtol=1e-12)


def test_newton_adjoint_vs_fd(orc):
    p = O.Problem(n=(4, 4), model=O.CH, fe=O.F_01, W=1.0, kappa=2.0, mob=1.0)
    c = 0.4 + rng.uniform(-0.1, 0.1, p.nnodes)
    Uold = np.concatenate([c, np.zeros_like(c)])
    dt = 0.5
    w = rng.standard_normal(p.ndof)

    def obj(q, uold):
        U, conv, _, _ = O.newton_be(q, dt, uold, rtol=1e-14, maxit=30, solver=0)
        return w @ U

    U, conv, _, _ = O.newton_be(p, dt, Uold, rtol=1e-14, maxit=30, solver=0)
    tb, ub = O.newton_adjoint(p, dt, U, w, solver=0)
    for k, name in enumerate(["mob", "kappa", "W"]):
        eps = 1e-6
        hp = O.Problem(**{**p.__dict__, name: getattr(p, name) + eps})
        hm = O.Problem(**{**p.__dict__, name: getattr(p, name) - eps})
        assert tb[k] == pytest.approx((obj(hp, Uold) - obj(hm, Uold)) / (2 * eps), rel=1e-6)
    for i in (0, 5, 9):
        e = np.zeros(p.ndof)
        e[i] = 1e-6
        assert ub[i] == pytest.approx((obj(p, Uold + e) - obj(p, Uold - e)) / 2e-6, rel=1e-6, abs=1e-10)


def test_gmres_matches_dense(orc):
    p = O.Problem(n=(5, 4, 3), model=O.CH, fe=O.F_01, W=1.0, kappa=2.0, mob=1.0)
    U = 0.4 + 0.05 * rng.standard_normal(p.ndof)
    b = rng.standard_normal(p.ndof)
    for tr in (False, True):
        x0 = O.linear_solve(p, 2.0, U, b, transpose=tr, solver=0)
        x1 = O.linear_solve(p, 2.0, U, b, transpose=tr, solver=1, lin_rtol=1e-13)
        assert _rel(x1, x0) < 1e-10


def test_energy_closed_forms(orc):
    # uniform state: E = V f(c); linear ramp on a no-flux grid with f == 0: E = kappa/2 |a|^2 V
    p = O.Problem(n=(5, 4), model=O.AC, fe=O.F_01, W=1.3, kappa=0.7, h=0.5)
    V = 5 * 4 * 0.25
    assert O.energy(p, np.full(20, 0.3)) == pytest.approx(V * 1.3 * 0.09 * 0.49, rel=1e-14)
    q = O.Problem(n=(5, 4), model=O.AC, fe=O.F_SYM, W=0.0, kappa=0.7, h=0.5, bc=O.NOFLUX)
    x = 0.5 * np.tile(np.arange(5), 4)
    V = (4 * 0.5) * (3 * 0.5)
    assert O.energy(q, 2.0 * x) == pytest.approx(0.5 * 0.7 * 4.0 * V, rel=1e-14)
