"""Pins of the oracle's Gauss-Lobatto (nodal) quadrature variant.

With the 2-point Lobatto rule per axis the quadrature points are the element's
nodes, so every Q1 shape function is 1 at its own node and 0 at the others.  Then
(derived from the element integrals, Sec. 2.2 weak forms with nodal quadrature):
  - the nonlinear term is nodal: N(c)_a = m_a f'(c_a), m_a the lumped mass;
  - the mass matrix is diagonal (consistent = lumped);
  - the stiffness is the 5-point stencil 4 c_i - (axis neighbours) in 2-D (no h)
    and h (6 c_i - axis neighbours) in 3-D; at a no-flux boundary node, K c / m is
    the interior stencil over the field reflected about the boundary, over h^2;
  - E_h = sum_a m_a f(c_a) + kappa/2 c^T K c, and c^T K c = h^(d-2) sum over axis
    edges of (c_i - c_j)^2 on a periodic grid.
Each test checks the oracle against one of these written out independently (numpy
rolls and pads), against finite differences of its own energy, against Fourier
multipliers, or against the tanh equilibrium at second order.
"""
import numpy as np
import pytest

import oracle as O

rng = np.random.default_rng(77)
L = O.LOBATTO


def _rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


def _grid(c, n):
    return np.asarray(c).reshape(tuple(reversed(n)))  # [z][y][x] or [y][x]


def _stencil(c, n, h, bc):
    """sum over axes of (2 c - c_prev - c_next) on the periodic or reflected field, times
    h^(d-2) (2-D: h-independent)."""
    C = _grid(c, n)
    d = len(n)
    P = np.pad(C, 1, mode="wrap" if bc == O.PERIODIC else "reflect")
    core = tuple(slice(1, -1) for _ in range(d))
    out = np.zeros_like(C)
    for ax in range(d):
        lo = list(core)
        hi = list(core)
        lo[ax] = slice(0, -2)
        hi[ax] = slice(2, None)
        out += 2 * C - P[tuple(lo)] - P[tuple(hi)]
    return (out * h ** (d - 2)).ravel()


def _boundary_factor(n):
    """2^-b, b = the number of axes on which a node is a boundary node."""
    d = len(n)
    idx = np.meshgrid(*[np.arange(m) for m in reversed(n)], indexing="ij")
    b = sum(((i == 0) | (i == m - 1)).astype(int) for i, m in zip(idx, reversed(n)))
    return (0.5 ** b).ravel()


def _df(fe, W, c):
    return W * (c ** 3 - c) if fe == O.F_SYM else 2 * W * c * (1 - c) * (1 - 2 * c)


def _f(fe, W, c):
    return 0.25 * W * (c * c - 1) ** 2 if fe == O.F_SYM else W * c * c * (1 - c) ** 2


@pytest.mark.parametrize("n,h", [((6, 5), 1.0), ((7, 4), 0.37), ((4, 5, 3), 1.0), ((3, 4, 5), 0.6)])
def test_lobatto_stiffness_stencil_periodic(orc, n, h):
    p = O.Problem(n=n, model=O.AC, fe=O.F_SYM, W=0.0, kappa=1.7, mob=0.8, h=h, quad=L)
    eta = rng.standard_normal(p.nnodes)
    r = O.residual(p, eta)
    assert _rel(r, p.mob * p.kappa * _stencil(eta, n, h, O.PERIODIC)) < 1e-13


@pytest.mark.parametrize("n,h", [((6, 5), 1.0), ((5, 7), 0.45), ((4, 5, 3), 1.0), ((3, 4, 5), 0.6)])
def test_lobatto_noflux_stiffness_is_reflected_stencil(orc, n, h):
    p = O.Problem(n=n, model=O.AC, fe=O.F_SYM, W=0.0, kappa=1.3, mob=1.0, h=h, bc=O.NOFLUX, quad=L)
    eta = rng.standard_normal(p.nnodes)
    m = O.lumped_mass(p)
    assert _rel(m, h ** len(n) * _boundary_factor(n)) < 1e-14
    r = O.residual(p, eta)
    ref = p.kappa * _stencil(eta, n, h, O.NOFLUX) / h ** len(n)  # K c / m on the reflected field
    assert _rel(r / m, ref) < 1e-13


@pytest.mark.parametrize("fe", [O.F_SYM, O.F_01])
@pytest.mark.parametrize("n,bc", [((5, 6), O.PERIODIC), ((6, 4), O.NOFLUX), ((3, 4, 3), O.PERIODIC),
                                  ((4, 3, 3), O.NOFLUX)])
def test_lobatto_nonlinear_term_is_nodal(orc, fe, n, bc):
    p = O.Problem(n=n, model=O.AC, fe=fe, W=1.3, kappa=0.0, mob=0.7, h=0.8, bc=bc, quad=L)
    c = rng.uniform(-0.3, 1.2, p.nnodes)
    r = O.residual(p, c)
    m = 0.8 ** len(n) * _boundary_factor(n) if bc == O.NOFLUX else np.full(p.nnodes, 0.8 ** len(n))
    assert _rel(r, p.mob * m * _df(fe, p.W, c)) < 1e-13


@pytest.mark.parametrize("n,h", [((6, 5), 0.9), ((4, 3, 5), 0.7)])
def test_lobatto_energy_closed_form(orc, n, h):
    for fe in (O.F_SYM, O.F_01):
        p = O.Problem(n=n, model=O.AC, fe=fe, W=1.1, kappa=1.7, h=h, quad=L)
        c = rng.uniform(-0.5, 1.1, p.nnodes)
        C = _grid(c, n)
        edges = sum(np.sum((C - np.roll(C, 1, axis=ax)) ** 2) for ax in range(len(n)))
        ref = h ** len(n) * np.sum(_f(fe, p.W, c)) + 0.5 * p.kappa * h ** (len(n) - 2) * edges
        assert O.energy(p, c) == pytest.approx(ref, rel=1e-13)


@pytest.mark.parametrize("n,fe,bc", [((2, 2), O.F_SYM, O.PERIODIC), ((3, 4), O.F_01, O.PERIODIC),
                                     ((4, 3), O.F_SYM, O.NOFLUX), ((2, 3, 2), O.F_01, O.PERIODIC),
                                     ((3, 3, 3), O.F_SYM, O.NOFLUX)])
def test_lobatto_residual_is_energy_gradient(orc, n, fe, bc):
    p = O.Problem(n=n, model=O.AC, fe=fe, bc=bc, W=1.1, kappa=0.9, mob=1.0, h=0.7, quad=L)
    u = 0.5 + 0.4 * rng.standard_normal(p.nnodes)
    r = O.residual(p, u)
    g = np.zeros(p.nnodes)
    eps = 1e-5
    for i in range(p.nnodes):
        e = np.zeros(p.nnodes)
        e[i] = eps
        g[i] = (O.energy(p, u + e) - O.energy(p, u - e)) / (2 * eps)
    assert _rel(r, g) < 1e-8
    q = O.Problem(n=n, model=O.CH, fe=fe, bc=bc, W=1.1, kappa=0.9, mob=1.3, h=0.7, quad=L)
    mu = rng.standard_normal(p.nnodes)
    rq = O.residual(q, np.concatenate([u, mu]))
    assert _rel(O.lumped_mass(q) * mu - rq[p.nnodes:], g) < 1e-8


@pytest.mark.parametrize("model,n", [(O.AC, (3, 4)), (O.CH, (3, 3)), (O.AC, (2, 3, 2)), (O.CH, (3, 2, 3))])
def test_lobatto_jvp_matches_fd_and_dot_test(orc, model, n):
    p = O.Problem(n=n, model=model, fe=O.F_01, W=1.0, kappa=2.0, mob=0.8, h=0.9, quad=L)
    U = 0.4 + 0.2 * rng.standard_normal(p.ndof)
    Uold = U + 0.01 * rng.standard_normal(p.ndof)
    v = rng.standard_normal(p.ndof)
    w = rng.standard_normal(p.ndof)
    dt = 0.3
    Jv = O.jvp(p, 1.0 / dt, U, v)
    eps = 1e-6
    fd = (O.be_residual(p, dt, Uold, U + eps * v) - O.be_residual(p, dt, Uold, U - eps * v)) / (2 * eps)
    assert _rel(Jv, fd) < 1e-7
    assert abs(Jv @ w - v @ O.jvp_t(p, 1.0 / dt, U, w)) < 1e-12 * np.linalg.norm(Jv) * np.linalg.norm(w)


def test_lobatto_consistent_mass_is_lumped(orc):
    """Nodal quadrature makes the Gauss-integrated mass diagonal: the backward-Euler
    residual is the same with either mass option."""
    for model, n in ((O.AC, (5, 4)), (O.CH, (4, 3, 3))):
        a = O.Problem(n=n, model=model, fe=O.F_01, W=1.0, kappa=1.5, mob=1.2, h=0.8, quad=L)
        b = O.Problem(**{**a.__dict__, "mass": O.CONSISTENT})
        U = rng.uniform(0.2, 0.8, a.ndof)
        Uold = rng.uniform(0.2, 0.8, a.ndof)
        assert _rel(O.be_residual(b, 0.4, Uold, U), O.be_residual(a, 0.4, Uold, U)) < 1e-15


@pytest.mark.parametrize("n,k", [((16, 12), (3, 2)), ((8, 8), (4, 1)), ((8, 6, 4), (1, 2, 1))])
def test_lobatto_fourier_multipliers(orc, n, k):
    """One explicit step of a small mode about a uniform state multiplies it by
    1 - dt L (kappa lambda_K + f'') (Allen-Cahn) or 1 - dt M lambda_K (f'' + kappa lambda_K)
    (Cahn-Hilliard), with lambda_K = sum_a (2 - 2 cos theta_a) / h^2 and no mass symbol."""
    h, dt, eps = 0.8, 0.02, 1e-6
    th = [2 * np.pi * k[a] / n[a] for a in range(len(n))]
    lk = sum(2 - 2 * np.cos(t) for t in th) / (h * h)
    grids = np.meshgrid(*[np.arange(m) for m in reversed(n)], indexing="ij")
    mode = np.cos(sum(th[a] * grids[len(n) - 1 - a] for a in range(len(n)))).ravel()
    p = O.Problem(n=n, model=O.AC, fe=O.F_SYM, W=1.2, kappa=0.9, mob=1.1, h=h, quad=L)
    out = O.explicit(p, eps * mode, dt, 1)
    assert _rel(out, (1 - dt * p.mob * (p.kappa * lk - p.W)) * eps * mode) < 1e-10
    q = O.Problem(n=n, model=O.CH, fe=O.F_01, W=1.2, kappa=0.9, mob=1.1, h=h, quad=L)
    U = np.concatenate([0.5 + eps * mode, np.zeros(q.nnodes)])
    out = O.explicit(q, U, dt, 1)[: q.nnodes]
    assert _rel(out - 0.5, (1 - dt * q.mob * lk * (-q.W + q.kappa * lk)) * eps * mode) < 1e-9


def _strip(h, X=10.0):
    nx = int(round(2 * X / h)) + 1
    x = -X + h * np.arange(nx)
    prof = np.tanh(x / np.sqrt(2.0))
    p = O.Problem(n=(nx, 2), model=O.AC, fe=O.F_SYM, bc=O.NOFLUX, W=1.0, kappa=1.0, mob=1.0, h=h, quad=L)
    U, _, _, hist = O.newton_be(p, 1e8, np.tile(prof, 2), rtol=1e-13, maxit=6, solver=0)
    assert hist[-1] < 1e-13  # the FP64 floor of r (rtol 1e-13 of a 1e-5 start is below it)
    return np.max(np.abs(U[:nx] - prof))


def test_lobatto_tanh_equilibrium_second_order(orc):
    """The Allen-Cahn kink tanh(x / sqrt(2 kappa / W)) is the steady state of the
    continuous problem; the nodal scheme reaches it at second order in h."""
    e = [_strip(h) for h in (0.5, 0.25, 0.125)]
    assert e[0] / e[1] > 3.5 and e[1] / e[2] > 3.5, e
    assert e[2] < 2e-3
