"""Pins of the FP64 elasticity oracle (Eshelby inclusion, Eqs. 3-4 and Eq. III.1)
against facts that do not come from the oracle itself: exact polynomial
solutions of the Q1 space (rigid-body modes, affine fields and their boundary
tractions, free dilation under a uniform eigenstrain), the discrete
average-strain identity of a traction-free body, Eshelby's closed-form interior
strain of a circular / spherical inclusion, symmetry and definiteness of the
stiffness, and central finite differences of the adjoint sensitivities.
"""
import itertools

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def coords(p):
    """Node coordinates, shape (N, dim), node index i + n0 (j + n1 k)."""
    axes = [np.arange(n) * p.h for n in p.n]
    grids = np.meshgrid(*axes, indexing="ij")
    return np.stack([g.transpose(*reversed(range(p.dim))).ravel() for g in grids], axis=1)


def field(p, comps):
    """Stack per-component nodal arrays into the component-major layout."""
    return np.concatenate([np.asarray(c, dtype=np.float64).ravel() for c in comps])


def lame(E, nu):
    return E * nu / ((1 + nu) * (1 - 2 * nu)), E / (2 * (1 + nu))


def test_eigenstrain_profile():
    p = oracle.ElasticProblem((3, 3), m=0.02, a=10.0, l=2.0)
    assert oracle.el_eigen(p, 10.0) == pytest.approx(0.01, rel=1e-15)
    # m inside the inclusion, 0 far outside, monotone in between
    assert oracle.el_eigen(p, 0.0) == pytest.approx(0.02, rel=1e-12)
    assert oracle.el_eigen(p, 40.0) == pytest.approx(0.0, abs=1e-20)
    r = np.linspace(0, 30, 61)
    v = [oracle.el_eigen(p, x) for x in r]
    assert all(a >= b for a, b in zip(v, v[1:]))
    # tanh form: s(a + t) + s(a - t) = m
    for t in (0.3, 1.7, 5.0):
        assert oracle.el_eigen(p, 10 + t) + oracle.el_eigen(p, 10 - t) == pytest.approx(0.02, rel=1e-14)
    flat = oracle.ElasticProblem((3, 3), m=0.02, a=10.0, l=0.0)
    assert oracle.el_eigen(flat, 3.0) == 0.01


@pytest.mark.parametrize("n", [(6, 5), (4, 5, 3)])
def test_rigid_body_modes_are_null(n):
    """With every face traction-free, translations and infinitesimal rotations
    carry no strain, so K annihilates them."""
    p = oracle.ElasticProblem(n, h=0.7, E=3.0, nu=0.27, sym=0)
    X = coords(p)
    modes = []
    for c in range(p.dim):
        comps = [np.zeros(p.nnodes) for _ in range(p.dim)]
        comps[c][:] = 1.0
        modes.append(field(p, comps))
    for i, j in itertools.combinations(range(p.dim), 2):
        comps = [np.zeros(p.nnodes) for _ in range(p.dim)]
        comps[i] = -X[:, j]
        comps[j] = X[:, i]
        modes.append(field(p, comps))
    for u in modes:
        assert np.abs(oracle.el_apply(p, u)).max() < 1e-12


def face_weight(p, idx, axis):
    """Integral of the node's shape function over the face normal to `axis` it lies on."""
    w = 1.0
    for k in range(p.dim):
        if k == axis:
            continue
        on_edge = idx[k] == 0 or idx[k] == p.n[k] - 1
        w *= p.h / 2 if on_edge else p.h
    return w


@pytest.mark.parametrize("n", [(5, 4), (4, 3, 5)])
def test_affine_field_gives_boundary_tractions(n):
    """u = G x has the uniform stress sigma = lambda tr(eps) I + 2 mu eps,
    eps = (G + G^T)/2; K u is then zero inside and equals the traction
    sigma . n_out integrated against each boundary node's shape function."""
    rng = np.random.default_rng(5)
    p = oracle.ElasticProblem(n, h=1.3, E=7.0, nu=0.21, sym=0)
    d = p.dim
    G = rng.standard_normal((d, d))
    X = coords(p)
    u = field(p, [X @ G[c] for c in range(d)])
    y = oracle.el_apply(p, u).reshape(d, p.nnodes)
    lam, mu = lame(p.E, p.nu)
    eps = 0.5 * (G + G.T)
    sig = lam * np.trace(eps) * np.eye(d) + 2 * mu * eps
    expect = np.zeros((d, p.nnodes))
    for a in range(p.nnodes):
        idx = [(a // int(np.prod(p.n[:k]))) % p.n[k] for k in range(d)]
        for axis in range(d):
            for side, normal in ((0, -1.0), (p.n[axis] - 1, 1.0)):
                if idx[axis] == side:
                    expect[:, a] += sig[:, axis] * normal * face_weight(p, idx, axis)
    assert np.abs(y - expect).max() < 1e-12 * max(1.0, np.abs(expect).max())


@pytest.mark.parametrize("n", [(7, 6), (5, 4, 6)])
def test_uniform_eigenstrain_is_free_dilation(n):
    """A uniform eigenstrain e0 I in a body with symmetry planes and free outer
    faces relaxes without stress: u = e0 x exactly (the Q1 space holds it)."""
    p = oracle.ElasticProblem(n, h=2.5, E=22.5, nu=0.3, m=0.04, a=5.0, l=0.0)
    e0 = 0.02
    u, it = oracle.el_solve(p, rtol=1e-14)
    assert it > 0
    X = coords(p)
    expect = field(p, [e0 * X[:, c] for c in range(p.dim)])
    assert np.abs(u - expect).max() < 1e-12


@pytest.mark.parametrize("n", [(6, 7), (4, 5, 4)])
def test_stiffness_symmetric_positive_definite(n):
    rng = np.random.default_rng(11)
    p = oracle.ElasticProblem(n, h=0.9, E=5.0, nu=0.33)
    mask = oracle.el_free_mask(p)
    for _ in range(3):
        u, v = rng.standard_normal((2, p.ndof))
        Ku, Kv = oracle.el_apply(p, u), oracle.el_apply(p, v)
        assert u @ Kv == pytest.approx(v @ Ku, rel=1e-12)
        assert u @ Ku > 0
    # fixed components: identity rows, and they do not feed the free rows
    u = rng.standard_normal(p.ndof)
    Ku = oracle.el_apply(p, u)
    assert np.array_equal(Ku[mask == 0], u[mask == 0])
    assert np.allclose(oracle.el_apply(p, u * mask)[mask == 1], Ku[mask == 1], rtol=0, atol=1e-14)


@pytest.mark.parametrize("n,E,nu", [((12, 10), 22.5, 0.3), ((12, 10), 3.0, 0.1),
                                    ((6, 7, 5), 22.5, 0.3), ((6, 7, 5), 9.0, 0.45)])
def test_volume_change_equals_eigenstrain_integral(n, E, nu):
    """Testing the discrete equilibrium with v = (g_1 x_1, ..., g_d x_d) (in the
    Q1 space and zero on the symmetry planes) gives sum_q |J| sigma_ii = 0, so
    with one homogeneous stiffness the volume change is d times the quadrature
    integral of the eigenstrain, whatever E and nu: dV/dE = dV/dnu = 0."""
    p = oracle.ElasticProblem(n, h=3.0, E=E, nu=nu, m=0.01, a=12.0, l=0.4)
    O, dE, dnu, u, ok = oracle.el_sensitivity(p, rtol=1e-14)
    assert ok
    ref = p.dim * oracle.el_eigen_integral(p)
    assert O == pytest.approx(ref, rel=1e-11)
    assert oracle.el_objective(p, u) == pytest.approx(O, rel=1e-15)
    assert abs(dE) < 1e-10 * abs(O) and abs(dnu) < 1e-10 * abs(O)


@pytest.mark.parametrize("n", [(9, 8), (5, 6, 4)])
def test_adjoint_sensitivity_matches_finite_differences(n):
    """A point-weighted objective does depend on nu; the adjoint derivative
    matches central differences of separate solves, and u (hence O) does not
    depend on E because K and f both scale with it."""
    rng = np.random.default_rng(3)
    base = dict(h=2.0, m=0.01, a=6.0, l=0.6)
    E, nu = 22.5, 0.3
    p = oracle.ElasticProblem(n, E=E, nu=nu, **base)
    g = rng.standard_normal(p.ndof)
    O, dE, dnu, _, ok = oracle.el_sensitivity(p, g=g, rtol=1e-14)
    assert ok

    def obj(E_, nu_):
        q = oracle.ElasticProblem(n, E=E_, nu=nu_, **base)
        return oracle.el_sensitivity(q, g=g, rtol=1e-14)[0]

    d = 1e-4
    fd_nu = (obj(E, nu + d) - obj(E, nu - d)) / (2 * d)
    fd_E = (obj(E + d, nu) - obj(E - d, nu)) / (2 * d)
    assert abs(dnu) > 1e-4 * abs(O)
    assert dnu == pytest.approx(fd_nu, rel=1e-6)
    assert abs(dE) < 1e-10 * abs(O) and abs(fd_E) < 1e-8 * abs(O)


def _interior_strain(p):
    u, it = oracle.el_solve(p, rtol=1e-12)
    assert it > 0
    # eps_xx at the corner node (centre of the full symmetric inclusion): one-sided
    # difference of u_x along x, exact for the fields near the centre (u_x ~ A x)
    return u[1] / p.h


def test_eshelby_circular_inclusion_plane_strain():
    """Plane strain, in-plane dilatational eigenstrain e0 in a circle of radius a
    in a large body: the inclusion strains uniformly by e0 (lam + mu)/(lam + 2 mu)
    = e0 / (2 (1 - nu)) (Eshelby).  A 40x40-element quarter body with a = 8 h
    and a sharp interface reproduces it to within 2 %."""
    nu = 0.3
    p = oracle.ElasticProblem((41, 41), h=1.0, E=22.5, nu=nu, m=0.01, a=8.0, l=4.0)
    A = _interior_strain(p)
    ref = 0.01 / (2 * (1 - nu))
    assert A == pytest.approx(ref, rel=0.02)


def test_eshelby_spherical_inclusion():
    """Sphere with dilatational eigenstrain e0: uniform interior strain
    e0 (1 + nu) / (3 (1 - nu)) (Eshelby), to within 3 % on a 16^3-element octant."""
    nu = 0.3
    p = oracle.ElasticProblem((17, 17, 17), h=1.0, E=22.5, nu=nu, m=0.01, a=5.0, l=4.0)
    A = _interior_strain(p)
    ref = 0.01 * (1 + nu) / (3 * (1 - nu))
    assert A == pytest.approx(ref, rel=0.03)
