"""FP64 CPU oracle for the phase-field FEM step -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never does, and this
package never imports the product library: the two share no code.

The arithmetic lives in ``pf_oracle.c`` (a plain Q1 element loop, built with
``gcc -O2 -ffp-contract=off``); this module only marshals NumPy float64 arrays
into it.  See the header of ``pf_oracle.c`` for what each routine follows in
the paper (Eqs. 1, 5-6, 9-14, 18 and Supplementary Note 2).
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SO_OMP = os.path.join(_HERE, "liboracle_omp.so")  # timing build (benchmark CPU baseline only)
_SRC = [os.path.join(_HERE, "pf_oracle.c"), os.path.join(_HERE, "conv_oracle.c"),
        os.path.join(_HERE, "coupled_oracle.c"), os.path.join(_HERE, "elastic_oracle.c"),
        os.path.join(_HERE, "grain_oracle.c")]

PERIODIC, NOFLUX = 0, 1
AC, CH = 0, 1
F_SYM, F_01 = 0, 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math, no FMA contraction), and the
    timing build of its explicit step (OpenMP over element colours, -DORC_OMP) that
    only the benchmark's CPU baseline loads."""
    if not force and os.path.exists(_SO):
        return _SO
    srcs = [s for s in _SRC if os.path.exists(s)]
    base = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99", "-shared", "-fPIC"]
    subprocess.run(base + ["-o", _SO + ".tmp"] + srcs + ["-lm"], check=True)
    os.replace(_SO + ".tmp", _SO)
    subprocess.run(base + ["-fopenmp", "-DORC_OMP", "-o", _SO_OMP + ".tmp", _SRC[0], "-lm"], check=True)
    os.replace(_SO_OMP + ".tmp", _SO_OMP)
    return _SO


class _Problem(ct.Structure):
    _fields_ = [("dim", ct.c_int32), ("bc", ct.c_int32), ("model", ct.c_int32),
                ("fe", ct.c_int32), ("n", ct.c_int64 * 3), ("h", ct.c_double),
                ("W", ct.c_double), ("kappa", ct.c_double), ("mob", ct.c_double),
                ("mass", ct.c_int32), ("quad", ct.c_int32)]


LUMPED, CONSISTENT = 0, 1
GAUSS, LOBATTO = 0, 1  # 2-point Gauss-Legendre or Gauss-Lobatto (nodal) quadrature per axis


@dataclass
class Problem:
    """Problem statement: grid, boundary condition, model, free energy, theta."""
    n: tuple
    model: int = AC
    fe: int = F_SYM
    bc: int = PERIODIC
    h: float = 1.0
    W: float = 1.0
    kappa: float = 1.0
    mob: float = 1.0
    mass: int = LUMPED  # CONSISTENT: Gauss-integrated mass in the implicit path
    quad: int = GAUSS  # LOBATTO: nodal quadrature for every integral

    @property
    def dim(self) -> int:
        return len(self.n)

    @property
    def nnodes(self) -> int:
        return int(np.prod(self.n))

    @property
    def ndof(self) -> int:
        return (2 if self.model == CH else 1) * self.nnodes

    def _c(self) -> _Problem:
        n3 = list(self.n) + [1] * (3 - len(self.n))
        return _Problem(self.dim, self.bc, self.model, self.fe, (ct.c_int64 * 3)(*n3),
                        self.h, self.W, self.kappa, self.mob, self.mass, self.quad)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        _lib = ct.CDLL(_SO)
        P = ct.POINTER(_Problem)
        D = ct.POINTER(ct.c_double)
        i64, f64, i32 = ct.c_int64, ct.c_double, ct.c_int
        sig = {
            "orc_ndof": (i64, [P]),
            "orc_lumped_mass": (i32, [P, D]),
            "orc_energy": (f64, [P, D]),
            "orc_total_mass": (f64, [P, D]),
            "orc_residual": (i32, [P, D, D]),
            "orc_explicit": (i32, [P, f64, i64, D]),
            "orc_be_residual": (i32, [P, f64, D, D, D]),
            "orc_jvp": (i32, [P, f64, D, D, D]),
            "orc_jvp_t": (i32, [P, f64, D, D, D]),
            "orc_dr_dtheta": (i32, [P, D, D, D]),
            "orc_linear_solve": (i32, [P, f64, D, i32, D, D, i32, f64]),
            "orc_newton_be": (i32, [P, f64, D, D, f64, i32, i32, f64,
                                    ct.POINTER(ct.c_int), D]),
            "orc_explicit_adjoint": (i32, [P, f64, i64, D, D, D, D]),
            "orc_newton_adjoint": (i32, [P, f64, D, D, D, D, i32]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(_lib, name)
            fn.restype = res
            fn.argtypes = args
        if hasattr(_lib, "orc_nn"):
            _bind_conv(_lib)
        if hasattr(_lib, "orc_cp_residual"):
            _bind_coupled(_lib)
        if hasattr(_lib, "orc_el_apply"):
            _bind_elastic(_lib)
        if hasattr(_lib, "orc_gg_residual"):
            _bind_grain(_lib)
    return _lib


def _d(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ct.POINTER(ct.c_double))


def _arr(x, n=None) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).ravel())
    if n is not None and a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


def lumped_mass(p: Problem) -> np.ndarray:
    m = np.zeros(p.nnodes)
    lib().orc_lumped_mass(ct.byref(p._c()), _d(m))
    return m


def energy(p: Problem, U) -> float:
    U = _arr(U)
    return lib().orc_energy(ct.byref(p._c()), _d(U))


def total_mass(p: Problem, U) -> float:
    U = _arr(U)
    return lib().orc_total_mass(ct.byref(p._c()), _d(U))


def residual(p: Problem, U) -> np.ndarray:
    """r(U, theta) of Eq. 11 (no mass term; Cahn-Hilliard mu-row holds m mu - g(c))."""
    U = _arr(U, p.ndof)
    r = np.zeros(p.ndof)
    lib().orc_residual(ct.byref(p._c()), _d(U), _d(r))
    return r


def explicit(p: Problem, U, dt: float, nsteps: int) -> np.ndarray:
    """nsteps of the lumped-mass forward-Euler step (Eq. 12); returns a new array."""
    U = _arr(U, p.ndof).copy()
    if lib().orc_explicit(ct.byref(p._c()), dt, int(nsteps), _d(U)) != 0:
        raise ValueError("explicit steps need the lumped mass")
    return U


_lib_omp = None


def explicit_threaded(p: Problem, U, dt: float, nsteps: int):
    """`explicit` from the OpenMP timing build (element colours in parallel; the
    same arithmetic summed in another order).  For the benchmark's CPU baseline
    only, never for parity.  Returns (new array, threads used)."""
    global _lib_omp
    if _lib_omp is None:
        if not os.path.exists(_SO_OMP):
            build()
        L = ct.CDLL(_SO_OMP)
        L.orc_explicit.restype = ct.c_int
        L.orc_explicit.argtypes = [ct.POINTER(_Problem), ct.c_double, ct.c_int64, ct.POINTER(ct.c_double)]
        L.orc_threads.restype = ct.c_int
        L.orc_threads.argtypes = []
        _lib_omp = L
    U = _arr(U, p.ndof).copy()
    if _lib_omp.orc_explicit(ct.byref(p._c()), dt, int(nsteps), _d(U)) != 0:
        raise ValueError("explicit steps need the lumped mass")
    return U, int(_lib_omp.orc_threads())


def be_residual(p: Problem, dt: float, Uold, U) -> np.ndarray:
    Uold, U = _arr(Uold, p.ndof), _arr(U, p.ndof)
    R = np.zeros(p.ndof)
    lib().orc_be_residual(ct.byref(p._c()), dt, _d(Uold), _d(U), _d(R))
    return R


def jvp(p: Problem, inv_dt: float, U, v) -> np.ndarray:
    U, v = _arr(U, p.ndof), _arr(v, p.ndof)
    out = np.zeros(p.ndof)
    lib().orc_jvp(ct.byref(p._c()), inv_dt, _d(U), _d(v), _d(out))
    return out


def jvp_t(p: Problem, inv_dt: float, U, w) -> np.ndarray:
    U, w = _arr(U, p.ndof), _arr(w, p.ndof)
    out = np.zeros(p.ndof)
    lib().orc_jvp_t(ct.byref(p._c()), inv_dt, _d(U), _d(w), _d(out))
    return out


def dr_dtheta(p: Problem, U, w) -> np.ndarray:
    """w^T dr/dtheta for theta = (mobility, kappa, W)."""
    U, w = _arr(U, p.ndof), _arr(w, p.ndof)
    g = np.zeros(3)
    lib().orc_dr_dtheta(ct.byref(p._c()), _d(U), _d(w), _d(g))
    return g


def linear_solve(p: Problem, inv_dt: float, U, b, transpose=False, solver=0, lin_rtol=1e-13):
    U, b = _arr(U, p.ndof), _arr(b, p.ndof)
    x = np.zeros(p.ndof)
    lib().orc_linear_solve(ct.byref(p._c()), inv_dt, _d(U), int(transpose), _d(b), _d(x),
                           int(solver), lin_rtol)
    return x


def newton_be(p: Problem, dt: float, Uold, U0=None, rtol=1e-8, maxit=20, solver=0,
              lin_rtol=1e-12):
    """One backward-Euler step by Newton (Eqs. 13-14). Returns (U, converged, its, hist)."""
    Uold = _arr(Uold, p.ndof)
    U = (Uold if U0 is None else _arr(U0, p.ndof)).copy()
    hist = np.zeros(maxit + 1)
    its = ct.c_int(0)
    rc = lib().orc_newton_be(ct.byref(p._c()), dt, _d(Uold), _d(U), rtol, maxit, solver,
                             lin_rtol, ct.byref(its), _d(hist))
    return U, rc == 0, its.value, hist[: its.value + 1]


def explicit_adjoint(p: Problem, dt: float, nsteps: int, U0, gU):
    """Discrete adjoint of `explicit`: returns (theta_bar[3], U0_bar)."""
    U0 = _arr(U0, p.ndof)
    gU = _arr(gU)
    tb = np.zeros(3)
    ub = np.zeros(p.nnodes)
    if lib().orc_explicit_adjoint(ct.byref(p._c()), dt, int(nsteps), _d(U0), _d(gU), _d(tb),
                                  _d(ub)) != 0:
        raise ValueError("explicit steps need the lumped mass")
    return tb, ub


def newton_adjoint(p: Problem, dt: float, U, gU, solver=0):
    """Adjoint of one BE step at its root U: returns (theta_bar[3], Uold_bar)."""
    U, gU = _arr(U, p.ndof), _arr(gU, p.ndof)
    tb = np.zeros(3)
    ub = np.zeros(p.ndof)
    lib().orc_newton_adjoint(ct.byref(p._c()), dt, _d(U), _d(gU), _d(ub), _d(tb), int(solver))
    return tb, ub


def _bind_conv(L):
    D = ct.POINTER(ct.c_double)
    L.orc_bf16.restype = ct.c_double
    L.orc_bf16.argtypes = [ct.c_double]
    L.orc_nn_nparams.restype = ct.c_int64
    L.orc_nn_nparams.argtypes = []
    L.orc_nn.restype = ct.c_double
    L.orc_nn.argtypes = [ct.c_int, ct.c_int, ct.c_int, D, D, D, D, D, ct.c_int, D, D]
    L.orc_adam.restype = None
    L.orc_adam.argtypes = [ct.c_int64, D, D, D, D, ct.c_double, ct.c_double, ct.c_double,
                           ct.c_double, ct.c_int]


def bf16(x: float) -> float:
    """Round to the nearest bfloat16, ties to even."""
    return lib().orc_bf16(float(x))


def nn_nparams() -> int:
    return int(lib().orc_nn_nparams())


NN_LAYOUT = [("W1", (3, 3, 3, 32)), ("b1", (32,)), ("W2", (3, 3, 32, 32)), ("b2", (32,)),
             ("W3", (3, 3, 32, 32)), ("b3", (32,)), ("W4", (3, 3, 32, 1)), ("b4", (1,))]


def nn(c, M, kappa, params, target=None, round_bf16=True, grad=False):
    """Surrogate forward (and parameter gradient of the loss). Arrays [B, H, W].
    Returns (c_hat, loss, grad or None)."""
    c = np.ascontiguousarray(c, dtype=np.float64)
    B, H, W = c.shape
    M = np.ascontiguousarray(np.broadcast_to(M, c.shape), dtype=np.float64)
    kap = np.ascontiguousarray(np.broadcast_to(kappa, c.shape), dtype=np.float64)
    p = _arr(params, nn_nparams())
    chat = np.zeros_like(c)
    t = None if target is None else np.ascontiguousarray(target, dtype=np.float64)
    g = np.zeros(nn_nparams()) if grad else None
    loss = lib().orc_nn(B, H, W, _d(c), _d(M), _d(kap), _d(t) if t is not None else None, _d(p),
                        int(round_bf16), _d(chat), _d(g) if g is not None else None)
    return chat, loss, g


def adam(p, m, v, g, lr, b1, b2, eps, t):
    """One bias-corrected Adam step in place on FP64 arrays p, m, v."""
    for a in (p, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = _arr(g, p.size)
    lib().orc_adam(p.size, _d(p), _d(m), _d(v), _d(g), lr, b1, b2, eps, int(t))


# ---------------------------------------------------------------------------
# Coupled Allen-Cahn / Cahn-Hilliard model (Eq. 7 with the polynomials of
# Supplementary Note 3); states are [c ; mu ; eta].  See coupled_oracle.c.
class _CpProblem(ct.Structure):
    _fields_ = [("dim", ct.c_int32), ("bc", ct.c_int32), ("n", ct.c_int64 * 3), ("h", ct.c_double),
                ("Mc", ct.c_double), ("Meta", ct.c_double), ("kappa", ct.c_double)]


@dataclass
class CoupledProblem:
    n: tuple
    bc: int = PERIODIC
    h: float = 1.0
    Mc: float = 1.0
    Meta: float = 150.0
    kappa: float = 0.3

    @property
    def dim(self) -> int:
        return len(self.n)

    @property
    def nnodes(self) -> int:
        return int(np.prod(self.n))

    @property
    def ndof(self) -> int:
        return 3 * self.nnodes

    def _c(self) -> _CpProblem:
        n3 = list(self.n) + [1] * (3 - len(self.n))
        return _CpProblem(self.dim, self.bc, (ct.c_int64 * 3)(*n3), self.h, self.Mc, self.Meta,
                          self.kappa)


def _bind_coupled(L):
    P = ct.POINTER(_CpProblem)
    D = ct.POINTER(ct.c_double)
    f64 = ct.c_double
    for name in ("orc_cp_fa", "orc_cp_dfa", "orc_cp_fb", "orc_cp_dfb", "orc_cp_h", "orc_cp_dh",
                 "orc_cp_d2fa", "orc_cp_d2fb", "orc_cp_d2h"):
        fn = getattr(L, name)
        fn.restype, fn.argtypes = f64, [f64]
    for name, res, args in (("orc_cp_lumped_mass", ct.c_int, [P, D]),
                            ("orc_cp_residual", ct.c_int, [P, D, D]),
                            ("orc_cp_explicit", ct.c_int, [P, f64, ct.c_int64, D]),
                            ("orc_cp_energy", f64, [P, D]),
                            ("orc_cp_total_mass", f64, [P, D]),
                            ("orc_cp_be_residual", ct.c_int, [P, f64, D, D, D]),
                            ("orc_cp_jvp", ct.c_int, [P, f64, D, D, D]),
                            ("orc_cp_newton_be", ct.c_int, [P, f64, D, D, f64, ct.c_int,
                                                            ct.POINTER(ct.c_int)])):
        fn = getattr(L, name)
        fn.restype, fn.argtypes = res, args


def cp_poly(name: str, x: float) -> float:
    """The benchmark polynomials: fa, dfa, d2fa, fb, dfb, d2fb, h, dh, d2h."""
    return getattr(lib(), "orc_cp_" + name)(float(x))


def cp_lumped_mass(p: CoupledProblem) -> np.ndarray:
    m = np.zeros(p.nnodes)
    lib().orc_cp_lumped_mass(ct.byref(p._c()), _d(m))
    return m


def cp_residual(p: CoupledProblem, U) -> np.ndarray:
    U = _arr(U, p.ndof)
    r = np.zeros(p.ndof)
    lib().orc_cp_residual(ct.byref(p._c()), _d(U), _d(r))
    return r


def cp_explicit(p: CoupledProblem, U, dt: float, nsteps: int) -> np.ndarray:
    U = _arr(U, p.ndof).copy()
    lib().orc_cp_explicit(ct.byref(p._c()), dt, int(nsteps), _d(U))
    return U


def cp_energy(p: CoupledProblem, U) -> float:
    U = _arr(U, p.ndof)
    return lib().orc_cp_energy(ct.byref(p._c()), _d(U))


def cp_total_mass(p: CoupledProblem, U) -> float:
    U = _arr(U)
    return lib().orc_cp_total_mass(ct.byref(p._c()), _d(U))


def cp_be_residual(p: CoupledProblem, dt: float, Uold, U) -> np.ndarray:
    Uold, U = _arr(Uold, p.ndof), _arr(U, p.ndof)
    R = np.zeros(p.ndof)
    lib().orc_cp_be_residual(ct.byref(p._c()), dt, _d(Uold), _d(U), _d(R))
    return R


def cp_jvp(p: CoupledProblem, inv_dt: float, U, v) -> np.ndarray:
    U, v = _arr(U, p.ndof), _arr(v, p.ndof)
    Jv = np.zeros(p.ndof)
    lib().orc_cp_jvp(ct.byref(p._c()), inv_dt, _d(U), _d(v), _d(Jv))
    return Jv


def cp_newton_be(p: CoupledProblem, dt: float, Uold, U0=None, rtol=1e-12, maxit=30):
    """One backward-Euler step by Newton with dense LU (small grids). Returns (U, converged, its)."""
    Uold = _arr(Uold, p.ndof)
    U = (Uold if U0 is None else _arr(U0, p.ndof)).copy()
    its = ct.c_int(0)
    rc = lib().orc_cp_newton_be(ct.byref(p._c()), dt, _d(Uold), _d(U), rtol, maxit, ct.byref(its))
    return U, rc == 0, its.value


# ---------------------------------------------------------------------------
# Eshelby inclusion: small-strain linear elasticity with a dilatational
# eigenstrain (Eqs. 3-4, Supplementary Note 3 Eq. III.1).  Displacements are
# [u_x ; u_y ; (u_z)].  See elastic_oracle.c.
class _ElProblem(ct.Structure):
    _fields_ = [("dim", ct.c_int32), ("sym", ct.c_int32), ("n", ct.c_int64 * 3), ("h", ct.c_double),
                ("E", ct.c_double), ("nu", ct.c_double), ("m", ct.c_double), ("a", ct.c_double),
                ("l", ct.c_double)]


@dataclass
class ElasticProblem:
    n: tuple
    h: float = 1.0
    E: float = 22.5
    nu: float = 0.3
    m: float = 0.01
    a: float = 20.0
    l: float = 0.5
    sym: int = 1

    @property
    def dim(self) -> int:
        return len(self.n)

    @property
    def nnodes(self) -> int:
        return int(np.prod(self.n))

    @property
    def ndof(self) -> int:
        return self.dim * self.nnodes

    def _c(self) -> _ElProblem:
        n3 = list(self.n) + [1] * (3 - len(self.n))
        return _ElProblem(self.dim, self.sym, (ct.c_int64 * 3)(*n3), self.h, self.E, self.nu,
                          self.m, self.a, self.l)


def _bind_elastic(L):
    P = ct.POINTER(_ElProblem)
    D = ct.POINTER(ct.c_double)
    f64, i32 = ct.c_double, ct.c_int
    for name, res, args in (("orc_el_eigen", f64, [P, f64]),
                            ("orc_el_free", i32, [P, ct.c_int64, i32]),
                            ("orc_el_apply", i32, [P, D, D]),
                            ("orc_el_rhs", i32, [P, D]),
                            ("orc_el_volume_weights", i32, [P, D]),
                            ("orc_el_solve", i32, [P, D, f64, i32]),
                            ("orc_el_sensitivity", i32, [P, D, f64, i32, D, D]),
                            ("orc_el_objective", f64, [P, D, D]),
                            ("orc_el_eigen_integral", f64, [P])):
        fn = getattr(L, name)
        fn.restype, fn.argtypes = res, args


def el_eigen(p: ElasticProblem, r: float) -> float:
    """The diagonal eigenstrain at distance r from the origin corner."""
    return lib().orc_el_eigen(ct.byref(p._c()), float(r))


def el_free_mask(p: ElasticProblem) -> np.ndarray:
    """1.0 where a displacement component is free, 0.0 where a symmetry plane fixes it."""
    L, c = lib(), p._c()
    return np.array([L.orc_el_free(ct.byref(c), a, comp) for comp in range(p.dim)
                     for a in range(p.nnodes)], dtype=np.float64)


def el_apply(p: ElasticProblem, u) -> np.ndarray:
    """K u with identity rows on the fixed components."""
    u = _arr(u, p.ndof)
    y = np.zeros(p.ndof)
    lib().orc_el_apply(ct.byref(p._c()), _d(u), _d(y))
    return y


def el_rhs(p: ElasticProblem) -> np.ndarray:
    f = np.zeros(p.ndof)
    lib().orc_el_rhs(ct.byref(p._c()), _d(f))
    return f


def el_volume_weights(p: ElasticProblem) -> np.ndarray:
    g = np.zeros(p.ndof)
    lib().orc_el_volume_weights(ct.byref(p._c()), _d(g))
    return g


def el_solve(p: ElasticProblem, rtol=1e-12, maxit=100000):
    """Equilibrium displacement by CG. Returns (u, iterations or -1)."""
    u = np.zeros(p.ndof)
    it = lib().orc_el_solve(ct.byref(p._c()), _d(u), rtol, maxit)
    return u, it


def el_sensitivity(p: ElasticProblem, g=None, rtol=1e-12, maxit=100000):
    """(O, dO/dE, dO/dnu, u, ok) for O = g . u (g = None: the volume change)."""
    out = np.zeros(3)
    u = np.zeros(p.ndof)
    gp = None if g is None else _d(_arr(g, p.ndof))
    rc = lib().orc_el_sensitivity(ct.byref(p._c()), gp, rtol, maxit, _d(out), _d(u))
    return out[0], out[1], out[2], u, rc == 0


def el_objective(p: ElasticProblem, u, g=None) -> float:
    u = _arr(u, p.ndof)
    gp = None if g is None else _d(_arr(g, p.ndof))
    return lib().orc_el_objective(ct.byref(p._c()), gp, _d(u))


def el_eigen_integral(p: ElasticProblem) -> float:
    return lib().orc_el_eigen_integral(ct.byref(p._c()))


# ---------------------------------------------------------------------------
# Multi-order-parameter Allen-Cahn (grain growth): p order parameters, states
# [eta_1 ; ... ; eta_p].  See grain_oracle.c.
class _GgProblem(ct.Structure):
    _fields_ = [("dim", ct.c_int32), ("bc", ct.c_int32), ("n", ct.c_int64 * 3), ("h", ct.c_double),
                ("L", ct.c_double), ("kappa", ct.c_double), ("gamma", ct.c_double),
                ("p", ct.c_int32), ("pad", ct.c_int32)]


@dataclass
class GrainProblem:
    n: tuple
    p: int = 4
    bc: int = PERIODIC
    h: float = 1.0
    L: float = 1.0
    kappa: float = 1.0
    gamma: float = 1.5

    @property
    def dim(self) -> int:
        return len(self.n)

    @property
    def nnodes(self) -> int:
        return int(np.prod(self.n))

    @property
    def ndof(self) -> int:
        return self.p * self.nnodes

    def _c(self) -> _GgProblem:
        n3 = list(self.n) + [1] * (3 - len(self.n))
        return _GgProblem(self.dim, self.bc, (ct.c_int64 * 3)(*n3), self.h, self.L, self.kappa,
                          self.gamma, self.p, 0)


def _bind_grain(L):
    P = ct.POINTER(_GgProblem)
    D = ct.POINTER(ct.c_double)
    for name, res, args in (("orc_gg_f", ct.c_double, [P, D]),
                            ("orc_gg_df", None, [P, D, D]),
                            ("orc_gg_lumped_mass", ct.c_int, [P, D]),
                            ("orc_gg_residual", ct.c_int, [P, D, D]),
                            ("orc_gg_explicit", ct.c_int, [P, ct.c_double, ct.c_int64, D]),
                            ("orc_gg_energy", ct.c_double, [P, D]),
                            ("orc_gg_be_residual", ct.c_int, [P, ct.c_double, D, D, D]),
                            ("orc_gg_jvp", ct.c_int, [P, ct.c_double, D, D, D]),
                            ("orc_gg_newton_be", ct.c_int, [P, ct.c_double, D, D, ct.c_double, ct.c_int,
                                                             ct.POINTER(ct.c_int)])):
        fn = getattr(L, name)
        fn.restype, fn.argtypes = res, args


def gg_f(p: GrainProblem, eta) -> float:
    eta = _arr(eta, p.p)
    return lib().orc_gg_f(ct.byref(p._c()), _d(eta))


def gg_df(p: GrainProblem, eta) -> np.ndarray:
    eta = _arr(eta, p.p)
    out = np.zeros(p.p)
    lib().orc_gg_df(ct.byref(p._c()), _d(eta), _d(out))
    return out


def gg_lumped_mass(p: GrainProblem) -> np.ndarray:
    m = np.zeros(p.nnodes)
    lib().orc_gg_lumped_mass(ct.byref(p._c()), _d(m))
    return m


def gg_residual(p: GrainProblem, U) -> np.ndarray:
    U = _arr(U, p.ndof)
    r = np.zeros(p.ndof)
    if lib().orc_gg_residual(ct.byref(p._c()), _d(U), _d(r)) != 0:
        raise ValueError("1 <= p <= 64 order parameters")
    return r


def gg_explicit(p: GrainProblem, U, dt: float, nsteps: int) -> np.ndarray:
    U = _arr(U, p.ndof).copy()
    if lib().orc_gg_explicit(ct.byref(p._c()), dt, int(nsteps), _d(U)) != 0:
        raise ValueError("1 <= p <= 64 order parameters")
    return U


def gg_energy(p: GrainProblem, U) -> float:
    U = _arr(U, p.ndof)
    return lib().orc_gg_energy(ct.byref(p._c()), _d(U))


def gg_be_residual(p: GrainProblem, dt: float, Uold, U) -> np.ndarray:
    Uold, U = _arr(Uold, p.ndof), _arr(U, p.ndof)
    R = np.zeros(p.ndof)
    lib().orc_gg_be_residual(ct.byref(p._c()), dt, _d(Uold), _d(U), _d(R))
    return R


def gg_jvp(p: GrainProblem, inv_dt: float, U, v) -> np.ndarray:
    U, v = _arr(U, p.ndof), _arr(v, p.ndof)
    Jv = np.zeros(p.ndof)
    lib().orc_gg_jvp(ct.byref(p._c()), inv_dt, _d(U), _d(v), _d(Jv))
    return Jv


def gg_newton_be(p: GrainProblem, dt: float, Uold, U0=None, rtol=1e-12, maxit=30):
    """One backward-Euler step by dense Newton (small grids). Returns (U, converged, its)."""
    Uold = _arr(Uold, p.ndof)
    U = (Uold if U0 is None else _arr(U0, p.ndof)).copy()
    its = ct.c_int(0)
    rc = lib().orc_gg_newton_be(ct.byref(p._c()), dt, _d(Uold), _d(U), rtol, maxit, ct.byref(its))
    return U, rc == 0, its.value
