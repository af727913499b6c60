"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects malformed requests before touching a GPU."""
import ctypes as ct

import pytest

from paper_2601_06079_amd import _abi as A


@pytest.fixture(scope="module")
def L():
    return A.lib()


@pytest.fixture(scope="module")
def C(L):
    """A host-only context: sizing and validation, no device needed."""
    h = ct.c_void_p()
    assert L.pf_create(A.HOST_ONLY, ct.byref(h)) == A.PF_OK and h.value
    yield h
    assert L.pf_destroy(h) == A.PF_OK


def _prob(**kw):
    d = dict(dim=2, bc=A.PERIODIC, model=A.CAHN_HILLIARD, fe=A.F_01, dtype=A.F32, mass=0,
             n=(64, 48, 1), h=1.0, W=1.0, kappa=2.0, mobility=1.0)
    d.update(kw)
    return A.pf_problem(d["dim"], d["bc"], d["model"], d["fe"], d["dtype"], d["mass"],
                        (ct.c_int64 * 3)(*d["n"]), d["h"], d["W"], d["kappa"], d["mobility"])


def test_exports_every_declared_symbol(L):
    names = A.exported_symbols()
    assert "pf_step_explicit" in names and "pf_newton_step" in names and "pf_vjp" in names
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_version(L):
    assert L.pf_version() >= 200


def test_context_lifecycle(L):
    """pf_create / pf_destroy: a host-only context reports no device and refuses to
    enqueue work; a device that does not exist is an error, not a crash."""
    h = ct.c_void_p()
    assert L.pf_create(A.HOST_ONLY, ct.byref(h)) == A.PF_OK
    d = ct.c_int(7)
    assert L.pf_ctx_device(h, ct.byref(d)) == A.PF_OK and d.value == A.HOST_ONLY
    p = _prob()
    fake = [ct.c_void_p(0x1000 * (i + 1)) for i in range(3)]
    assert L.pf_residual(h, ct.byref(p), fake[0], fake[1], None, None) == A.PF_EINVAL
    assert b"host-only" in L.pf_last_error()
    assert L.pf_destroy(h) == A.PF_OK
    assert L.pf_destroy(None) == A.PF_OK
    assert L.pf_create(-5, ct.byref(h)) == A.PF_EINVAL and not h.value
    assert L.pf_create(1 << 20, ct.byref(h)) == A.PF_EDEVICE and not h.value
    assert L.pf_create(0, None) == A.PF_EINVAL
    # every call that takes a context rejects NULL
    nb = ct.c_size_t(0)
    assert L.pf_workspace_size(None, ct.byref(p), A.OP_STEP_EXPLICIT, ct.byref(nb)) == A.PF_EINVAL
    assert b"ctx" in L.pf_last_error()
    assert L.pf_step_explicit(None, ct.byref(p), 0.01, 1, fake[0], fake[1], None) == A.PF_EINVAL


def test_oversized_batch_is_an_error(L, C):
    """A batch count beyond PF_BATCH_MAX_COUNT is rejected before any sample is read
    or any host table is sized from it."""
    from paper_2601_06079_amd import batch as B
    B._bind()
    base = _prob(model=A.ALLEN_CAHN, fe=A.F_SYM)
    one = (A.pf_batch_sample * 1)(A.pf_batch_sample(0, (ct.c_int64 * 3)(64, 64, 1), 1.0, 1.0, 1.0, 1.0))
    nb = ct.c_size_t(0)
    assert L.pf_batch_plan_size(ct.byref(base), one, 1, 2, 16, ct.byref(nb)) == A.PF_OK
    for count in (A.BATCH_MAX_COUNT + 1, 2 ** 31 - 1):
        assert L.pf_batch_plan_size(ct.byref(base), one, count, 2, 16, ct.byref(nb)) == A.PF_EINVAL
        info = A.pf_batch_info()
        assert L.pf_batch_plan(C, ct.byref(base), one, count, 0.05, 2, 16, 4, ct.c_void_p(0x1000), 1 << 20,
                               ct.byref(info), None) == A.PF_EINVAL
        assert b"PF_BATCH_MAX_COUNT" in L.pf_last_error()


@pytest.mark.parametrize("bad,status", [
    (dict(dim=4), A.PF_EINVAL), (dict(model=7), A.PF_EINVAL), (dict(fe=9), A.PF_EINVAL),
    (dict(dtype=3), A.PF_EINVAL), (dict(mass=2), A.PF_EINVAL), (dict(n=(1, 8, 1)), A.PF_EINVAL),
    (dict(h=0.0), A.PF_EINVAL), (dict(h=float("nan")), A.PF_EINVAL),
    (dict(kappa=float("inf")), A.PF_EINVAL), (dict(bc=5), A.PF_EINVAL)])
def test_problem_validation(L, C, bad, status):
    p = _prob(**bad)
    nb = ct.c_size_t(0)
    assert L.pf_workspace_size(C, ct.byref(p), A.OP_STEP_EXPLICIT, ct.byref(nb)) == status
    assert L.pf_last_error()  # a message is set


def test_argument_validation_before_launch(L, C):
    p = _prob()
    fake = ct.c_void_p(0x1000)  # never dereferenced: every call below fails validation first
    assert L.pf_residual(C, ct.byref(p), None, fake, None, None) == A.PF_EINVAL
    assert L.pf_residual(C, ct.byref(p), fake, fake, None, None) == A.PF_EINVAL  # aliasing
    assert L.pf_residual(C, ct.byref(p), ct.c_void_p(0x1002), ct.c_void_p(0x2000), None, None) == A.PF_EINVAL
    assert L.pf_step_explicit(C, ct.byref(p), 0.0, 1, fake, fake, None) == A.PF_EINVAL
    assert L.pf_step_explicit(C, ct.byref(p), 0.01, -1, fake, fake, None) == A.PF_EINVAL
    assert L.pf_step_explicit(C, ct.byref(p), float("nan"), 1, fake, fake, None) == A.PF_EINVAL
    assert L.pf_jvp(C, ct.byref(p), -1.0, fake, ct.c_void_p(0x2000), ct.c_void_p(0x3000), None) == A.PF_EINVAL
    assert L.pf_energy(C, ct.byref(p), fake, None, fake, None) == A.PF_EINVAL
    assert b"NULL" in L.pf_last_error()
    tb = (ct.c_double * 3)()
    f2, f3, f4 = ct.c_void_p(0x2000), ct.c_void_p(0x3000), ct.c_void_p(0x4000)
    # the backward-Euler residual's VJP (U_old given) needs dt > 0; unknown flags
    assert L.pf_vjp(C, ct.byref(p), A.VJP_RESIDUAL, 0.0, fake, f2, f3, f4, tb, 0, ct.c_void_p(0x5000),
                    None) == A.PF_EINVAL
    assert L.pf_vjp(C, ct.byref(p), A.VJP_RESIDUAL, 0.1, fake, None, f3, f4, tb, 8, ct.c_void_p(0x5000),
                    None) == A.PF_EINVAL


def test_workspace_sizes(L, C):
    p = _prob()
    nb = ct.c_size_t(0)
    assert L.pf_workspace_size(C, ct.byref(p), A.OP_STEP_EXPLICIT, ct.byref(nb)) == A.PF_OK
    assert nb.value == 64 * 48 * 4
    assert L.pf_workspace_size(C, ct.byref(p), A.OP_RESIDUAL, ct.byref(nb)) == A.PF_OK
    assert nb.value == 0
    assert L.pf_workspace_size(C, ct.byref(p), A.OP_ENERGY, ct.byref(nb)) == A.PF_OK
    assert nb.value >= 16
    assert L.pf_workspace_size(C, ct.byref(p), 99, ct.byref(nb)) == A.PF_EINVAL


def test_tuning_roundtrip(L):
    v = ct.c_int(-1)
    assert L.pf_tune_set(A.TUNE_STREAM2D_ROWS, 48) == A.PF_OK
    assert L.pf_tune_get(A.TUNE_STREAM2D_ROWS, ct.byref(v)) == A.PF_OK and v.value == 48
    assert L.pf_tune_set(A.TUNE_STREAM2D_ROWS, 0) == A.PF_OK
    assert L.pf_tune_set(A.TUNE_STREAM2D_ROWS, -3) == A.PF_EINVAL
    assert L.pf_tune_set(77, 1) == A.PF_EINVAL
    # every declared key round-trips and resets to its default (0)
    for key in (A.TUNE_STREAM2D_DEPTH, A.TUNE_STREAM2D_FUSE, A.TUNE_JVP3D_PLANES, A.TUNE_STREAM2D_SEAM,
                A.TUNE_NN_GROUP, A.TUNE_GS_REORTH, A.TUNE_GG_STREAM, A.TUNE_JVP2D_STREAM):
        assert L.pf_tune_set(key, 3) == A.PF_OK
        assert L.pf_tune_get(key, ct.byref(v)) == A.PF_OK and v.value == 3
        assert L.pf_tune_set(key, 0) == A.PF_OK


def test_launch_shape_defaults(L, C):
    """The default fused plan of the 2048^2 Cahn-Hilliard benchmark: three steps per
    launch, chunks for just under four waves per SIMD in whole workgroups of four
    (host-only context: 256 CUs)."""
    p = A.pf_problem(2, A.PERIODIC, A.CAHN_HILLIARD, A.F_01, A.F32, 0, (ct.c_int64 * 3)(2048, 2048, 1),
                     1.0, 1.0, 2.0, 1.0, 0.0, 1, 0, 1.5)
    ks, ty, dp = ct.c_int(), ct.c_int(), ct.c_int()
    assert L.pf_launch_shape(C, ct.byref(p), ct.byref(ks), ct.byref(ty), ct.byref(dp)) == A.PF_OK
    assert (ks.value, ty.value, dp.value) == (3, 21, 4)
    p.quad = A.QUAD_LOBATTO  # nodal quadrature: four steps, 43 strips x 92 chunks of 23 rows
    assert L.pf_launch_shape(C, ct.byref(p), ct.byref(ks), ct.byref(ty), ct.byref(dp)) == A.PF_OK
    assert (ks.value, ty.value) == (4, 23)
    p.quad = A.QUAD_GAUSS
    p.model = A.ALLEN_CAHN  # Allen-Cahn: four steps, 37 strips x 108 chunks of 19 rows
    assert L.pf_launch_shape(C, ct.byref(p), ct.byref(ks), ct.byref(ty), ct.byref(dp)) == A.PF_OK
    assert (ks.value, ty.value) == (4, 19)


def test_noflux_problem_accepted(L, C):
    """No-flux grids are valid single-problem input (batches stay periodic-only)."""
    p = _prob(bc=A.NOFLUX)
    nb = ct.c_size_t(0)
    assert L.pf_workspace_size(C, ct.byref(p), A.OP_STEP_EXPLICIT, ct.byref(nb)) == A.PF_OK


def test_coupled_model_entry_points(L, C):
    """The coupled model: residual, explicit steps and energy; the rest is rejected."""
    p = _prob(model=A.COUPLED)
    nb = ct.c_size_t(0)
    assert L.pf_workspace_size(C, ct.byref(p), A.OP_STEP_EXPLICIT, ct.byref(nb)) == A.PF_OK
    assert nb.value == 2 * 64 * 48 * 4  # two ping-pong fields (c, eta)
    assert L.pf_workspace_size(C, ct.byref(p), A.OP_NEWTON, ct.byref(nb)) == A.PF_OK
    assert L.pf_workspace_size(C, ct.byref(p), A.OP_VJP, ct.byref(nb)) == A.PF_EUNSUPPORTED
    fake = [ct.c_void_p(0x1000 * (i + 1)) for i in range(4)]
    tb = (ct.c_double * 3)()
    assert L.pf_vjp(C, ct.byref(p), A.VJP_RESIDUAL, 0.1, fake[0], None, fake[1], fake[2], tb, 0, fake[3],
                    None) == A.PF_EUNSUPPORTED
    q = _prob(model=A.COUPLED, fe=9)  # the coupled model ignores fe
    assert L.pf_workspace_size(C, ct.byref(q), A.OP_RESIDUAL, ct.byref(nb)) == A.PF_OK


def _el(**kw):
    from paper_2601_06079_amd import elastic as EL
    d = dict(dim=3, dtype=A.F32, n=(9, 8, 7), h=1.0, E=22.5, nu=0.3, m=0.01, a=3.0, l=0.5)
    d.update(kw)
    return EL.pf_elastic(d["dim"], d["dtype"], (ct.c_int64 * 3)(*d["n"]), d["h"], d["E"], d["nu"],
                         d["m"], d["a"], d["l"])


def test_elastic_validation_before_launch(L, C):
    """The elasticity entry points (Eshelby inclusion) reject malformed problems
    and arguments before anything is enqueued."""
    from paper_2601_06079_amd import elastic as EL
    EL._lib()
    nb = ct.c_size_t(0)
    p = _el()
    assert L.pf_el_workspace_size(C, ct.byref(p), ct.byref(nb)) == A.PF_OK
    vec = 9 * 8 * 7 * 3 * 4
    assert nb.value >= 7 * vec
    for bad in (dict(dim=1), dict(dtype=4), dict(n=(1, 8, 7)), dict(h=0.0), dict(E=-1.0),
                dict(nu=0.5), dict(nu=-1.0), dict(m=float("nan")), dict(l=float("inf"))):
        assert L.pf_el_workspace_size(C, ct.byref(_el(**bad)), ct.byref(nb)) == A.PF_EINVAL, bad
    fake, fake2 = ct.c_void_p(0x1000), ct.c_void_p(0x2000)
    assert L.pf_el_apply(C, ct.byref(p), fake, fake, None) == A.PF_EINVAL  # aliasing
    assert L.pf_el_apply(C, ct.byref(p), ct.c_void_p(0x1004), fake2, None) == A.PF_EINVAL  # alignment
    assert L.pf_el_apply(C, ct.byref(p), None, fake2, None) == A.PF_EINVAL
    rep = EL.pf_el_report()
    assert L.pf_el_solve(C, ct.byref(p), None, fake, 0.0, 10, ct.byref(rep), fake2, None) == A.PF_EINVAL
    assert L.pf_el_solve(C, ct.byref(p), None, fake, 1e-6, 0, ct.byref(rep), fake2, None) == A.PF_EINVAL
    assert L.pf_el_solve(C, ct.byref(p), None, fake, 1e-6, 10, ct.byref(rep), ct.c_void_p(0x2010),
                         None) == A.PF_EINVAL  # workspace alignment
    out = (ct.c_double * 3)()
    assert L.pf_el_sensitivity(C, ct.byref(p), None, fake, None, 1e-6, 10, None, fake2, None) == A.PF_EINVAL
    assert L.pf_el_objective(C, ct.byref(p), None, fake, None, fake2, None) == A.PF_EINVAL
    assert L.pf_el_sensitivity(C, ct.byref(_el(E=0.0)), None, fake, out, 1e-6, 10, None, fake2,
                               None) == A.PF_EINVAL
    v = ct.c_int(-1)
    assert L.pf_tune_set(EL.TUNE_EL_PLANES, 12) == A.PF_OK
    assert L.pf_tune_get(EL.TUNE_EL_PLANES, ct.byref(v)) == A.PF_OK and v.value == 12
    assert L.pf_tune_set(EL.TUNE_EL_PLANES, 0) == A.PF_OK


def _grain(**kw):
    d = dict(dim=2, bc=A.PERIODIC, model=A.GRAIN, fe=0, dtype=A.F32, mass=0, n=(40, 30, 1), h=1.0,
             W=0.0, kappa=1.0, mobility=1.0, mobility_eta=0.0, nfields=6, quad=0, gamma=1.5)
    d.update(kw)
    return A.pf_problem(d["dim"], d["bc"], d["model"], d["fe"], d["dtype"], d["mass"],
                        (ct.c_int64 * 3)(*d["n"]), d["h"], d["W"], d["kappa"], d["mobility"],
                        d["mobility_eta"], d["nfields"], d["quad"], d["gamma"])


def test_grain_model_entry_points(L, C):
    """Grain growth: the explicit workspace holds all order parameters; the implicit
    path takes at most 24 order parameters (FP32); adjoints are rejected before
    anything is enqueued."""
    nb = ct.c_size_t(0)
    p = _grain()
    assert L.pf_workspace_size(C, ct.byref(p), A.OP_STEP_EXPLICIT, ct.byref(nb)) == A.PF_OK
    assert nb.value == 6 * 40 * 30 * 4
    assert L.pf_workspace_size(C, ct.byref(p), A.OP_NEWTON, ct.byref(nb)) == A.PF_OK
    assert L.pf_workspace_size(C, ct.byref(_grain(nfields=25)), A.OP_NEWTON, ct.byref(nb)) == A.PF_EUNSUPPORTED
    assert L.pf_workspace_size(C, ct.byref(p), A.OP_VJP, ct.byref(nb)) == A.PF_EUNSUPPORTED
    for bad, st in ((dict(nfields=0), A.PF_EINVAL), (dict(nfields=33), A.PF_EINVAL),
                    (dict(dtype=A.F64, nfields=13), A.PF_EINVAL), (dict(gamma=float("nan")), A.PF_EINVAL),
                    (dict(quad=2), A.PF_EINVAL), (dict(quad=1), A.PF_EUNSUPPORTED),
                    (dict(dim=3, n=(8, 8, 8)), A.PF_EUNSUPPORTED),
                    (dict(mass=1), A.PF_EUNSUPPORTED)):
        assert L.pf_workspace_size(C, ct.byref(_grain(**bad)), A.OP_RESIDUAL, ct.byref(nb)) == st, bad
    fake = [ct.c_void_p(0x1000 * (i + 1)) for i in range(4)]
    assert L.pf_jvp(C, ct.byref(_grain(nfields=25)), 1.0, fake[0], fake[1], fake[2], None) == A.PF_EUNSUPPORTED
    tb = (ct.c_double * 3)()
    assert L.pf_vjp(C, ct.byref(p), A.VJP_RESIDUAL, 0.1, fake[0], None, fake[1], fake[2], tb, 0, fake[3],
                    None) == A.PF_EUNSUPPORTED
