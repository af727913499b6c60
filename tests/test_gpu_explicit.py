"""Parity of the HIP residual, Jacobian product, energy and explicit step with
the FP64 oracle, element by element, on seeded inputs."""
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
TOL_STEP = {F32: 1e-5, F64: 1e-12}

SHAPES_2D = [(2, 2), (3, 5), (64, 64), (130, 97), (61, 200)]
SHAPES_3D = [(2, 2, 2), (3, 4, 5), (17, 9, 12)]


def _rand_state(o, lo, hi, seed, base=0.0):
    c = I.uniform_field(o.n, lo, hi, seed=seed, base=base)
    if o.model == O.CH:
        mu = I.uniform_field(o.n, -0.5, 0.5, seed=seed + 1)
        return np.concatenate([c, mu])
    return c


@pytest.mark.parametrize("dtype", [F32, F64])
@pytest.mark.parametrize("model", [O.AC, O.CH])
@pytest.mark.parametrize("n", SHAPES_2D + SHAPES_3D)
def test_residual_parity(n, model, dtype):
    announce("residual", n, model, dtype)
    g, o = pair(n, model, O.F_01 if model == O.CH else O.F_SYM, dtype, h=0.7, W=1.3, kappa=0.9, mob=1.1)
    U = rounded(_rand_state(o, -1.0, 1.0, seed=3), dtype)
    r = host(S.residual(g, dev(U, dtype)))
    assert rel_l2(r, O.residual(o, U)) < TOL_STEP[dtype]


@pytest.mark.parametrize("dtype", [F32, F64])
@pytest.mark.parametrize("model", [O.AC, O.CH])
@pytest.mark.parametrize("n", [(5, 7), (96, 70), (3, 4, 5), (12, 10, 9)])
def test_jvp_parity(n, model, dtype):
    announce("jvp", n, model, dtype)
    g, o = pair(n, model, O.F_01, dtype, h=1.0, W=1.0, kappa=2.0, mob=0.8)
    U = rounded(_rand_state(o, 0.2, 0.8, seed=5), dtype)
    v = rounded(np.random.default_rng(9).standard_normal(o.ndof), dtype)
    for inv_dt in (0.0, 2.0):
        Jv = host(S.jvp(g, inv_dt, dev(U, dtype), dev(v, dtype)))
        assert rel_l2(Jv, O.jvp(o, inv_dt, U, v)) < TOL_STEP[dtype]


@pytest.mark.parametrize("dtype", [F32, F64])
@pytest.mark.parametrize("n,fe", [((7, 5), O.F_SYM), ((128, 96), O.F_01), ((4, 5, 6), O.F_01),
                                  ((20, 16, 12), O.F_SYM)])
def test_energy_parity(n, fe, dtype):
    announce("energy", n, fe, dtype)
    g, o = pair(n, O.AC, fe, dtype, h=0.8, W=1.2, kappa=1.7)
    U = rounded(I.uniform_field(n, -1, 1, seed=11), dtype)
    out = host(S.energy(g, dev(U, dtype)))
    assert out[0] == pytest.approx(O.energy(o, U), rel=1e-12)
    assert out[1] == pytest.approx(O.total_mass(o, U), rel=1e-12, abs=1e-12)


def _run_explicit(g, o, U0, dt, nsteps, dtype):
    Ug = dev(U0, dtype)
    S.step_explicit(g, Ug, dt, nsteps)
    return host(Ug), O.explicit(o, U0, dt, nsteps)


@pytest.mark.parametrize("dtype", [F32, F64])
@pytest.mark.parametrize("model", [O.AC, O.CH])
@pytest.mark.parametrize("n", SHAPES_2D + SHAPES_3D)
def test_explicit_one_step(n, model, dtype):
    announce("explicit-1", n, model, dtype)
    if model == O.AC:
        g, o = pair(n, O.AC, O.F_SYM, dtype, W=1.0, kappa=1.0, mob=1.0)
        U0 = rounded(_rand_state(o, -0.05, 0.05, 1), dtype)
        dt = 0.1
    else:
        g, o = pair(n, O.CH, O.F_01, dtype, W=1.0, kappa=2.0, mob=1.0)
        U0 = rounded(_rand_state(o, -0.01, 0.01, 2, base=0.5), dtype)
        dt = 0.01
    ug, uo = _run_explicit(g, o, U0, dt, 1, dtype)
    N = o.nnodes
    assert rel_l2(ug[:N], uo[:N]) < TOL_STEP[dtype]
    # the update itself (c_new - c_old), a far stricter measure than the field
    tol_upd = 2e-3 if dtype == F32 else 1e-9
    assert rel_l2(ug[:N] - U0[:N], uo[:N] - U0[:N]) < tol_upd
    if model == O.CH:  # mu plane = [N(c)+kappa K c]/m of the final c
        assert rel_l2(ug[N:], uo[N:]) < (1e-4 if dtype == F32 else 1e-11)


def test_allen_cahn_128_fp64_1000_steps():
    """Allen-Cahn 128x128 periodic, f=(c^2-1)^2/4, kappa=L=h=1, dt=0.1, FP64."""
    cfg = I.AC128
    announce("AC128 fp64 1000")
    g, o = pair(cfg["n"], O.AC, O.F_SYM, F64, W=1.0, kappa=1.0, mob=1.0)
    U0 = I.initial_state(cfg, seed=0)
    ug, uo = _run_explicit(g, o, U0, cfg["dt"], cfg["steps"], F64)
    assert rel_l2(ug, uo) < 1e-10


def test_allen_cahn_128_fp32_1000_steps():
    cfg = I.AC128
    announce("AC128 fp32 1000")
    g, o = pair(cfg["n"], O.AC, O.F_SYM, F32, W=1.0, kappa=1.0, mob=1.0)
    U0 = rounded(I.initial_state(cfg, seed=0), F32)
    ug, uo = _run_explicit(g, o, U0, cfg["dt"], 1, F32)
    assert rel_l2(ug, uo) < 1e-5
    ug, uo = _run_explicit(g, o, U0, cfg["dt"], cfg["steps"], F32)
    assert rel_l2(ug, uo) < 1e-3


@pytest.mark.parametrize("n,steps", [((128, 128), 1000), ((256, 192), 300)])
def test_cahn_hilliard_fp32_many_steps(n, steps):
    announce("CH fp32", n, steps)
    g, o = pair(n, O.CH, O.F_01, F32, W=1.0, kappa=2.0, mob=1.0)
    U0 = rounded(I.initial_state(dict(I.CH2048, n=n), seed=0), F32)
    ug, uo = _run_explicit(g, o, U0, 0.01, steps, F32)
    N = o.nnodes
    assert rel_l2(ug[:N], uo[:N]) < 1e-3
    # fluctuation about the mean, reported alongside (stricter than the field norm)
    assert rel_l2(ug[:N] - 0.5, uo[:N] - 0.5) < 2e-2


def test_cahn_hilliard_2048_full_size_one_step():
    """The benchmark workload at full size (2048^2, launch shape of the benchmark)."""
    cfg = I.CH2048
    announce("CH2048 fp32 one step")
    g, o = pair(cfg["n"], O.CH, O.F_01, F32, W=1.0, kappa=2.0, mob=1.0)
    U0 = rounded(I.initial_state(cfg, seed=0), F32)
    ug, uo = _run_explicit(g, o, U0, cfg["dt"], 1, F32)
    N = o.nnodes
    assert rel_l2(ug[:N], uo[:N]) < 1e-5
    assert rel_l2(ug[:N] - U0[:N], uo[:N] - U0[:N]) < 2e-3


def test_cahn_hilliard_2048_benchmark_plan_12_steps():
    """The benchmark's own launch plan at full size: 2048^2 with the default shape
    (three fused steps per launch on the seam-sharing kernel, balanced chunks), 12
    steps = 4 fused launches and the chemical-potential epilogue, element by element
    against the FP64 oracle.

    Tolerances: c to the benchmark spec's 1e-5 relative L2 (FP32 fields).  The mu plane
    is formed from 9 c - box(c) with c near 0.5, where FP32 cancellation leaves an
    absolute error of a few ulp(4.5) ~ 1e-6 against mu values of RMS ~ 3e-2, so mu is
    held to 1e-4.  The update c_n - c_0 (a far stricter measure: it removes the
    uniform 0.5) is held to 2e-3, as for one step."""
    cfg = I.CH2048
    announce("CH2048 fp32 benchmark plan, 12 steps")
    g, o = pair(cfg["n"], O.CH, O.F_01, F32, W=1.0, kappa=2.0, mob=1.0)
    ks, ty, depth = S.launch_shape(g)
    assert ks == 3 and _seam_plan_applies(cfg["n"], O.CH, ks, ty), (ks, ty, depth)  # the plan the benchmark times
    U0 = rounded(I.initial_state(cfg, seed=0), F32)
    ug, uo = _run_explicit(g, o, U0, cfg["dt"], 4 * ks, F32)
    N = o.nnodes
    assert rel_l2(ug[:N], uo[:N]) < 1e-5
    assert rel_l2(ug[N:], uo[N:]) < 1e-4
    assert rel_l2(ug[:N] - U0[:N], uo[:N] - U0[:N]) < 2e-3


def test_cahn_hilliard_2048_mass_and_energy_over_steps():
    cfg = I.CH2048
    announce("CH2048 invariants")
    g = S.Problem(n=cfg["n"], model=A.CAHN_HILLIARD, fe=A.F_01, dtype=F32, W=1.0, kappa=2.0,
                  mobility=1.0)
    U = dev(I.initial_state(cfg, seed=0, dtype=np.float32), F32)
    ws = S.workspace(g, A.OP_STEP_EXPLICIT)
    gE = S.Problem(n=cfg["n"], model=A.ALLEN_CAHN, fe=A.F_01, dtype=F32, W=1.0, kappa=2.0)
    e0 = host(S.energy(gE, U[: g.nnodes].contiguous()))
    S.step_explicit(g, U, cfg["dt"], 200, ws)
    e1 = host(S.energy(gE, U[: g.nnodes].contiguous()))
    assert abs(e1[1] - e0[1]) < 1e-6 * abs(e0[1])  # conserved
    assert e1[0] <= e0[0]  # energy decays


def test_explicit_deterministic_and_step_split():
    g, o = pair((300, 257), O.CH, O.F_01, F32, W=1.0, kappa=2.0, mob=1.0)
    U0 = I.initial_state(dict(I.CH2048, n=(300, 257)), seed=4, dtype=np.float32)
    a = dev(U0, F32)
    b = dev(U0, F32)
    c = dev(U0, F32)
    S.step_explicit(g, a, 0.01, 7)
    S.step_explicit(g, b, 0.01, 7)
    S.step_explicit(g, c, 0.01, 3)
    S.step_explicit(g, c, 0.01, 4)
    assert torch.equal(a, b)
    assert torch.equal(a[: g.nnodes], c[: g.nnodes])


def test_explicit_zero_steps_sets_mu():
    g, o = pair((40, 33), O.CH, O.F_01, F64, W=1.0, kappa=2.0, mob=1.0)
    U0 = _rand_state(o, -0.1, 0.1, 8, base=0.5)
    ug = dev(U0, F64)
    S.step_explicit(g, ug, 0.01, 0)
    u = host(ug)
    assert np.array_equal(u[: o.nnodes], U0[: o.nnodes])
    assert rel_l2(u[o.nnodes:], O.explicit(o, U0, 0.01, 0)[o.nnodes:]) < 1e-12


@pytest.mark.parametrize("rows", [8, 13, 64, 1000])
def test_explicit_launch_shapes_agree(rows):
    """Every launch shape gives bitwise the same field (arithmetic is per node)."""
    g, _ = pair((200, 150), O.CH, O.F_01, F32, W=1.0, kappa=2.0, mob=1.0)
    U0 = I.initial_state(dict(I.CH2048, n=(200, 150)), seed=6, dtype=np.float32)
    ref = dev(U0, F32)
    S.step_explicit(g, ref, 0.01, 5)
    try:
        S.tune_set(A.TUNE_STREAM2D_ROWS, rows)
        t = dev(U0, F32)
        S.step_explicit(g, t, 0.01, 5)
    finally:
        S.tune_set(A.TUNE_STREAM2D_ROWS, 0)
    assert torch.equal(ref, t)


def _fused_vs_single(g, U0, dt, nsteps, ks, dtype):
    """(single-step launches, launches fusing ks steps) from the same state."""
    out = []
    for fuse in (1, ks):
        try:
            S.tune_set(A.TUNE_STREAM2D_FUSE, fuse)
            t = dev(U0, dtype)
            S.step_explicit(g, t, dt, nsteps)
        finally:
            S.tune_set(A.TUNE_STREAM2D_FUSE, 0)
        out.append(t)
    return out


@pytest.mark.parametrize("ks", [2, 3, 4])
@pytest.mark.parametrize("dtype", [F32, F64])
@pytest.mark.parametrize("model,n", [(O.AC, (128, 128)), (O.CH, (200, 150)), (O.CH, (61, 37)),
                                     (O.AC, (5, 7)), (O.CH, (2048, 64))])
def test_explicit_temporal_blocking_bitwise(ks, dtype, model, n):
    """ks fused steps per launch give bitwise the field of ks single-step launches
    (the reference runs with fusion switched off)."""
    announce("fused", ks, dtype, model, n)
    fe = O.F_01 if model == O.CH else O.F_SYM
    g, o = pair(n, model, fe, dtype, W=1.0, kappa=2.0 if model == O.CH else 1.0, mob=1.0)
    base = 0.5 if model == O.CH else 0.0
    U0 = _rand_state(o, -0.05, 0.05, 12, base=base)
    dt = 0.01 if model == O.CH else 0.1
    ref, t = _fused_vs_single(g, U0, dt, 2 * ks + 1, ks, dtype)
    assert torch.equal(ref, t)


def _seam_plan_applies(n, model, ks, rows):
    """The chunk plan of the LDS seam-sharing fused kernel: chunks rounded to whole
    workgroups of 4, whose top chunk is H (ks - 1) rows shorter than the others; the
    shortest chunk long enough for the barrier."""
    H = 1 if model == O.AC else 2
    nch = -(-n[1] // rows)
    nch = -(-nch // 4) * 4
    first = -(-(2 * H * ks) // 4) * 4
    rmin = n[1] // (nch // 4)
    shortest = rmin - 3 * (rmin + H * (ks - 1)) // 4
    return shortest >= max(first + 4 - 2 * H, 8)


@pytest.mark.parametrize("dtype", [F32, F64])
@pytest.mark.parametrize("model,n,ks,rows", [(O.CH, (512, 600), 2, 19), (O.CH, (512, 600), 2, 40),
                                             (O.CH, (200, 333), 3, 24), (O.CH, (130, 640), 4, 32),
                                             (O.AC, (300, 512), 2, 12), (O.AC, (97, 401), 4, 24),
                                             (O.CH, (64, 97), 2, 25)])
def test_explicit_seam_kernel_bitwise(dtype, model, n, ks, rows):
    """Fused launches whose workgroups share the chunk seams through LDS (the plan
    applies to every case here): bitwise the single-step launches, and bitwise the
    fused kernel that recomputes the seams."""
    announce("seam", dtype, model, n, ks, rows)
    assert _seam_plan_applies(n, model, ks, rows)
    fe = O.F_01 if model == O.CH else O.F_SYM
    g, o = pair(n, model, fe, dtype, W=1.0, kappa=2.0 if model == O.CH else 1.0, mob=1.0)
    U0 = _rand_state(o, -0.05, 0.05, 31, base=0.5 if model == O.CH else 0.0)
    dt = 0.01 if model == O.CH else 0.1
    try:
        S.tune_set(A.TUNE_STREAM2D_ROWS, rows)
        S.tune_set(A.TUNE_STREAM2D_SEAM, 0)
        ref, t = _fused_vs_single(g, U0, dt, 3 * ks + 1, ks, dtype)
        assert torch.equal(ref, t)
        S.tune_set(A.TUNE_STREAM2D_SEAM, 1)
        _, t2 = _fused_vs_single(g, U0, dt, 3 * ks + 1, ks, dtype)
        assert torch.equal(t, t2)
    finally:
        S.tune_set(A.TUNE_STREAM2D_SEAM, 0)
        S.tune_set(A.TUNE_STREAM2D_ROWS, 0)


def test_explicit_temporal_blocking_bitwise_benchmark_shape():
    """The 2048^2 Cahn-Hilliard workload: its default fused plan against single-step
    launches, bitwise, over 6 steps (3 fused launches); the kernel that recomputes the
    seams on the same plan alike."""
    announce("fused 2048^2 vs single steps")
    cfg = I.CH2048
    g, o = pair(cfg["n"], O.CH, O.F_01, F32, W=1.0, kappa=2.0, mob=1.0)
    ks, rows, _ = S.launch_shape(g)
    assert ks >= 2 and _seam_plan_applies(cfg["n"], O.CH, ks, rows)
    U0 = I.initial_state(cfg, seed=1, dtype=np.float32)
    ref, t = _fused_vs_single(g, U0, cfg["dt"], 3 * ks, ks, F32)
    assert torch.equal(ref, t)
    try:  # the fused kernel that recomputes the seams gives the same bits
        S.tune_set(A.TUNE_STREAM2D_SEAM, 1)
        _, t2 = _fused_vs_single(g, U0, cfg["dt"], 3 * ks, ks, F32)
    finally:
        S.tune_set(A.TUNE_STREAM2D_SEAM, 0)
    assert torch.equal(t, t2)


@pytest.mark.parametrize("planes", [1, 3, 7, 40])
@pytest.mark.parametrize("model", [O.AC, O.CH])
def test_jvp3d_plane_counts_agree(planes, model):
    """The 3-D Jacobian product is bitwise independent of the z-planes per block."""
    announce("jvp3d planes", planes, model)
    g, o = pair((33, 17, 29), model, O.F_01, F32, h=1.0, W=1.0, kappa=2.0, mob=0.8)
    U = dev(_rand_state(o, 0.2, 0.8, seed=21), F32)
    v = dev(np.random.default_rng(22).standard_normal(o.ndof), F32)
    ref = S.jvp(g, 2.0, U, v)
    try:
        S.tune_set(A.TUNE_JVP3D_PLANES, planes)
        out = S.jvp(g, 2.0, U, v)
    finally:
        S.tune_set(A.TUNE_JVP3D_PLANES, 0)
    assert torch.equal(ref, out)
    assert rel_l2(host(out), O.jvp(o, 2.0, host(U).astype(np.float64), host(v).astype(np.float64))) < 1e-5


@pytest.mark.parametrize("reps", [181, 182])
def test_explicit_largest_fields_tiled(reps):
    """The largest 2-D fields: 23168^2 FP32 (2 147 024 896 bytes, the streaming
    kernel at the top of its 32-bit offset range) and 23296^2 (beyond 2 GiB: the
    node-centric path).  A periodic field that repeats a 128^2 pattern stays a
    repetition of it, so every node of the big result must equal the 128^2 oracle
    result tiled."""
    announce("CH largest fields, tiled", reps)
    p_small = 128
    n = p_small * reps
    assert (n * n * 4 < 2 ** 31) == (reps == 181)
    g, o = pair((p_small, p_small), O.CH, O.F_01, F32, W=1.0, kappa=2.0, mob=1.0)
    U0 = rounded(I.initial_state(dict(I.CH2048, n=(p_small, p_small)), seed=3), F32)
    ref = torch.as_tensor(O.explicit(o, U0, 0.01, 2), dtype=F32, device="cuda")
    N = p_small * p_small
    gb = S.Problem(n=(n, n), model=A.CAHN_HILLIARD, fe=A.F_01, dtype=F32, W=1.0, kappa=2.0,
                   mobility=1.0)
    c = torch.as_tensor(U0[:N].astype(np.float32), device="cuda").view(p_small, p_small)
    U = torch.zeros(2 * n * n, dtype=F32, device="cuda")
    U[: n * n].view(n, n).copy_(c.repeat(reps, reps))
    S.step_explicit(gb, U, 0.01, 2)
    for plane in range(2):
        got = U[plane * n * n:(plane + 1) * n * n].view(n, n)
        want = ref[plane * N:(plane + 1) * N].view(p_small, p_small).repeat(reps, reps)
        err = torch.linalg.vector_norm((got - want).double()) / torch.linalg.vector_norm(want.double())
        assert float(err) < (1e-5 if plane == 0 else 1e-4), (plane, float(err))
    del U
    torch.cuda.empty_cache()
