#!/usr/bin/env python3
"""Benchmark: explicit Cahn-Hilliard split step on a 2048x2048 periodic grid.

Workload (one GPU): f = W c^2 (1-c)^2 with W = 1, kappa = 2, M = 1, h = 1,
c0 = 0.5 + U(-0.01, 0.01) (seed 0), dt = 0.01, FP32 fields; 4 194 304 DOF
(the time-integrated c field).  A step is one fused launch of the HIP kernel
(residual + lumped-mass forward-Euler update, Eqs. 9-12).  Inputs are resident
in HBM before the timed region starts.

Prints ONE JSON line (rank 0):
  metric/value/unit: DOF-steps per second over the timed region,
  roofline: the step kernel against its bound.  A launch that fuses ks >= 2 steps
    does ks x 80 algorithmic flops per node per 8 bytes moved and is bound by the FP32 vector ALUs
    (non-packed: 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz = 78.6 TFLOP/s);
    a single-step launch (80 flops per 8 bytes) is bound by HBM (8 TB/s),
  hbm: the single-step launch timed on the same workload and on a 16384^2 grid
    (1 GiB per field, beyond the 256 MB Infinity Cache) against 8 TB/s,
  adjoint: wall time of the checkpointed batched adjoint gradient vs the six
    forward runs central differences need (64 ragged Allen-Cahn samples),
  surrogate: cost of one checked surrogate jump vs the K = 20 plain steps it replaces,
  cpu_baseline: the FP64 CPU reference timed on a bounded sample: one core (the
    oracle as the tests use it), all host cores (its OpenMP timing build), and
    bounded legs of the other workloads.

Before the W warm-up steps the step runs untimed for --settle-ms: a per-launch
kernel trace of a cold process shows the first ~500 launches (about 10 ms of work)
running about 10% slower than the steady state (the device's clocks ramping up
from idle); the timed K steps then measure the steady state however small W is.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12  # non-packed FP32 FMA issue: 78.6
BYTES_PER_NODE_STEP = 8  # read c, write c (FP32) per launch; mu never leaves the chip
# algorithmic flops per node-step of the Cahn-Hilliard split step (FMA = 2): values at the
# four Gauss points of an element, f' there, the scatter back to the nodes, the two 3x3
# stiffness stencils and the updates; the per-unit figure the roofline is priced with
# (the sum-factorised kernel itself executes 69)
FLOPS_PER_NODE_STEP_CH = 80
# the same split step with Gauss-Lobatto (nodal) quadrature: f' at the node (5), two
# 5-point stencils (5 each), mu (2) and the update (2)
FLOPS_PER_NODE_STEP_CH_LOBATTO = 19
# coupled model, per node-step with every Gauss point evaluated once (FMA = 2):
# interpolation of c and eta 30, the two sources at 4 points 144 (f_a 8, f_a' 6, f_b 4,
# f_b' 2, h 7, h' 4, combinations 5), scatters 36, mu/eta'/c' updates 19
FLOPS_PER_NODE_STEP_COUPLED = 229  # sum-factorised Q1 split step, FMA = 2 flops (see DESIGN)
# elasticity operator per node (FMA = 2): 3-D row sums 60, z-combinations 105, x-operator
# sums 27, x-assembly 72; 2-D: z-combinations 40, sums 8, x-assembly 48
FLOPS_PER_NODE_ELASTIC = {3: 264, 2: 96}
# grain growth per node and order parameter (FMA = 2): Gauss-point values 24, S 8,
# df/deta 20, projection onto the nodes 28, node sum + stiffness + update 21
FLOPS_PER_NODE_FIELD_GRAIN = 101
METRIC = "DOF-steps/sec + %HBM peak (explicit CH, 4.19M DOF); adjoint & surrogate speedup"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4200)
    # the step time settles after about 2000 steps on a freshly started process
    # (clock ramp); the warm-up is untimed
    ap.add_argument("--warmup", type=int, default=3000)
    ap.add_argument("--n", type=int, default=2048, help="grid side (default: the 2048^2 workload)")
    ap.add_argument("--settle-ms", type=float, default=300.0,
                    help="untimed run of the step before the warm-up steps (clock ramp), milliseconds")
    ap.add_argument("--fuse", type=int, default=0,
                    help="steps fused per launch (0: the library's choice; for profiling one kernel)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=40)
    ap.add_argument("--coupled", type=int, default=0, metavar="STEPS",
                    help="only time STEPS explicit steps of the 1024^2 coupled Allen-Cahn/"
                         "Cahn-Hilliard benchmark shape and print their record")
    ap.add_argument("--implicit", type=int, default=0, metavar="STEPS",
                    help="only time STEPS backward-Euler Newton steps of the 128^3 Cahn-Hilliard "
                         "workload (4.19M DOF) and print their record")
    ap.add_argument("--grain", type=int, default=0, metavar="STEPS",
                    help="only time STEPS explicit steps of the 20-order-parameter grain-growth "
                         "workload (2048^2) and print its record")
    ap.add_argument("--eshelby", action="store_true",
                    help="only time the Eshelby-inclusion solves (129^3 and 1025^2) and print their records")
    ap.add_argument("--adjoint", action="store_true",
                    help="only time the batched adjoint record (64 ragged Allen-Cahn samples)")
    ap.add_argument("--surrogate-gain", type=int, default=0, metavar="ITERS",
                    help="only train the surrogate for ITERS iterations on 512^2 Cahn-Hilliard "
                         "and print the matched-error gain record")
    ap.add_argument("--nn-backward", type=int, default=0, metavar="ITERS",
                    help="only time ITERS surrogate training iterations (forward + backward + "
                         "Adam) on 16 x 512^2 and print their record")
    ap.add_argument("--nn-forward", type=int, default=0, metavar="ITERS",
                    help="only time ITERS surrogate inference passes on 16 x 512^2 and print their record")
    ap.add_argument("--lobatto", action="store_true",
                    help="only the Gauss-Lobatto records (explicit 2048^2 CH at every fusion depth, "
                         "implicit 2048^2 AC)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the hbm / adjoint / surrogate records (the step alone)")
    ap.add_argument("--traffic", default=None,
                    help="counter record of the step kernel (default profiles/ch<n>_ks<ks>_traffic.json)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (counter calibration) and exit")
    ap.add_argument("--summarize-counters", nargs=3, metavar=("STEP_DIR", "COPY_DIR", "COPY_MIB"),
                    help="turn two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) of the step and of "
                         "the copy into the traffic record read by the roofline")
    return ap.parse_args()


KERNEL_SRC = os.path.join(ROOT, "paper_2601_06079_amd", "csrc", "k_stream2d.hip")


def kernel_hash():
    import hashlib
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def calibrate_copy(mib):
    import torch
    x = torch.ones(mib * 2 ** 18, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(20):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_mib": mib, "bytes_read": x.numel() * 4, "bytes_written": x.numel() * 4}))


def _counter_means(d):
    """Mean per dispatch of each (kernel, counter) in a rocprofv3 --pmc output tree."""
    import csv
    import glob
    acc = {}
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            key = (r["Kernel_Name"], r["Counter_Name"])
            acc.setdefault(key, []).append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in acc.items()}


def summarize_counters(step_dir, copy_dir, copy_mib, n=2048):
    """FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of the step kernel, scaled by the
    ratio true bytes / counter reading of a plain copy of known size."""
    step = {}
    for sub in ("fetch", "write"):
        step.update(_counter_means(os.path.join(step_dir, sub)))
    cp = {}
    for sub in ("fetch", "write"):
        cp.update(_counter_means(os.path.join(copy_dir, sub)))
    nbytes = copy_mib * 2 ** 20
    cf = [v for (k, c), v in cp.items() if c == "FETCH_SIZE" and v * 1024 > 0.5 * nbytes]
    cw = [v for (k, c), v in cp.items() if c == "WRITE_SIZE" and v * 1024 > 0.5 * nbytes]
    f_scale = nbytes / (max(cf) * 1024) if cf else 1.0
    w_scale = nbytes / (max(cw) * 1024) if cw else 1.0
    # the dominant step kernel: the one fusing the most steps (a run whose step count
    # is not a multiple of the fusion depth also holds single-step launches)
    names = sorted({k for (k, c) in step if _step_kernel(k)}, key=lambda k: -_step_kernel(k)[1])
    name = names[0] if names else None
    kf = [v for (k, c), v in step.items() if c == "FETCH_SIZE" and k == name]
    kw = [v for (k, c), v in step.items() if c == "WRITE_SIZE" and k == name]
    ks = _step_kernel(name)[1] if name else None
    rec = {"n": n, "ks": ks, "kernel": name, "kernel_src_sha256_16": kernel_hash(),
           "fetch_kib_raw": kf[0] if kf else None, "write_kib_raw": kw[0] if kw else None,
           "copy_fetch_scale": f_scale, "copy_write_scale": w_scale}
    if kf and kw:
        rec["bytes_per_launch"] = kf[0] * 1024 * f_scale + kw[0] * 1024 * w_scale
        rec["algorithmic_bytes_per_launch"] = BYTES_PER_NODE_STEP * n * n
    out = _traffic_path(n, ks)
    json.dump(rec, open(out, "w"), indent=1)
    print(json.dumps(rec))


def _step_kernel(name):
    """(kind, steps fused) of a 2-D explicit step kernel name, or None:
    k_explicit2d<T, MODEL, PF, KS, MIRROR, LOB> or k_explicit2d_seam<T, MODEL, KS, LOB>."""
    import re
    m = re.search(r"k_explicit2d(_seam)?<([^>]*)>", name)
    if not m:
        return None
    args = [a.strip() for a in m.group(2).split(",")]
    return ("seam", int(args[2])) if m.group(1) else ("halo", int(args[3]))


def _traffic_path(n, ks):
    return os.path.join(ROOT, "profiles", f"ch{n}_ks{ks}_traffic.json")


def _host():
    """Host CPU model and the cores this process may use."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cores": usable,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def cpu_baseline(n, steps):
    """The FP64 oracle on the workload's host cores, on bounded samples:
      - value: `steps` explicit split steps of the n^2 workload, single-threaded (the
        oracle the tests use);
      - all_cores: the same steps with the oracle's OpenMP timing build (element
        colours in parallel) on every thread OMP_NUM_THREADS allows;
      - legs: bounded runs of the other workloads, each extrapolated (labelled) to the
        full run: the 128^2 FP64 Allen-Cahn run (whole), one 64^3 backward-Euler
        Cahn-Hilliard step, 4 of the 64 calibration samples for 100 of 2000 steps, and
        the 20 plain steps one 512^2 surrogate jump replaces."""
    import numpy as np

    import oracle as O
    from paper_2601_06079_amd import inputs as I

    cfg = dict(I.CH2048, n=(n, n))
    o = O.Problem(n=(n, n), model=O.CH, fe=O.F_01, W=1.0, kappa=2.0, mob=1.0, h=1.0)
    U0 = I.initial_state(cfg, seed=0, dtype=np.float32).astype(np.float64)
    t0 = time.perf_counter()
    O.explicit(o, U0, cfg["dt"], steps)
    el = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, threads = O.explicit_threaded(o, U0, cfg["dt"], steps)
    el_mt = time.perf_counter() - t0
    legs = {}
    # 128^2 Allen-Cahn, FP64, 1000 steps: the whole run
    c1 = I.AC128
    o1 = O.Problem(n=c1["n"], model=O.AC, fe=O.F_SYM, W=1.0, kappa=1.0, mob=1.0)
    t0 = time.perf_counter()
    O.explicit(o1, I.initial_state(c1, seed=0), c1["dt"], c1["steps"])
    e1 = time.perf_counter() - t0
    legs["ac128_fp64"] = {"sample": f"the whole run: {c1['steps']} steps", "seconds": e1,
                          "dof_steps_per_s": 128 * 128 * c1["steps"] / e1}
    # one backward-Euler step of 3-D Cahn-Hilliard at 64^3 (the 128^3 workload is 8x the nodes)
    c3 = I.CH3D128
    o3 = O.Problem(n=(64, 64, 64), model=O.CH, fe=O.F_01, W=1.0, kappa=2.0, mob=1.0)
    cc = I.uniform_field((64, 64, 64), c3["lo"], c3["hi"], seed=0, base=c3["base"])
    U3 = O.explicit(o3, np.concatenate([cc, np.zeros_like(cc)]), 1.0, 0)
    t0 = time.perf_counter()
    _, conv, its, _ = O.newton_be(o3, c3["dt"], U3, rtol=1e-8, maxit=30, solver=1, lin_rtol=1e-6)
    e3 = time.perf_counter() - t0
    legs["implicit_ch3d"] = {"sample": "one 64^3 backward-Euler step (Newton + block-Jacobi GMRES, rtol 1e-8)",
                             "seconds": e3, "newton_its": its, "converged": bool(conv),
                             "extrapolated_s_per_128cubed_step": 8 * e3,
                             "extrapolated_s_200_steps_128cubed": 8 * e3 * 200}
    # calibration batch: 4 of the 64 samples, 100 of the 2000 steps, FP64
    sizes, theta, _, fields = I.batch_samples(count=64, seed=0)
    t0 = time.perf_counter()
    nodes4 = 0
    for i in range(4):
        nn_ = int(sizes[i])
        oi = O.Problem(n=(nn_, nn_), model=O.AC, fe=O.F_SYM, W=float(theta[i][2]), kappa=float(theta[i][1]),
                       mob=float(theta[i][0]))
        O.explicit(oi, np.asarray(fields[i], dtype=np.float64).ravel(), 0.05, 100)
        nodes4 += nn_ * nn_
    e4 = time.perf_counter() - t0
    nodes64 = int(sum(int(v) ** 2 for v in sizes))
    fwd = e4 * (nodes64 / nodes4) * (2000 / 100)
    legs["calibration_batch"] = {"sample": "4 of 64 samples, 100 of 2000 steps", "seconds": e4,
                                 "extrapolated_forward_s": fwd, "extrapolated_central_fd_s": 6 * fwd}
    # the 20 plain steps one surrogate jump replaces, 512^2 Cahn-Hilliard
    o5 = O.Problem(n=(512, 512), model=O.CH, fe=O.F_01, W=1.0, kappa=1.0, mob=1.0)
    U5 = I.initial_state(dict(I.CH2048, n=(512, 512)), seed=0, dtype=np.float32).astype(np.float64)
    t0 = time.perf_counter()
    O.explicit(o5, U5, 0.01, 20)
    e5 = time.perf_counter() - t0
    legs["surrogate_plain_20_steps_512"] = {"sample": "20 explicit steps, one 512^2 sample", "seconds": e5}
    return {"value": n * n * steps / el, "unit": "DOF-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} explicit split steps of the {n}x{n} workload, single-threaded "
                      f"FP64 element loop ({el:.1f} s)",
            "all_cores": {"value": n * n * steps / el_mt, "unit": "DOF-steps/s", "cores": threads,
                          "kind": "oracle (OpenMP timing build, 2^d element colours)",
                          "sample": f"the same {steps} steps ({el_mt:.1f} s)"},
            "host": _host(), "legs": legs}


def _settle(p, U, dt, ws, ms):
    """Run the step untimed until `ms` milliseconds of device work have passed."""
    import torch

    from paper_2601_06079_amd import solver as S
    t0 = time.perf_counter()
    while (time.perf_counter() - t0) * 1e3 < ms:
        S.step_explicit(p, U, dt, 100, ws)
        torch.cuda.synchronize()


def _events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def _time_ms(fn, stream):
    """Wall time of fn's GPU work on `stream` (events recorded on that stream)."""
    import torch
    a, b = _events()
    torch.cuda.synchronize()
    a.record(stream)
    fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b)


def ch_problem(n):
    import torch

    from paper_2601_06079_amd import _abi as A
    from paper_2601_06079_amd import solver as S
    return S.Problem(n=(n, n), model=A.CAHN_HILLIARD, fe=A.F_01, dtype=torch.float32, W=1.0,
                     kappa=2.0, mobility=1.0, h=1.0)


def single_step_hbm(n, steps, stream):
    """The single-step (unfused) launch of the CH split step on an n x n grid:
    8 algorithmic bytes per node per launch against 8 TB/s."""
    import numpy as np
    import torch

    from paper_2601_06079_amd import _abi as A
    from paper_2601_06079_amd import inputs as I
    from paper_2601_06079_amd import solver as S
    p = ch_problem(n)
    cfg = dict(I.CH2048, n=(n, n))
    U = torch.as_tensor(I.initial_state(cfg, seed=0, dtype="float32"), device="cuda")
    ws = S.workspace(p, A.OP_STEP_EXPLICIT)
    old = S.tune_get(A.TUNE_STREAM2D_FUSE)
    S.tune_set(A.TUNE_STREAM2D_FUSE, 1)
    try:
        S.step_explicit(p, U, cfg["dt"], 20, ws)
        epi = float(np.median([_time_ms(lambda: S.step_explicit(p, U, cfg["dt"], 0, ws), stream)
                               for _ in range(5)]))
        ms = _time_ms(lambda: S.step_explicit(p, U, cfg["dt"], steps, ws), stream)
    finally:
        S.tune_set(A.TUNE_STREAM2D_FUSE, old)
    kern_ms = max(ms - epi, 1e-6) / steps
    gbs = BYTES_PER_NODE_STEP * n * n / (kern_ms * 1e-3) / 1e9
    del U, ws
    torch.cuda.empty_cache()
    return {"n": n, "kernel_ms": kern_ms, "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": gbs / HBM_PEAK_GBS, "field_bytes": 4 * n * n}


def copy_ceiling(mib, stream, reps=20):
    """The library's 16-byte stream copy of `mib` MiB: read + write bytes over time."""
    import ctypes as ct

    import torch

    from paper_2601_06079_amd import _abi as A
    L = A.lib()
    L.pf_stream_copy.restype = ct.c_int
    L.pf_stream_copy.argtypes = [ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_size_t, ct.c_void_p]
    nb = mib * 2 ** 20
    x = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    args = (A.ctx(), ct.c_void_p(x.data_ptr()), ct.c_void_p(y.data_ptr()), nb, ct.c_void_p(stream.cuda_stream))
    for _ in range(3):
        A.check(L.pf_stream_copy(*args))
    ms = _time_ms(lambda: [L.pf_stream_copy(*args) for _ in range(reps)], stream) / reps
    assert torch.equal(x, y)
    del x, y
    torch.cuda.empty_cache()
    return {"mib": mib, "ms": ms, "gbs": 2 * nb / (ms * 1e-3) / 1e9, "kernel": "k_stream_copy (16-byte loads/stores)"}


def fma_ceiling(stream, blocks=8192, iters=4096, reps=5):
    """The library's FMA probe: independent non-packed FP32 FMA chains on every SIMD
    (blocks of 256 threads; 8192 blocks = 32 waves per SIMD), TFLOP/s."""
    import ctypes as ct

    import torch

    from paper_2601_06079_amd import _abi as A
    L = A.lib()
    L.pf_fma_probe.restype = ct.c_int
    L.pf_fma_probe.argtypes = [ct.c_void_p, ct.c_int, ct.c_int, ct.c_void_p, ct.c_void_p]
    out = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
    args = (A.ctx(), blocks, iters, ct.c_void_p(out.data_ptr()), ct.c_void_p(stream.cuda_stream))
    A.check(L.pf_fma_probe(*args))
    ms = min(_time_ms(lambda: L.pf_fma_probe(*args), stream) for _ in range(reps))
    flops = 16.0 * iters * blocks * 256
    return {"blocks": blocks, "waves_per_simd": blocks * 4 / 1024, "ms": ms,
            "tflops": flops / (ms * 1e-3) / 1e12, "peak": VALU_PEAK_TFLOPS,
            "kernel": "k_fma_probe (8 independent FMA chains per thread)"}


def nn_train_record(stream, iters=10, n=512, Bn=16):
    """Surrogate training iterations (forward, backward, Adam) on Bn random n^2
    fields: time per iteration, samples/s, and the BF16 rate of the network's flops
    (forward once, backward twice the forward: 3 x 39 168 flop per pixel)."""
    import numpy as np
    import torch

    from paper_2601_06079_amd import nn as NN
    r = np.random.default_rng(0)
    c = torch.as_tensor((0.5 + 0.1 * r.standard_normal((Bn, n, n))).astype(np.float32), device="cuda")
    M = torch.as_tensor(r.uniform(0.5, 2, Bn).astype(np.float32), device="cuda")
    k = torch.as_tensor(r.uniform(0.5, 2, Bn).astype(np.float32), device="cuda")
    tgt = c + 0.01
    model = NN.Surrogate(seed=0)
    model.train_step(c, M, k, tgt)
    ms = _time_ms(lambda: [model.train_step(c, M, k, tgt) for _ in range(iters)], stream) / iters
    flop = 3 * 39168.0 * Bn * n * n
    return {"workload": f"surrogate training iteration, {Bn} x {n}^2", "iters": iters, "ms_per_iter": ms,
            "samples_per_s": Bn / (ms * 1e-3), "tflops": flop / (ms * 1e-3) / 1e12,
            "frac_of_bf16_peak": flop / (ms * 1e-3) / 2.5e15}


def nn_forward_record(stream, iters=20, n=512, Bn=16):
    """Surrogate inference (pf_nn_forward: c, M, kappa -> c_hat) on Bn random n^2 fields:
    time per pass and the BF16 rate of the network's 39 168 flop per pixel."""
    import numpy as np
    import torch

    from paper_2601_06079_amd import nn as NN
    r = np.random.default_rng(0)
    c = torch.as_tensor((0.5 + 0.1 * r.standard_normal((Bn, n, n))).astype(np.float32), device="cuda")
    M = torch.as_tensor(r.uniform(0.5, 2, Bn).astype(np.float32), device="cuda")
    k = torch.as_tensor(r.uniform(0.5, 2, Bn).astype(np.float32), device="cuda")
    model = NN.Surrogate(seed=0)
    model.forward(c, M, k)
    ms = min(_time_ms(lambda: [model.forward(c, M, k) for _ in range(iters)], stream) / iters for _ in range(3))
    flop = 39168.0 * Bn * n * n
    return {"workload": f"surrogate inference, {Bn} x {n}^2", "iters": iters, "ms_per_forward": ms,
            "tflops": flop / (ms * 1e-3) / 1e12, "frac_of_bf16_peak": flop / (ms * 1e-3) / 2.5e15}


def ac128_record(stream, steps=1000):
    """The 128^2 periodic Allen-Cahn workload in FP64 (f = (c^2-1)^2/4, kappa = L = 1,
    dt = 0.1): one call of `steps` explicit steps."""
    import torch

    from paper_2601_06079_amd import _abi as A
    from paper_2601_06079_amd import inputs as I
    from paper_2601_06079_amd import solver as S
    cfg = I.AC128
    p = S.Problem(n=cfg["n"], model=A.ALLEN_CAHN, fe=A.F_SYM, dtype=torch.float64, W=1.0, kappa=1.0,
                  mobility=1.0, h=1.0)
    U = torch.as_tensor(I.initial_state(cfg, seed=0), device="cuda")
    ws = S.workspace(p, A.OP_STEP_EXPLICIT)
    S.step_explicit(p, U.clone(), cfg["dt"], 100, ws)
    ms = _time_ms(lambda: S.step_explicit(p, U, cfg["dt"], steps, ws), stream)
    n = p.nnodes
    return {"workload": "2D Allen-Cahn 128x128 periodic, FP64, explicit dt=0.1", "steps": steps,
            "ms_per_step": ms / steps, "dof_steps_per_s": n * steps / (ms * 1e-3)}


def coupled_record(stream, n=1024, steps=2000):
    """Coupled Allen-Cahn / Cahn-Hilliard benchmark shape (Eq. 7, Supp. Note 3):
    [0, 100]^2 with n^2 nodes, no-flux, M_c = 1, M_eta = 150, kappa_eta = 0.3, FP32,
    explicit steps at dt = 5e-7 (the explicit limit of the c-equation at h = 100/1023).
    DOF = 2 n^2 (c and eta are time-integrated; mu is the algebraic row)."""
    import torch

    from paper_2601_06079_amd import _abi as A
    from paper_2601_06079_amd import inputs as I
    from paper_2601_06079_amd import solver as S
    cfg = I.COUPLED
    p = S.Problem(n=(n, n), model=A.COUPLED, dtype=torch.float32, h=cfg["L"] / (n - 1),
                  kappa=cfg["kappa"], mobility=cfg["Mc"], mobility_eta=cfg["Meta"], bc=A.NOFLUX)
    U = torch.as_tensor(I.coupled_state(n, seed=0, dtype="float32"), device="cuda")
    ws = S.workspace(p, A.OP_STEP_EXPLICIT)
    S.step_explicit(p, U, 5e-7, 200, ws)  # warm-up
    ms = _time_ms(lambda: S.step_explicit(p, U, 5e-7, steps, ws), stream)
    dof = 2 * n * n
    tflops = FLOPS_PER_NODE_STEP_COUPLED * n * n * steps / (ms * 1e-3) / 1e12
    return {"workload": f"coupled Allen-Cahn/Cahn-Hilliard {n}x{n} on [0,100]^2, no-flux, "
                        "M_c=1, M_eta=150, kappa_eta=0.3, FP32 explicit dt=5e-7",
            "dof": dof, "steps": steps, "ms_per_step": ms / steps,
            "dof_steps_per_s": dof * steps / (ms * 1e-3),
            "roofline": {"bound": "alu", "kernel": "k_cp_explicit2d<float, no-flux>",
                         "flops_per_node_step": FLOPS_PER_NODE_STEP_COUPLED, "achieved": tflops,
                         "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": tflops / VALU_PEAK_TFLOPS,
                         "hbm_gbs": 16 * n * n * steps / (ms * 1e-3) / 1e9}}


def lobatto_record(stream, n=2048, steps=2000):
    """The explicit benchmark workload (Cahn-Hilliard 2048^2 periodic, dt = 0.01, W = 1,
    kappa = 2, M = 1, h = 1) with Gauss-Lobatto (nodal) quadrature, at every fusion
    depth (tuning key STREAM2D_FUSE) and at the library's default."""
    import torch

    from paper_2601_06079_amd import _abi as A
    from paper_2601_06079_amd import inputs as I
    from paper_2601_06079_amd import solver as S
    p = ch_problem(n)
    p.quad = A.QUAD_LOBATTO
    c0 = torch.as_tensor(I.uniform_field((n, n), -0.05, 0.05, seed=0, base=0.5), dtype=torch.float32)
    U0 = torch.cat([c0, torch.zeros_like(c0)]).to("cuda")
    ws = S.workspace(p, A.OP_STEP_EXPLICIT)
    old = S.tune_get(A.TUNE_STREAM2D_FUSE)
    by_ks = {}
    try:
        for ks in (0, 1, 2, 3, 4):
            S.tune_set(A.TUNE_STREAM2D_FUSE, ks)
            U = U0.clone()
            S.step_explicit(p, U, 0.01, 240, ws)  # warm-up
            ms = min(_time_ms(lambda: S.step_explicit(p, U, 0.01, steps, ws), stream) for _ in range(3))
            by_ks["default" if ks == 0 else f"ks{ks}"] = ms / steps
    finally:
        S.tune_set(A.TUNE_STREAM2D_FUSE, old)
    best = min(by_ks, key=by_ks.get)
    ms = by_ks["default"]
    N = n * n
    return {"workload": f"2D Cahn-Hilliard {n}x{n} periodic, explicit split step, Gauss-Lobatto "
                        "(nodal) quadrature, dt=0.01, W=1, kappa=2, M=1, FP32", "dof": N,
            "steps": steps, "ms_per_step": ms, "dof_steps_per_s": N / (ms * 1e-3),
            "ms_per_step_by_fusion": by_ks, "best": best,
            "tflops": FLOPS_PER_NODE_STEP_CH_LOBATTO * N / (ms * 1e-3) / 1e12,
            "flops_per_node_step": FLOPS_PER_NODE_STEP_CH_LOBATTO}


def implicit2d_record(stream, model, n, steps=10, dt=0.05, mass=0, krylov=0, quad=0):
    """The paper's 2-D implicit benchmark shapes (backward Euler, Newton + GMRES(30)
    with block Jacobi, FP32 fields): [0, 100]^2 with n^2 nodes, no-flux,
    f' = 4c(c-1)(c-1/2) (W = 1), M = 1, kappa = 2 (Allen-Cahn) or 1.5 (Cahn-Hilliard);
    initial field 0.5 + U(-0.05, 0.05).  dt = 0.05: block-Jacobi GMRES iterations grow
    with dt kappa / h^2 (34 per Newton iteration at 2048^2, 57 at dt = 0.2)."""
    import numpy as np
    import torch

    from paper_2601_06079_amd import _abi as A
    from paper_2601_06079_amd import inputs as I
    from paper_2601_06079_amd import solver as S
    ch = model == A.CAHN_HILLIARD
    p = S.Problem(n=(n, n), model=model, fe=A.F_01, dtype=torch.float32, W=1.0,
                  kappa=1.5 if ch else 2.0, mobility=1.0, h=100.0 / (n - 1), bc=A.NOFLUX, mass=mass,
                  quad=quad)
    c0 = I.uniform_field((n, n), -0.05, 0.05, seed=0, base=0.5).astype(np.float32)
    U = torch.as_tensor(np.concatenate([c0, np.zeros_like(c0)]) if ch else c0, device="cuda")
    if ch:
        S.step_explicit(S.Problem(**{**p.__dict__, "mass": 0}), U, 1e-30, 0)  # mu0 (lumped row)
    ws = S.workspace(p, A.OP_NEWTON)
    opts = S.newton_opts(krylov=krylov)
    Uold = torch.empty_like(U)
    Uold.copy_(U)
    S.newton_step(p, dt, Uold, U, opts, ws=ws)  # warm-up (not timed)
    torch.cuda.synchronize()
    newton, gmres, ok = [], [], 0
    t0 = time.perf_counter()
    for _ in range(steps):
        Uold.copy_(U)
        rep = S.newton_step(p, dt, Uold, U, opts, ws=ws)
        newton.append(rep.newton_its)
        gmres.append(rep.gmres_its)
        ok += int(rep.converged)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    name = "Cahn-Hilliard" if ch else "Allen-Cahn"
    dof = n * n
    mname = "consistent mass (all terms Gauss-integrated)" if mass else "lumped mass"
    if quad == A.QUAD_LOBATTO:
        mname = "Gauss-Lobatto (nodal) quadrature"
    lin = "CG with point Jacobi" if krylov == A.KRYLOV_CG else "GMRES(30) with block-Jacobi"
    return {"workload": f"2D {name} {n}x{n} on [0,100]^2, no-flux, backward Euler dt={dt}, {mname}, "
                        f"Newton + {lin}, FP32 fields",
            "dof": dof, "steps": steps, "converged_steps": ok, "ms_per_step": 1e3 * el / steps,
            "dof_steps_per_s": dof * steps / el, "newton_its_per_step": float(np.mean(newton)),
            "gmres_its_per_newton": float(np.sum(gmres) / max(np.sum(newton), 1))}


def coupled_implicit_record(stream, n=512, steps=20, dt=0.01):
    """The coupled benchmark shape with backward-Euler steps: 512^2, no-flux, dt = 0.01,
    Newton + GMRES(30) with 3x3 block Jacobi, FP32 fields, FP64 reductions."""
    import numpy as np
    import torch

    from paper_2601_06079_amd import _abi as A
    from paper_2601_06079_amd import inputs as I
    from paper_2601_06079_amd import solver as S
    cfg = I.COUPLED
    p = S.Problem(n=(n, n), model=A.COUPLED, dtype=torch.float32, h=cfg["L"] / (n - 1),
                  kappa=cfg["kappa"], mobility=cfg["Mc"], mobility_eta=cfg["Meta"], bc=A.NOFLUX)
    U = torch.as_tensor(I.coupled_state(n, seed=0, dtype="float32"), device="cuda")
    S.step_explicit(p, U, 1e-9, 0)  # mu consistent with (c, eta)
    ws = S.workspace(p, A.OP_NEWTON)
    Uold = torch.empty_like(U)
    Uold.copy_(U)
    S.newton_step(p, dt, Uold, U, ws=ws)  # warm-up step (not timed)
    torch.cuda.synchronize()
    newton, gmres, ok = [], [], 0
    t0 = time.perf_counter()
    for _ in range(steps):
        Uold.copy_(U)
        rep = S.newton_step(p, dt, Uold, U, ws=ws)
        newton.append(rep.newton_its)
        gmres.append(rep.gmres_its)
        ok += int(rep.converged)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    dof = 2 * n * n
    return {"workload": f"coupled Allen-Cahn/Cahn-Hilliard {n}x{n} on [0,100]^2, no-flux, backward "
                        f"Euler dt={dt}, Newton + GMRES(30) with 3x3 block-Jacobi, FP32 fields",
            "dof": dof, "unknowns": 3 * n * n, "steps": steps, "converged_steps": ok,
            "ms_per_step": 1e3 * el / steps, "dof_steps_per_s": dof * steps / el,
            "newton_its_per_step": float(np.mean(newton)),
            "gmres_its_per_newton": float(np.sum(gmres) / max(np.sum(newton), 1))}


def eshelby_record(stream, n=(129, 129, 129), rtol=1e-6, reps=50):
    """The Eshelby-inclusion benchmark (Eqs. 3-4, Eq. III.1): [0, 100]^dim with the
    given nodes per axis, E = 22.5, nu = 0.3, dilatational misfit m = 0.01 inside
    radius a = 20 (interface l = 0.5), symmetry planes through the origin and
    traction-free outer faces; FP32 fields, multigrid-preconditioned CG (FP64
    scalars) to rtol.  One solve, its volume change and the adjoint (E, nu)
    sensitivities, the same solve by plain CG for comparison, plus the operator
    kernel alone (reps launches replayed from a HIP graph, timed with events on the
    stream)."""
    import torch

    from paper_2601_06079_amd import elastic as EL
    dim = len(n)
    p = EL.ElasticProblem(n=tuple(n), h=100.0 / (n[0] - 1), dtype=torch.float32)
    ws = EL.workspace(p)
    u = torch.empty(p.ndof, dtype=torch.float32, device="cuda")
    EL.el_solve(p, out=u, rtol=rtol, ws=ws)  # warm-up (not timed)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u, rep = EL.el_solve(p, out=u, rtol=rtol, ws=ws)
    torch.cuda.synchronize()
    solve_s = time.perf_counter() - t0
    vol = float(EL.el_objective(p, u, ws=ws).item())
    t0 = time.perf_counter()
    (O, dE, dnu), arep = EL.el_sensitivity(p, u, rtol=rtol, ws=ws)
    sens_s = time.perf_counter() - t0
    # plain CG on the same problem (one level), for comparison
    from paper_2601_06079_amd import _abi as A
    L = A.lib()
    L.pf_tune_set(EL.TUNE_EL_MG, 1)
    try:
        uc = torch.empty_like(u)
        wsc = EL.workspace(p)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        uc, crep = EL.el_solve(p, out=uc, rtol=rtol, ws=wsc)
        torch.cuda.synchronize()
        cg_s = time.perf_counter() - t0
    finally:
        L.pf_tune_set(EL.TUNE_EL_MG, 0)
    del uc, wsc
    # the operator alone: `reps` launches captured in one HIP graph and replayed
    # (no host launch overhead between them), timed with events on the stream
    v = torch.randn(p.ndof, dtype=torch.float32, device="cuda")
    y = torch.empty_like(v)
    for _ in range(5):
        EL.el_apply(p, v, out=y)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for _ in range(reps):
            EL.el_apply(p, v, out=y)
    graph.replay()
    torch.cuda.synchronize()
    ms = _time_ms(graph.replay, stream)
    apply_ms = ms / reps
    del graph
    N = p.nnodes
    tflops = FLOPS_PER_NODE_ELASTIC[dim] * N / (apply_ms * 1e-3) / 1e12
    apply_gbs = 2 * 4 * p.ndof / (apply_ms * 1e-3) / 1e9
    it_ms = 1e3 * solve_s / max(rep.iterations, 1)
    del ws, u, v, y
    torch.cuda.empty_cache()
    shape = "x".join(str(k) for k in n)
    return {"workload": f"Eshelby inclusion {shape} nodes on [0,100]^{dim}"
                        f"{' (plane strain)' if dim == 2 else ''}, E=22.5, nu=0.3, m=0.01, a=20, l=0.5, "
                        f"symmetry + traction-free, FP32 fields, multigrid-preconditioned CG to rtol {rtol:g}",
            "dof": p.ndof, "solve_ms": 1e3 * solve_s, "cg_iterations": rep.iterations,
            "mg_levels": rep.levels, "converged": bool(rep.converged), "ms_per_iteration": it_ms,
            "plain_cg": {"solve_ms": 1e3 * cg_s, "iterations": crep.iterations,
                         "converged": bool(crep.converged)},
            "volume_change": vol, "sensitivity": {"dV_dE": dE, "dV_dnu": dnu, "ms": 1e3 * sens_s,
                                                  "adjoint_iterations": arep.iterations},
            "operator": {"kernel": f"k_el_apply<float, {dim}>", "us_per_launch": 1e3 * apply_ms,
                         "bound": "alu", "flops_per_node": FLOPS_PER_NODE_ELASTIC[dim],
                         "achieved": tflops, "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": tflops / VALU_PEAK_TFLOPS, "hbm_gbs": apply_gbs}}


def grain_record(stream, n=2048, steps=200):
    """Grain growth (p = 20 Allen-Cahn order parameters coupled by the multi-well
    energy, gamma = 1.5, kappa = L = 1, h = 1, dt = 0.1; 60 Voronoi grains), FP32,
    periodic: `steps` explicit steps in one call, all order parameters per launch."""
    import torch

    from paper_2601_06079_amd import _abi as A
    from paper_2601_06079_amd import inputs as I
    from paper_2601_06079_amd import solver as S
    cfg = I.GRAIN
    P = cfg["p"]
    p = S.Problem(n=(n, n), model=A.GRAIN, dtype=torch.float32, h=1.0, kappa=cfg["kappa"],
                  mobility=cfg["L"], nfields=P, gamma=cfg["gamma"])
    U = torch.as_tensor(I.grain_state(n, P, cfg["grains"], seed=0, dtype="float32"), device="cuda")
    ws = S.workspace(p, A.OP_STEP_EXPLICIT)
    S.step_explicit(p, U, cfg["dt"], 20, ws)  # warm-up
    ms = _time_ms(lambda: S.step_explicit(p, U, cfg["dt"], steps, ws), stream)
    kern_ms = ms / steps
    N = n * n
    dof = P * N
    tflops = FLOPS_PER_NODE_FIELD_GRAIN * dof / (kern_ms * 1e-3) / 1e12
    gbs = 8 * dof / (kern_ms * 1e-3) / 1e9
    e = S.energy(p, U)
    torch.cuda.synchronize()
    del U, ws
    torch.cuda.empty_cache()
    return {"workload": f"grain growth {n}x{n} periodic, {P} order parameters, 60 Voronoi grains, "
                        f"gamma={cfg['gamma']}, kappa=L=1, FP32 explicit dt={cfg['dt']}",
            "dof": dof, "steps": steps, "ms_per_step": kern_ms, "dof_steps_per_s": dof / (kern_ms * 1e-3),
            "energy_after": float(e[0]),
            "roofline": {"kernel": f"k_gg_stream2d<float, {P}>", "bound": "alu",
                         "flops_per_node_field": FLOPS_PER_NODE_FIELD_GRAIN, "achieved": tflops,
                         "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": tflops / VALU_PEAK_TFLOPS,
                         "hbm_gbs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS}}


def grain_implicit_record(stream, n=1024, steps=10, dt=2.0):
    """Grain growth with backward-Euler steps (the paper's grain-growth runs are
    implicit): 20 order parameters on n^2 (grid units), the explicit record's
    physics and initial state, Newton + GMRES(30) with point Jacobi over all
    unknowns, FP32 fields, FP64 reductions; dt is 20x the explicit step."""
    import numpy as np
    import torch

    from paper_2601_06079_amd import _abi as A
    from paper_2601_06079_amd import inputs as I
    from paper_2601_06079_amd import solver as S
    cfg = I.GRAIN
    P = cfg["p"]
    p = S.Problem(n=(n, n), model=A.GRAIN, dtype=torch.float32, h=1.0, kappa=cfg["kappa"],
                  mobility=cfg["L"], nfields=P, gamma=cfg["gamma"])
    U = torch.as_tensor(I.grain_state(n, P, cfg["grains"], seed=0, dtype="float32"), device="cuda")
    ws = S.workspace(p, A.OP_NEWTON)
    Uold = torch.empty_like(U)
    Uold.copy_(U)
    S.newton_step(p, dt, Uold, U, ws=ws)  # warm-up step (not timed)
    torch.cuda.synchronize()
    newton, gmres, ok = [], [], 0
    t0 = time.perf_counter()
    for _ in range(steps):
        Uold.copy_(U)
        r = S.newton_step(p, dt, Uold, U, ws=ws)
        newton.append(r.newton_its)
        gmres.append(r.gmres_its)
        ok += int(r.converged)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    dof = P * n * n
    del U, Uold, ws
    torch.cuda.empty_cache()
    return {"workload": f"grain growth {n}x{n} periodic, {P} order parameters, backward Euler dt={dt}, "
                        "Newton + GMRES(30) with point Jacobi, FP32 fields",
            "dof": dof, "steps": steps, "converged_steps": ok, "ms_per_step": 1e3 * el / steps,
            "dof_steps_per_s": dof * steps / el, "newton_its_per_step": float(np.mean(newton)),
            "gmres_its_per_newton": float(np.sum(gmres) / max(np.sum(newton), 1))}


def adjoint_record(stream, count=64, nsteps=2000, every=100):
    """Batched calibration workload (64 ragged Allen-Cahn samples, 128^2..512^2,
    2000 FP32 steps, dt = 0.05): forward plus the hand-written adjoint, against the
    six plain forward runs that central differences in (L, kappa, W) need.  Two
    variants: a snapshot every 100 steps with recomputation of each segment, and the
    whole trajectory kept in HBM (61 GB here) with no recomputation."""
    import numpy as np
    import torch

    from paper_2601_06079_amd import _abi as A
    from paper_2601_06079_amd import batch as B
    from paper_2601_06079_amd import inputs as I
    sizes, theta, hidden, fields = I.batch_samples(count=count, seed=0)
    sizes = [(int(n), int(n)) for n in sizes]
    mk = lambda th: B.Batch(sizes, th, 0.05, model=A.ALLEN_CAHN, fe=A.F_SYM, dtype=torch.float32)
    b = mk(theta)
    U0 = b.pack(fields)
    tgt = U0.clone()
    mk(hidden).step(tgt, nsteps)
    ws = b.workspace(A.OP_STEP_EXPLICIT)
    U = U0.clone()
    b.step(U, 100, ws)  # warm-up
    t_plain = _time_ms(lambda: b.step(U, nsteps, ws), stream)
    th = torch.tensor(theta, dtype=torch.float64, device="cuda", requires_grad=True)
    # warm-up of the whole autograd path (its snapshot and segment buffers then come
    # from the allocator's cache, as in any repeated calibration iteration)
    B.per_sample_mse(b, B.explicit_run(th, U0, b, nsteps, every=every), tgt).backward()
    th.grad = None
    state = {}

    def fwd():
        state["UN"] = B.explicit_run(th, U0, b, nsteps, every=every)
        state["loss"] = B.per_sample_mse(b, state["UN"], tgt)

    t_fwd = _time_ms(fwd, stream)
    t_bwd = _time_ms(lambda: state["loss"].backward(), stream)
    nodes = sum(a * c for a, c in sizes)
    whole = None
    state.clear()
    torch.cuda.empty_cache()
    if B.trajectory_fits(b, nsteps):
        th.grad = None
        B.per_sample_mse(b, B.explicit_run(th, U0, b, nsteps, every=None), tgt).backward()
        th.grad = None

        def fwd_all():
            state["UN"] = B.explicit_run(th, U0, b, nsteps, every=None)
            state["loss"] = B.per_sample_mse(b, state["UN"], tgt)

        tf = _time_ms(fwd_all, stream)
        tb = _time_ms(lambda: state["loss"].backward(), stream)
        state.clear()
        torch.cuda.empty_cache()
        whole = {"forward_ms": tf, "adjoint_ms": tb, "speedup_vs_central_fd": 6 * t_plain / (tf + tb),
                 "trajectory_gb": (nsteps + 1) * b.total * 4 / 1e9}

    # the same 64 samples as 64 separate single-problem runs (one after another)
    from paper_2601_06079_amd import solver as S
    probs = [S.Problem(n=sz, model=A.ALLEN_CAHN, fe=A.F_SYM, dtype=torch.float32, W=float(th[2]),
                       kappa=float(th[1]), mobility=float(th[0])) for sz, th in zip(sizes, theta)]
    fields = [v.clone() for v in b.views(U0)]
    wss = [S.workspace(q, A.OP_STEP_EXPLICIT) for q in probs]
    for q, f, w in zip(probs, fields, wss):
        S.step_explicit(q, f, 0.05, 20, w)

    def separate():
        for q, f, w in zip(probs, fields, wss):
            S.step_explicit(q, f, 0.05, nsteps, w)

    t_sep = _time_ms(separate, stream)
    return {"workload": f"{count} ragged Allen-Cahn samples 128^2..512^2 ({nodes} nodes), "
                        f"{nsteps} FP32 steps, checkpoint every {every}",
            "forward_ms": t_fwd, "adjoint_ms": t_bwd, "plain_forward_ms": t_plain,
            "central_fd_ms": 6 * t_plain,
            "speedup_vs_central_fd": 6 * t_plain / (t_fwd + t_bwd),
            "batched_dof_steps_per_s": nodes * nsteps / (t_plain * 1e-3),
            "separate_runs_ms": t_sep, "batching_speedup": t_sep / t_plain,
            "whole_trajectory": whole}


def surrogate_record(stream, n=512, Bn=16, K=20, dt=0.01):
    """One checked surrogate jump (network forward, one explicit step of c_hat, the
    residual/mass reductions) vs the K plain FP32 steps it replaces, on a batch of
    Bn 512^2 Cahn-Hilliard samples.  Cost only: the matched-error gain needs a
    trained network and is measured by the surrogate gain test."""
    import numpy as np

    from paper_2601_06079_amd import nn as NN
    rng = np.random.default_rng(0)
    ens = NN.CHEnsemble(Bn, n, rng.uniform(0.5, 2, Bn), rng.uniform(0.5, 2, Bn), dt=dt, seed=1)
    ens.advance(200)
    model = NN.Surrogate(seed=0)
    c = ens.field().clone()
    U = ens.U.clone()
    reps = 10

    def jump():
        chat = model.forward(c, ens.Mt, ens.kt)
        step = chat.reshape(-1).clone()
        ens.batch.step(step, 1, ens.ws)
        model.check(chat, c, step.view_as(chat), K * dt, dt)

    jump()
    ens.batch.step(U, K, ens.ws)
    # each: the best of three windows of `reps` calls
    best = lambda fn: min(_time_ms(lambda: [fn() for _ in range(reps)], stream) for _ in range(3)) / reps
    t_fwd = best(lambda: model.forward(c, ens.Mt, ens.kt))
    t_jump = best(jump)
    t_plain = best(lambda: ens.batch.step(U, K, ens.ws))
    flop = 39168.0 * Bn * n * n
    return {"workload": f"{Bn} x {n}^2 Cahn-Hilliard, K = {K} steps of dt = {dt}",
            "network_forward_ms": t_fwd, "checked_jump_ms": t_jump, "plain_K_steps_ms": t_plain,
            "speedup_per_jump": t_plain / t_jump,
            "network_forward_tflops": flop / (t_fwd * 1e-3) / 1e12}


def implicit_record(steps, stream):
    """Backward-Euler Newton steps of 128^3 periodic Cahn-Hilliard (c, mu both
    unknowns: 4 194 304 DOF), dt = 0.5, matrix-free JVP + GMRES(30) with 2x2
    block-Jacobi, FP32 fields and FP64 reductions (Eqs. 13-14)."""
    import numpy as np
    import torch

    from paper_2601_06079_amd import _abi as A
    from paper_2601_06079_amd import inputs as I
    from paper_2601_06079_amd import solver as S
    cfg = I.CH3D128
    n = cfg["n"]
    p = S.Problem(n=n, model=A.CAHN_HILLIARD, fe=A.F_01, dtype=torch.float32, W=1.0, kappa=2.0,
                  mobility=1.0, h=1.0)
    c0 = I.uniform_field(n, cfg["lo"], cfg["hi"], seed=0, base=cfg["base"]).astype(np.float32)
    U = torch.as_tensor(np.concatenate([c0, np.zeros_like(c0)]), device="cuda")
    S.step_explicit(p, U, 1e-30, 0)  # mu0 = [N(c0) + kappa K c0]/m
    ws = S.workspace(p, A.OP_NEWTON)
    Uold = torch.empty_like(U)
    newton, gmres, ok = [], [], 0
    Uold.copy_(U)
    S.newton_step(p, cfg["dt"], Uold, U, ws=ws)  # warm-up step (not timed)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        Uold.copy_(U)
        rep = S.newton_step(p, cfg["dt"], Uold, U, ws=ws)
        newton.append(rep.newton_its)
        gmres.append(rep.gmres_its)
        ok += int(rep.converged)
        if (k + 1) % 20 == 0:
            print(f"[implicit] step {k + 1}/{steps}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    dof = 2 * int(np.prod(n))
    return {"workload": "3D Cahn-Hilliard 128^3 periodic, backward Euler dt=0.5, Newton + GMRES(30) "
                        "with 2x2 block-Jacobi, FP32 fields, FP64 reductions",
            "dof": dof, "steps": steps, "converged_steps": ok, "ms_per_step": 1e3 * el / steps,
            "dof_steps_per_s": dof * steps / el,
            "newton_its_per_step": float(np.mean(newton)),
            "gmres_its_per_newton": float(np.sum(gmres) / max(np.sum(newton), 1)),
            "mass_drift": float(abs(U[: dof // 2].double().mean() - float(c0.astype(np.float64).mean())))}


def main():
    args = parse()
    if (args.implicit or args.surrogate_gain or args.adjoint or args.coupled or args.eshelby or args.grain
            or args.nn_backward or args.nn_forward or args.lobatto):
        import torch
        stream = torch.cuda.current_stream()
        if args.grain:
            print(json.dumps(grain_record(stream, steps=args.grain)), flush=True)
            print(json.dumps(grain_record(stream, n=1024, steps=args.grain)), flush=True)
            print(json.dumps(grain_implicit_record(stream)), flush=True)
        if args.eshelby:
            print(json.dumps(eshelby_record(stream)), flush=True)
            print(json.dumps(eshelby_record(stream, n=(1025, 1025))), flush=True)
        if args.adjoint:
            print(json.dumps(adjoint_record(stream)), flush=True)
        if args.lobatto:
            from paper_2601_06079_amd import _abi as A
            print(json.dumps(lobatto_record(stream)), flush=True)
            print(json.dumps(implicit2d_record(stream, A.ALLEN_CAHN, 2048, steps=5,
                                               quad=A.QUAD_LOBATTO)), flush=True)
        if args.implicit:
            print(json.dumps(implicit_record(args.implicit, stream)), flush=True)
            from paper_2601_06079_amd import _abi as A
            print(json.dumps(implicit2d_record(stream, A.ALLEN_CAHN, 2048)), flush=True)
            print(json.dumps(implicit2d_record(stream, A.ALLEN_CAHN, 2048, krylov=A.KRYLOV_CG)), flush=True)
            print(json.dumps(implicit2d_record(stream, A.CAHN_HILLIARD, 512)), flush=True)
            print(json.dumps(implicit2d_record(stream, A.ALLEN_CAHN, 2048, steps=5,
                                               mass=A.MASS_CONSISTENT)), flush=True)
            print(json.dumps(implicit2d_record(stream, A.CAHN_HILLIARD, 512, steps=5,
                                               mass=A.MASS_CONSISTENT)), flush=True)
        if args.coupled:
            print(json.dumps(coupled_record(stream, steps=args.coupled)), flush=True)
            print(json.dumps(coupled_implicit_record(stream)), flush=True)
        if args.nn_backward:
            print(json.dumps(nn_train_record(stream, iters=args.nn_backward)), flush=True)
        if args.nn_forward:
            print(json.dumps(nn_forward_record(stream, iters=args.nn_forward)), flush=True)
        if args.surrogate_gain:
            from paper_2601_06079_amd import nn as NN
            rec = NN.gain_experiment(train_iters=args.surrogate_gain,
                                     log=lambda m: print(m, file=sys.stderr, flush=True))
            print(json.dumps(rec), flush=True)
        return
    if args.summarize_counters:
        summarize_counters(args.summarize_counters[0], args.summarize_counters[1],
                           int(args.summarize_counters[2]), n=args.n)
        return
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: the library has no "
                                   "multi-GPU path (--gpus must be 1)"}))
        sys.exit(2)
    import torch

    import ctypes as ct

    from paper_2601_06079_amd import _abi as A
    from paper_2601_06079_amd import inputs as I
    from paper_2601_06079_amd import solver as S

    n = args.n
    cfg = dict(I.CH2048, n=(n, n))
    N = n * n
    p = ch_problem(n)
    U = torch.as_tensor(I.initial_state(cfg, seed=0, dtype="float32"), device="cuda")
    ws = S.workspace(p, A.OP_STEP_EXPLICIT)
    dt = cfg["dt"]
    stream = torch.cuda.current_stream()

    if args.fuse:
        S.tune_set(A.TUNE_STREAM2D_FUSE, args.fuse)
    _settle(p, U, dt, ws, args.settle_ms)
    S.step_explicit(p, U, dt, args.warmup, ws)
    torch.cuda.synchronize()

    # timed region: K steps in one call (the library enqueues the fused launches);
    # the call's arguments are marshalled beforehand
    L = A.lib()
    call = (A.ctx(), ct.byref(p.c()), dt)
    uptr, wptr = ct.c_void_p(U.data_ptr()), ct.c_void_p(ws.data_ptr())
    sptr = ct.c_void_p(stream.cuda_stream)
    e0, e1 = _events()
    torch.cuda.synchronize()
    e0.record(stream)
    rc = L.pf_step_explicit(*call, args.steps, uptr, wptr, sptr)
    e1.record(stream)
    torch.cuda.synchronize()
    A.check(rc)
    ms_total = e0.elapsed_time(e1)
    ms_per_step = ms_total / args.steps
    value = N * args.steps / (ms_total * 1e-3)

    # Average duration of one launch of the dominant kernel over the timed region:
    # the K steps ran as back-to-back launches of the fused kernel (ks steps each)
    # plus one chemical-potential epilogue, measured separately and subtracted.
    ks_, ty_, dp_ = ct.c_int(0), ct.c_int(0), ct.c_int(0)
    A.check(A.lib().pf_launch_shape(A.ctx(), ct.byref(p.c()), ct.byref(ks_), ct.byref(ty_), ct.byref(dp_)))
    ks = ks_.value
    import numpy as np
    epi = float(np.median([_time_ms(lambda: L.pf_step_explicit(*call, 0, uptr, wptr, sptr), stream)
                           for _ in range(11)]))
    launches = args.steps // ks + args.steps % ks
    kern_ms = max(ms_total - epi, 1e-6) / launches
    steps_per_launch = args.steps / launches
    gbs = BYTES_PER_NODE_STEP * N / (kern_ms * 1e-3) / 1e9  # c read once, written once per launch
    tflops = FLOPS_PER_NODE_STEP_CH * steps_per_launch * N / (kern_ms * 1e-3) / 1e12

    # measured HBM bytes per launch, only if taken on this exact kernel source
    traffic = None
    tpath = args.traffic or _traffic_path(n, ks)
    if os.path.exists(tpath):
        try:
            t = json.load(open(tpath))
            if (t.get("n") == n and t.get("kernel_src_sha256_16") == kernel_hash()
                    and t.get("ks") == ks):
                traffic = t.get("bytes_per_launch")
        except (OSError, ValueError):
            traffic = None

    # the library's choice for this plan: the seam-sharing kernel (unless switched off) where
    # the chunks round to whole workgroups of 4 and stay long enough for its barrier
    nch = -(-(-(-n // ty_.value)) // 4) * 4
    rmin = n // (nch // 4)
    shortest = rmin - 3 * (rmin + 2 * (ks - 1)) // 4
    seam = (ks >= 2 and S.tune_get(A.TUNE_STREAM2D_SEAM) != 1
            and shortest >= max(-(-(4 * ks) // 4) * 4, 8))
    kname = (f"k_explicit2d_seam<float, CH, {ks}>" if seam else f"k_explicit2d<float, CH, {dp_.value}, {ks}>")
    if ks >= 2:
        roof = {"bound": "alu", "achieved": tflops, "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": tflops / VALU_PEAK_TFLOPS, "traffic": traffic,
                "hbm_achieved_gbs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS}
    else:
        roof = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": gbs / HBM_PEAK_GBS, "traffic": traffic,
                "alu_achieved_tflops": tflops, "alu_frac": tflops / VALU_PEAK_TFLOPS}
    roof.update({"kernel": f"{kname} ({ks} fused steps per launch, {ty_.value} rows per wave)",
                 "kernel_ms": kern_ms, "launches": launches,
                 "effective_gbs_per_step": BYTES_PER_NODE_STEP * N * args.steps / (ms_total * 1e-3) / 1e9})

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "DOF-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"2D Cahn-Hilliard spinodal, {n}x{n} periodic, explicit split step, "
                               "dt=0.01, W=1, kappa=2, M=1", "dof": N, "parallelism": "single GPU"},
        "roofline": roof,
        "settle_ms": args.settle_ms,
    }
    if args.fuse:
        S.tune_set(A.TUNE_STREAM2D_FUSE, 0)
    del U, ws
    torch.cuda.empty_cache()
    if not args.no_extras:
        out["hbm"] = {"single_step_launch": single_step_hbm(n, 1000, stream),
                      "single_step_launch_16384": single_step_hbm(16384, 40, stream),
                      "copy_ceiling_1gib": copy_ceiling(1024, stream),
                      "copy_ceiling_32mib": copy_ceiling(32, stream)}
        out["valu_ceiling"] = fma_ceiling(stream)
        if out["roofline"]["bound"] == "alu":  # the same work against the measured FMA rate
            out["roofline"]["frac_of_fma_probe"] = out["roofline"]["achieved"] / out["valu_ceiling"]["tflops"]
        out["ac128_fp64"] = ac128_record(stream)
        out["adjoint"] = adjoint_record(stream)
        out["surrogate"] = surrogate_record(stream)
        out["implicit_ch3d128"] = implicit_record(20, stream)
        out["coupled_1024"] = coupled_record(stream)
        out["coupled_implicit_512"] = coupled_implicit_record(stream)
        from paper_2601_06079_amd import _abi as A
        out["implicit_ac2048_2d"] = implicit2d_record(stream, A.ALLEN_CAHN, 2048, steps=5)
        out["implicit_ac2048_2d_cg"] = implicit2d_record(stream, A.ALLEN_CAHN, 2048, steps=5,
                                                         krylov=A.KRYLOV_CG)
        out["implicit_ch512_2d"] = implicit2d_record(stream, A.CAHN_HILLIARD, 512, steps=5)
        out["implicit_ch512_2d_consistent"] = implicit2d_record(stream, A.CAHN_HILLIARD, 512, steps=5,
                                                                mass=A.MASS_CONSISTENT)
        out["lobatto_ch2048"] = lobatto_record(stream)
        out["implicit_ac2048_2d_lobatto"] = implicit2d_record(stream, A.ALLEN_CAHN, 2048, steps=5,
                                                              quad=A.QUAD_LOBATTO)
        out["eshelby_129"] = eshelby_record(stream)
        out["grain_2048"] = grain_record(stream)
        out["grain_implicit_1024"] = grain_implicit_record(stream)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(n, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
