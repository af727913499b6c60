"""ctypes binding of libpfhip.so (declared in include/pf.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of the library.  PyTorch supplies device memory and the current
stream.  If the library is missing this module raises on first use; there is
no CPU fallback.
"""
from __future__ import annotations

import atexit
import ctypes as ct
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpfhip.so")

PF_OK, PF_EINVAL, PF_EDEVICE, PF_ENOCONV, PF_ENONFINITE, PF_EUNSUPPORTED = range(6)
HOST_ONLY = -1  # pf_create: a context without a device (sizing and validation)
VJP_THETA_HOST = 1  # pf_vjp flags: theta_bar is a host pointer
BATCH_MAX_COUNT = 1 << 20
PERIODIC, NOFLUX = 0, 1
ALLEN_CAHN, CAHN_HILLIARD, COUPLED, GRAIN = 0, 1, 2, 3
F_SYM, F_01 = 0, 1
F32, F64 = 0, 1
MASS_LUMPED, MASS_CONSISTENT = 0, 1
QUAD_GAUSS, QUAD_LOBATTO = 0, 1
OP_RESIDUAL, OP_STEP_EXPLICIT, OP_ENERGY, OP_NEWTON, OP_VJP, OP_JVP = range(6)
TUNE_STREAM2D_ROWS, TUNE_STREAM2D_DEPTH, TUNE_STREAM2D_FUSE, TUNE_JVP3D_PLANES = 0, 1, 2, 3
TUNE_STREAM2D_SEAM = 6
TUNE_NN_GROUP = 7
TUNE_GS_REORTH = 8
TUNE_GG_STREAM = 9
TUNE_JVP2D_STREAM = 10
PRECOND_NONE, PRECOND_JACOBI = 0, 1
VJP_RESIDUAL, VJP_EXPLICIT_STEP, VJP_NEWTON_STEP = 0, 1, 2
VJP_BEGIN, VJP_END = 1, 2  # flags of pf_vjp_explicit_batched


class pf_problem(ct.Structure):
    _fields_ = [("dim", ct.c_int32), ("bc", ct.c_int32), ("model", ct.c_int32),
                ("fe", ct.c_int32), ("dtype", ct.c_int32), ("mass", ct.c_int32),
                ("n", ct.c_int64 * 3), ("h", ct.c_double), ("W", ct.c_double),
                ("kappa", ct.c_double), ("mobility", ct.c_double), ("mobility_eta", ct.c_double),
                ("nfields", ct.c_int32), ("quad", ct.c_int32), ("gamma", ct.c_double)]


KRYLOV_GMRES, KRYLOV_CG = 0, 1


class pf_newton_opts(ct.Structure):
    _fields_ = [("rtol", ct.c_double), ("atol", ct.c_double), ("max_newton", ct.c_int32),
                ("gmres_restart", ct.c_int32), ("gmres_max_its", ct.c_int32),
                ("precond", ct.c_int32), ("lin_rtol_max", ct.c_double),
                ("lin_rtol_min", ct.c_double), ("stagnation", ct.c_int32),
                ("krylov", ct.c_int32)]


class pf_newton_report(ct.Structure):
    _fields_ = [("newton_its", ct.c_int32), ("gmres_its", ct.c_int32),
                ("converged", ct.c_int32), ("reason", ct.c_int32),
                ("res_norm", ct.c_double * 33)]


class pf_batch_sample(ct.Structure):
    _fields_ = [("offset", ct.c_int64), ("n", ct.c_int64 * 3), ("h", ct.c_double),
                ("W", ct.c_double), ("kappa", ct.c_double), ("mobility", ct.c_double)]


class pf_batch_info(ct.Structure):
    _fields_ = [("count", ct.c_int32), ("n_items", ct.c_int32), ("fe", ct.c_int32),
                ("ks", ct.c_int32), ("ty", ct.c_int32), ("depth", ct.c_int32),
                ("model", ct.c_int32), ("dtype", ct.c_int32), ("total", ct.c_int64),
                ("plan_bytes", ct.c_int64), ("dt", ct.c_double), ("off_samples", ct.c_int64),
                ("off_items", ct.c_int64), ("reserved1", ct.c_int64)]


class PFError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"pf status {status}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load libpfhip.so (built in-tree by paper_2601_06079_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run paper_2601_06079_amd/build.py "
                           "(there is no CPU fallback)")
    L = ct.CDLL(LIB_PATH)
    P = ct.POINTER(pf_problem)
    vp, i32, i64, f64 = ct.c_void_p, ct.c_int, ct.c_int64, ct.c_double
    ip = ct.POINTER(ct.c_int)
    sig = {
        "pf_last_error": (ct.c_char_p, []),
        "pf_version": (i32, []),
        "pf_create": (i32, [i32, ct.POINTER(vp)]),
        "pf_destroy": (i32, [vp]),
        "pf_ctx_device": (i32, [vp, ip]),
        "pf_tune_set": (i32, [i32, i32]),
        "pf_tune_get": (i32, [i32, ip]),
        "pf_launch_shape": (i32, [vp, P, ip, ip, ip]),
        "pf_workspace_size": (i32, [vp, P, i32, ct.POINTER(ct.c_size_t)]),
        "pf_residual": (i32, [vp, P, vp, vp, vp, vp]),
        "pf_step_explicit": (i32, [vp, P, f64, i64, vp, vp, vp]),
        "pf_energy": (i32, [vp, P, vp, vp, vp, vp]),
        "pf_jvp": (i32, [vp, P, f64, vp, vp, vp, vp]),
        "pf_newton_default_opts": (None, [ct.POINTER(pf_newton_opts)]),
        "pf_newton_step": (i32, [vp, P, f64, vp, vp, ct.POINTER(pf_newton_opts),
                                 ct.POINTER(pf_newton_report), vp, vp]),
        "pf_vjp": (i32, [vp, P, i32, f64, vp, vp, vp, vp, vp, i32, vp, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


_ctxs = {}


def ctx(device=None) -> ct.c_void_p:
    """The library's default context for a device (torch's current device when
    None): made by pf_create on first use, freed by pf_destroy at exit."""
    if device is None or getattr(device, "type", None) == "cuda":
        index = getattr(device, "index", None)
        if index is None:
            import torch
            index = torch.cuda.current_device()
        device = index
    device = int(device)
    h = _ctxs.get(device)
    if h is None:
        h = ct.c_void_p()
        check(lib().pf_create(device, ct.byref(h)))
        _ctxs[device] = h
    return h


def host_ctx() -> ct.c_void_p:
    """A context without a device: size queries and argument validation only."""
    return ctx(HOST_ONLY)


def _destroy_contexts():
    if _lib is None:
        return
    for h in _ctxs.values():
        _lib.pf_destroy(h)
    _ctxs.clear()


atexit.register(_destroy_contexts)


def bind_optional(name, restype, argtypes):
    """Bind an export added by a later section of the library (None if absent)."""
    L = lib()
    if not hasattr(L, name):
        return None
    fn = getattr(L, name)
    fn.restype = restype
    fn.argtypes = argtypes
    return fn


def check(status: int, allow=()):
    if status == PF_OK or status in allow:
        return status
    msg = lib().pf_last_error()
    raise PFError(status, msg.decode() if msg else "")


def exported_symbols():
    """Names declared in include/pf.h (parsed from the header text)."""
    import re
    hdr = os.path.join(os.path.dirname(_HERE), "include", "pf.h")
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(pf_[a-z_0-9]+)\s*\(",
                       open(hdr).read(), flags=re.M)
    return sorted(set(names))
