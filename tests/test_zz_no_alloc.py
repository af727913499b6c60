"""pf_energy_noalloc: the energy reduction with its partial sums in the library's
static device scratch (for callers that cannot allocate), against pf_energy with a
caller-provided workspace, through the C ABI."""
import ctypes as ct

import numpy as np
import pytest
import torch

from paper_2601_06079_amd import _abi as A
from paper_2601_06079_amd import solver as S

pytestmark = pytest.mark.gpu


def _fn():
    L = A.lib()
    f = L.pf_energy_noalloc
    f.restype = ct.c_int
    f.argtypes = [ct.c_void_p, ct.POINTER(A.pf_problem), ct.c_void_p, ct.c_void_p, ct.c_void_p]
    return f


def _stream():
    return ct.c_void_p(torch.cuda.current_stream().cuda_stream)


def _case(n, model, dtype, seed):
    fe = A.F_01 if model == A.CAHN_HILLIARD else A.F_SYM
    p = S.Problem(n=n, model=model, fe=fe, dtype=dtype, W=1.2, kappa=1.7, mobility=1.0, h=0.9)
    U = torch.as_tensor(np.random.default_rng(seed).uniform(-0.8, 0.8, p.ndof), dtype=dtype, device="cuda")
    return p, U


def _noalloc(p, U):
    out = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
    A.check(_fn()(A.ctx(), ct.byref(p.c()), ct.c_void_p(U.data_ptr()), ct.c_void_p(out.data_ptr()), _stream()))
    return out


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_noalloc_energy_matches_workspace_energy_twice(dtype):
    """Two calls in a row, the second on a smaller grid (the scratch keeps the first
    call's partials beyond the second's range): each equals pf_energy bitwise (same
    kernels, same fixed reduction order)."""
    for n, model, seed in (((1024, 1000), A.CAHN_HILLIARD, 1), ((37, 29), A.ALLEN_CAHN, 2),
                           ((24, 20, 18), A.CAHN_HILLIARD, 3), ((9, 7), A.ALLEN_CAHN, 4)):
        p, U = _case(n, model, dtype, seed)
        got = _noalloc(p, U)
        ref = S.energy(p, U)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), (n, got, ref)


def test_noalloc_energy_other_models_and_limit():
    """The coupled and grain-growth energies share the reduction; a grid beyond the
    scratch's capacity is rejected before anything is enqueued."""
    pc = S.Problem(n=(96, 80), model=A.COUPLED, dtype=torch.float32, kappa=0.3, mobility=1.0,
                   mobility_eta=150.0)
    Uc = torch.as_tensor(np.random.default_rng(5).uniform(0, 1, pc.ndof), dtype=torch.float32, device="cuda")
    assert torch.equal(_noalloc(pc, Uc), S.energy(pc, Uc))
    pg = S.Problem(n=(64, 48), model=A.GRAIN, dtype=torch.float32, kappa=1.0, mobility=1.0, nfields=5, gamma=1.5)
    Ug = torch.as_tensor(np.random.default_rng(6).uniform(0, 1, pg.ndof), dtype=torch.float32, device="cuda")
    assert torch.equal(_noalloc(pg, Ug), S.energy(pg, Ug))
    big = S.Problem(n=(4097, 4096), model=A.ALLEN_CAHN, dtype=torch.float32)
    fake = torch.empty(8, dtype=torch.float32, device="cuda")
    out = torch.empty(2, dtype=torch.float64, device="cuda")
    st = _fn()(A.ctx(), ct.byref(big.c()), ct.c_void_p(fake.data_ptr()), ct.c_void_p(out.data_ptr()), _stream())
    assert st == A.PF_EINVAL and b"scratch" in A.lib().pf_last_error()
