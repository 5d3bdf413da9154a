"""The allocation-free decomposition (mgr_decompose_noalloc) against
mgr_decompose, through the C ABI: two calls in a row on the library's
device scratch array, the second with a smaller problem, each equal to the
per-problem path bit for bit (same kernels, same arithmetic) and to the
oracle within the parity tolerance; a problem larger than the array is
refused before anything is enqueued."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import paper_2007_04457_amd as mgr
from paper_2007_04457_amd import _lib, synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = {torch.float64: 1e-12, torch.float32: 2e-5}


def noalloc(src, dst, coords=None, nlevels=-1):
    lib = _lib.load()
    cp, keep = _lib.coords_arg(tuple(src.shape), coords)
    code = _lib.MGR_F32 if src.dtype == torch.float32 else _lib.MGR_F64
    st = lib.mgr_decompose_noalloc(src.data_ptr(), dst.data_ptr(), code, src.dim(), _lib.shape_arg(src.shape), cp,
                                   int(nlevels), torch.cuda.current_stream().cuda_stream)
    del keep
    return st


@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
def test_noalloc_two_calls_smaller_second(dt):
    cases = [((129, 65, 257), True, -1), ((33, 17, 65), False, 3)]
    outs = []
    for shape, nu, L in cases:
        print(f"\n[noalloc] {shape} {dt} nonuniform={nu} L={L}", flush=True)
        u, coords = synth.sinusoid_field(shape, 21, nonuniform=nu)
        x = torch.from_numpy(u).to(dt).to(DEV)
        y = torch.full_like(x, float("nan"))
        assert noalloc(x, y, coords, L) == 0, _lib.load().mgr_last_error().decode()
        ref = mgr.decompose(x, coords, L)
        torch.cuda.synchronize()
        outs.append((x, y, ref, coords, L))
    for x, y, ref, coords, L in outs:
        assert torch.equal(y, ref)
        xd = x.double().cpu().numpy()
        want = oracle.decompose(xd, coords, L)
        err = float(np.max(np.abs(y.double().cpu().numpy() - want))) / float(np.max(np.abs(xd)))
        assert err <= TOL[dt], err


def test_noalloc_in_place_and_repeat():
    shape = (65, 65, 65)
    u, _ = synth.blob_field(shape, 22)
    x = torch.from_numpy(u).to(torch.float32).to(DEV)
    ref = mgr.decompose(x)
    for _ in range(2):
        z = x.clone()
        assert noalloc(z, z) == 0
        torch.cuda.synchronize()
        assert torch.equal(z, ref)


def test_noalloc_refuses_too_large_problem():
    lib = _lib.load()
    shape = (513, 513, 513)
    st = lib.mgr_decompose_noalloc(16, 16, _lib.MGR_F64, 3, _lib.shape_arg(shape), None, -1, None)
    assert st == 6  # MGR_ERR_ALLOC, nothing enqueued
    assert "scratch" in lib.mgr_last_error().decode()
