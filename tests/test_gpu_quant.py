"""GPU quantisation of the refactored classes against the CPU oracle.

Codes are integers decided by floating point, so both sides take that
decision in the data's precision and the comparison is bit-exact: codes, the
clamped count and the dequantised values, in the in-place and the
class-packed layouts.  The whole lossy path (decompose, quantise with the
bins for a max-norm bound, dequantise, recompose) stays within the bound on
the GPU.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2007_04457_amd as mgr
from paper_2007_04457_amd import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

CASES = [
    # shape, dtype, nlevels, tol (relative to max|x|)
    ((257,), torch.float64, -1, 1e-4),
    ((129, 65), torch.float32, -1, 1e-3),
    ((33, 17, 65), torch.float64, -1, 1e-6),
    ((65, 65, 65), torch.float32, 3, 1e-2),
    ((9, 129, 33), torch.float32, -1, 1e-4),
    ((3, 5, 9), torch.float64, 1, 1e-3),
    ((1025, 3, 5), torch.float32, 1, 1e-3),
]


def case_id(c):
    return f"{'x'.join(map(str, c[0]))}-{str(c[1]).split('.')[-1]}-L{c[2]}"


def refactored(shape, dtype, L, seed=11):
    u, _ = synth.sinusoid_field(shape, seed)
    x = torch.from_numpy(u).to(dtype).to(DEV)
    return x, mgr.decompose(x, None, L)


@pytest.mark.parametrize("packed", [False, True], ids=["inplace", "packed"])
@pytest.mark.parametrize("case", CASES, ids=[case_id(c) for c in CASES])
def test_quantize_dequantize_bitwise(case, packed):
    shape, dt, L, tol = case
    print(f"\n[quant] {case_id(case)} packed={packed}", flush=True)
    x, y = refactored(shape, dt, L)
    Lf = mgr.mgr_max_levels(shape) if L < 0 else L
    bins = mgr.quant_bins(len(shape), Lf, tol * float(x.abs().max()))
    src = mgr.pack_classes(y, L) if packed else y
    codes, nc = mgr.quantize(src, bins, shape, L, packed)
    back = mgr.dequantize(codes, bins, dt, shape, L, packed)
    torch.cuda.synchronize()
    host = src.cpu().numpy()
    want, wnc = oracle.quantize(host, bins, L, packed, shape)
    assert np.array_equal(codes.cpu().numpy(), want)
    assert int(nc.item()) == wnc == 0
    wback = oracle.dequantize(want, bins, host.dtype, L, packed, shape)
    assert np.array_equal(back.cpu().numpy(), wback)


@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
@pytest.mark.parametrize("packed", [False, True], ids=["inplace", "packed"])
def test_ties_clamping_and_nan(dt, packed):
    """Exact ties round half to even, quotients past the int32 range and NaN
    are clamped and counted, the same as the oracle."""
    shape = (17, 9, 33)
    L = mgr.mgr_max_levels(shape)
    bins = np.array([2.0 ** -(c % 5) for c in range(L + 1)])
    rng = np.random.default_rng(5)
    n = int(np.prod(shape))
    k = rng.integers(-1000, 1000, n).astype(np.float64)
    y = k + 0.5  # ties in units of a bin, scaled per class below
    cls = oracle.class_map(shape, L).reshape(-1)
    if packed:
        off = oracle.class_offsets(shape, L)
        cls = np.repeat(np.arange(L + 1), np.diff(off))
    y = y * bins[cls]
    y[::97] = 3e12  # beyond 2^31 - 1 bins
    y[5::89] = -3e12
    y[7::101] = np.nan
    y[11::103] = np.inf
    y = y.reshape(shape if not packed else (n,))
    host = y.astype(np.float32 if dt == torch.float32 else np.float64)
    t = torch.from_numpy(host).to(DEV)
    codes, nc = mgr.quantize(t, bins, shape, L, packed)
    torch.cuda.synchronize()
    want, wnc = oracle.quantize(host, bins, L, packed, shape)
    assert wnc > 0
    assert np.array_equal(codes.cpu().numpy(), want)
    assert int(nc.item()) == wnc
    back = mgr.dequantize(codes, bins, dt, shape, L, packed)
    assert np.array_equal(back.cpu().numpy(), oracle.dequantize(want, bins, host.dtype, L, packed, shape))


@pytest.mark.parametrize("case", CASES, ids=[case_id(c) for c in CASES])
def test_lossy_roundtrip_within_bound(case):
    """decompose -> quantise (bins for tol) -> dequantise -> recompose, all on
    the GPU, lands within tol of the input in the max norm (float32: plus the
    float32 parity gate of the two transforms, 2e-5 of max|x|)."""
    shape, dt, L, tol = case
    x, y = refactored(shape, dt, L, seed=12)
    Lf = mgr.mgr_max_levels(shape) if L < 0 else L
    scale = float(x.abs().max())
    bound = tol * scale
    bins = mgr.quant_bins(len(shape), Lf, bound)
    codes, nc = mgr.quantize(y, bins, None, L)
    r = mgr.recompose(mgr.dequantize(codes, bins, dt, None, L), None, L)
    torch.cuda.synchronize()
    err = float((r.double() - x.double()).abs().max())
    slack = 2e-5 * scale if dt == torch.float32 else 1e-12 * scale
    assert int(nc.item()) == 0
    assert err <= bound + slack, (err, bound)


def test_full_size_quantize_513_float32():
    """513^3 float32 sinusoid field: every code of the class-packed layout
    and the clamped count against the oracle."""
    shape = (513, 513, 513)
    print("\n[quant] 513^3 float32", flush=True)
    u, _ = synth.sinusoid_field(shape, 1)
    x = torch.from_numpy(u).to(torch.float32).to(DEV)
    del u
    y = mgr.decompose(x)
    L = mgr.mgr_max_levels(shape)
    bins = mgr.quant_bins(3, L, 1e-4 * float(x.abs().max()))
    p = mgr.pack_classes(y)
    codes, nc = mgr.quantize(p, bins, shape, L, packed=True)
    torch.cuda.synchronize()
    want, wnc = oracle.quantize(p.cpu().numpy(), bins, L, True, shape)
    assert np.array_equal(codes.cpu().numpy(), want)
    assert int(nc.item()) == wnc == 0
