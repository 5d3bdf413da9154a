"""The C ABI library loads and exports what include/mgr.h declares, and its
host-side validation behaves (CPU only: nothing here launches a kernel)."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_2007_04457_amd as mgr
from paper_2007_04457_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(mgr_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2007_04457_amd import build
        build.build()
    return _lib.load()


def test_exports_every_declared_symbol(lib):
    names = declared_symbols()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n


def test_max_levels(lib):
    assert lib.mgr_max_levels(3, _lib.shape_arg((513, 513, 513))) == 8
    assert lib.mgr_max_levels(2, _lib.shape_arg((8193, 8193))) == 12
    assert lib.mgr_max_levels(3, _lib.shape_arg((1025, 1025, 257))) == 7
    assert lib.mgr_max_levels(3, _lib.shape_arg((65, 65, 65))) == 5
    # any size >= 3 and up to four dimensions (nested grids keep the last
    # node): the oracle's count
    for shape in [(10, 9), (9, 9, 9, 9), (3, 100), (6, 7, 12, 5), (1000,), (33, 20, 513)]:
        assert lib.mgr_max_levels(len(shape), _lib.shape_arg(shape)) == oracle.max_levels(shape), shape
    assert lib.mgr_max_levels(2, _lib.shape_arg((2, 9))) == -2
    assert lib.mgr_max_levels(5, _lib.shape_arg((9, 9, 9, 9, 9))) == -1


@pytest.mark.parametrize("shape,L", [((10, 9), -1), ((6, 7, 12, 5), -1), ((6, 7, 12, 5), 1), ((100,), 3),
                                     ((5, 17, 9, 9), -1), ((20, 3, 13), 1)])
def test_class_map_general_shapes_matches_oracle(lib, shape, L):
    from paper_2007_04457_amd import mgr_class_map
    assert np.array_equal(mgr_class_map(shape, L), oracle.class_map(shape, L))


@pytest.mark.parametrize("shape,L", [((17, 9, 33), -1), ((17, 9, 33), 3), ((65,), 2), ((9, 17), 1)])
def test_class_map_matches_oracle(lib, shape, L):
    from paper_2007_04457_amd import mgr_class_map
    assert np.array_equal(mgr_class_map(shape, L), oracle.class_map(shape, L))


def _call(lib, fn, shape, nlevels=-1, coords=None, dtype=0, ptr=16):
    cp, keep = _lib.coords_arg(shape, coords)
    return getattr(lib, fn)(ptr, ptr, dtype, len(shape), _lib.shape_arg(shape), cp, nlevels, None)


@pytest.mark.parametrize("fn", ["mgr_decompose", "mgr_recompose", "mgr_decompose_adjoint"])
def test_validation_errors_before_any_device_work(lib, fn):
    # validation happens before any HIP call, so these run without a GPU
    general = fn in ("mgr_decompose", "mgr_recompose")  # any size >= 3, up to 4-D
    if general:
        # accepted; the call then needs a device (here: a HIP status)
        assert _call(lib, fn, (10, 9)) not in (1, 2, 3, 4)
        assert _call(lib, fn, (9, 9, 9, 9)) not in (1, 2, 3, 4)
        assert _call(lib, fn, (10, 9), nlevels=4) == 3
    else:
        assert _call(lib, fn, (10, 9)) == 2
        assert _call(lib, fn, (9, 9, 9, 9)) == 2
    assert _call(lib, fn, (9, 9, 9, 9, 9)) == 1
    assert _call(lib, fn, (2, 9)) == 2
    assert _call(lib, fn, (9, 9), nlevels=4) == 3
    assert _call(lib, fn, (9, 9), nlevels=-2) == 3
    assert _call(lib, fn, (9, 9), dtype=7) == 1
    bad = [np.array([0, 1, 2, 3, 3, 5, 6, 7, 8.0]), None]
    assert _call(lib, fn, (9, 9), coords=bad) == 4
    nan = [np.array([0, 1, 2, np.nan, 4, 5, 6, 7, 8.0]), None]
    assert _call(lib, fn, (9, 9), coords=nan) == 4
    assert _call(lib, fn, (9, 9), ptr=0) == 1
    assert lib.mgr_last_error().decode() != ""


def test_plane_addressing_limit(lib):
    """Planes of 2 GiB or more are refused before any device work: the
    kernels address within a plane with 32-bit byte offsets."""
    assert _call(lib, "mgr_decompose", (2 ** 29 + 1,), dtype=0) == 2          # 1-D float32, 2 GiB + 4 B
    assert _call(lib, "mgr_decompose", (3, 2 ** 28 + 1), dtype=1) == 2       # 2-D float64 row
    assert _call(lib, "mgr_decompose_adjoint", (3, 16385, 16385), dtype=1) == 2
    assert "2 GiB" in lib.mgr_last_error().decode()
    assert _call(lib, "mgr_recompose", (3, 16385, 32769), dtype=0) == 2      # float32, 2 GiB + 192 KiB
    # the largest accepted planes (validation passes; the call then needs a
    # device, so on a machine without one it fails later with a HIP status)
    assert _call(lib, "mgr_decompose", (2 ** 28 + 1,), dtype=0) not in (1, 2, 3, 4)
    assert _call(lib, "mgr_decompose", (3, 8193, 8193), dtype=1) not in (1, 2, 3, 4)


def test_status_strings(lib):
    for s in range(8):
        assert lib.mgr_status_string(s).decode()
    assert lib.mgr_kernel_name(0).decode() == "coef_decompose"
    assert lib.mgr_kernel_name(999) is None


def test_bench_copy_validation(lib):
    assert lib.mgr_bench_copy(None, None, 16, None) == 1
    assert lib.mgr_bench_copy(16, 32, 15, None) == 1


@pytest.mark.parametrize("shape,L", [((17, 9, 33), -1), ((9, 17), 1), ((33,), 0)])
def test_class_masks_partition_the_grid(shape, L):
    """class_masks: one mask per class 0..L, disjoint, covering every node,
    each equal to the oracle's class map at that class."""
    import oracle
    masks = mgr.class_masks(shape, L)
    full = oracle.max_levels(shape) if L < 0 else L
    assert len(masks) == full + 1
    cm = oracle.class_map(shape, L)
    total = np.zeros(shape, dtype=int)
    for l, m in enumerate(masks):
        assert np.array_equal(m, cm == l), l
        total += m
    assert np.all(total == 1)


@pytest.mark.parametrize("shape,L", [((17, 9, 33), -1), ((9, 17), 1), ((33,), 0), ((513, 513, 513), -1)])
def test_class_offsets_match_oracle(shape, L):
    if np.prod(shape) > 1e6:
        full = oracle.max_levels(shape)
        sizes = [int(np.prod([(n - 1) // 2 ** (full - l) + 1 for n in shape])) for l in range(full + 1)]
        want = np.concatenate([[0], np.cumsum([sizes[0]] + [sizes[l] - sizes[l - 1] for l in range(1, full + 1)])])
    else:
        want = oracle.class_offsets(shape, L)
    assert np.array_equal(mgr.class_offsets(shape, L), want)


def test_packed_and_progressive_validation(lib):
    """Argument errors of the class-packed and progressive entry points come
    back before any device work."""
    shp = _lib.shape_arg((9, 9))
    assert lib.mgr_pack_classes(16, 16, 0, 2, shp, -1, None) == 1          # in place
    assert lib.mgr_unpack_classes(16, 32, 0, 2, _lib.shape_arg((9, 10)), -1, None) == 2
    assert lib.mgr_pack_classes(0, 32, 0, 2, shp, -1, None) == 1
    assert lib.mgr_recompose_level(16, 32, 0, 2, shp, None, -1, 3, 0, None) == 3   # level > L
    assert lib.mgr_recompose_level(16, 32, 0, 2, shp, None, -1, -1, 0, None) == 3
    assert lib.mgr_recompose_level(16, 32, 0, 2, shp, None, -1, 1, 2, None) == 1   # bad layout flag
    assert lib.mgr_recompose_level(16, 16, 0, 2, shp, None, -1, 1, 0, None) == 1   # in place
    off = (ctypes.c_int64 * 4)()
    assert lib.mgr_class_offsets(2, shp, -1, off) == 0 and list(off) == [0, 9, 25, 81]


@pytest.mark.parametrize("ndim,L,tol", [(1, 5, 1e-3), (2, 12, 0.25), (3, 8, 1e-6), (3, 0, 2.0)])
def test_quant_bins_match_the_oracle(lib, ndim, L, tol):
    """The library's bin widths for a max-norm bound are the oracle's closed
    form, bit for bit (host code; both write b_0 = 2 tol / (L + 1) and
    b_c = 2 tol / ((L + 1)(1 + 3^ndim)))."""
    assert np.array_equal(mgr.quant_bins(ndim, L, tol), oracle.quant_bins(ndim, L, tol))


def test_quant_argument_errors(lib):
    """Validation of the quantisation entry points happens on the host,
    before anything is enqueued (no kernel runs here)."""
    dp = ctypes.POINTER(ctypes.c_double)
    shape = (17, 9)
    bins = np.ones(4, dtype=np.float64)
    bad = bins.copy()
    bad[2] = 0.0
    call = lambda b, L=3, packed=0, codes=16: lib.mgr_quantize(16, codes, 0, 2, _lib.shape_arg(shape), L, packed,
                                                               b.ctypes.data_as(dp) if b is not None else None,
                                                               None, None)
    assert call(None) == 1
    assert call(bad) == 1
    assert call(bins, codes=None) == 1
    assert call(bins, packed=2) == 1
    assert call(bins, L=9) == 3
    assert lib.mgr_quantize(16, 16, 0, 2, _lib.shape_arg((10, 9)), 3, 0, bins.ctypes.data_as(dp), None, None) == 2
    assert lib.mgr_dequantize(16, None, 0, 2, _lib.shape_arg(shape), 3, 0, bins.ctypes.data_as(dp), None) == 1
    out = np.zeros(4)
    assert lib.mgr_quant_bins(2, 3, -1.0, out.ctypes.data_as(dp)) == 1
    assert lib.mgr_quant_bins(4, 3, 1.0, out.ctypes.data_as(dp)) == 1

