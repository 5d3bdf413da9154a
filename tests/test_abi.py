"""The C ABI library loads and exports what include/mgr.h declares, and its
host-side validation behaves (CPU only: nothing here launches a kernel)."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
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
    assert lib.mgr_max_levels(2, _lib.shape_arg((10, 9))) == -2
    assert lib.mgr_max_levels(4, _lib.shape_arg((9, 9, 9, 9))) == -1


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
    assert _call(lib, fn, (10, 9)) == 2
    assert _call(lib, fn, (2, 9)) == 2
    assert _call(lib, fn, (9, 9), nlevels=4) == 3
    assert _call(lib, fn, (9, 9), nlevels=-2) == 3
    assert _call(lib, fn, (9, 9), dtype=7) == 1
    assert _call(lib, fn, (9, 9, 9, 9)) == 1
    bad = [np.array([0, 1, 2, 3, 3, 5, 6, 7, 8.0]), None]
    assert _call(lib, fn, (9, 9), coords=bad) == 4
    nan = [np.array([0, 1, 2, np.nan, 4, 5, 6, 7, 8.0]), None]
    assert _call(lib, fn, (9, 9), coords=nan) == 4
    assert _call(lib, fn, (9, 9), ptr=0) == 1
    assert lib.mgr_last_error().decode() != ""


def test_status_strings(lib):
    for s in range(8):
        assert lib.mgr_status_string(s).decode()
    assert lib.mgr_kernel_name(0).decode() == "coef_decompose"
    assert lib.mgr_kernel_name(999) is None


def test_bench_copy_validation(lib):
    assert lib.mgr_bench_copy(None, None, 16, None) == 1
    assert lib.mgr_bench_copy(16, 32, 15, None) == 1
