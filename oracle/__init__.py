"""Python access to the plain FP64 CPU oracle (oracle/mgr_oracle.c).

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg import this package; the GPU product path never
does.  Every function works on float64 NumPy arrays and returns a new array
(the C library transforms a private copy in place).

What each function computes is documented in oracle/mgr_oracle.c, with the
paper passages (Sec. II-A, Eq. (1)-(2), Sec. III-A) that it follows.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None

_ERRORS = {1: "argument", 2: "shape", 3: "levels", 4: "coordinates", 6: "allocation"}


class OracleError(RuntimeError):
    pass


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        lib = ctypes.CDLL(_build.LIB)
        i64p = ctypes.POINTER(ctypes.c_int64)
        dp = ctypes.POINTER(ctypes.c_double)
        dpp = ctypes.POINTER(dp)
        for name in ("oracle_decompose", "oracle_recompose", "oracle_decompose_adjoint",
                     "oracle_recompose_adjoint"):
            fn = getattr(lib, name)
            fn.argtypes = [dp, ctypes.c_int, i64p, dpp, ctypes.c_int]
            fn.restype = ctypes.c_int
        lib.oracle_max_levels.argtypes = [ctypes.c_int, i64p]
        lib.oracle_max_levels.restype = ctypes.c_int
        lib.oracle_coefficients_level.argtypes = [dp, ctypes.c_int, i64p, dpp, ctypes.c_int]
        lib.oracle_coefficients_level.restype = ctypes.c_int
        lib.oracle_load_vector_level.argtypes = [dp, dp, ctypes.c_int, i64p, dpp, ctypes.c_int]
        lib.oracle_load_vector_level.restype = ctypes.c_int
        lib.oracle_correction_level.argtypes = [dp, ctypes.c_int, i64p, dpp, ctypes.c_int]
        lib.oracle_correction_level.restype = ctypes.c_int
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        lib.oracle_set_threads.restype = ctypes.c_int
        lib.oracle_class_map.argtypes = [ctypes.c_int, i64p, ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_uint8)]
        lib.oracle_class_map.restype = ctypes.c_int
        i32p = ctypes.POINTER(ctypes.c_int32)
        lib.oracle_quantize.argtypes = [ctypes.c_void_p, i32p, ctypes.c_int, ctypes.c_int, i64p, ctypes.c_int,
                                        ctypes.c_int, dp, i64p]
        lib.oracle_quantize.restype = ctypes.c_int
        lib.oracle_dequantize.argtypes = [i32p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, i64p, ctypes.c_int,
                                          ctypes.c_int, dp]
        lib.oracle_dequantize.restype = ctypes.c_int
        lib.oracle_quant_bins.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, dp]
        lib.oracle_quant_bins.restype = ctypes.c_int
        _lib = lib
    return _lib


def _shape_arg(shape):
    arr = (ctypes.c_int64 * len(shape))(*[int(s) for s in shape])
    return arr


def _coords_arg(shape, coords):
    """Returns (ctypes double** or None, keep-alive list)."""
    if coords is None:
        return None, []
    keep = []
    ptrs = (ctypes.POINTER(ctypes.c_double) * len(shape))()
    for d, c in enumerate(coords):
        if c is None:
            ptrs[d] = ctypes.POINTER(ctypes.c_double)()
            continue
        a = np.ascontiguousarray(c, dtype=np.float64)
        if a.shape != (shape[d],):
            raise ValueError(f"coords[{d}] must have length {shape[d]}")
        keep.append(a)
        ptrs[d] = a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return ctypes.cast(ptrs, ctypes.POINTER(ctypes.POINTER(ctypes.c_double))), keep


def _check(rc):
    if rc != 0:
        raise OracleError(f"oracle error {rc} ({_ERRORS.get(rc, '?')})")


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def set_threads(n):
    """Threads for the oracle's loops over independent fibres and nodes
    (results do not depend on it); returns the previous count."""
    return _load().oracle_set_threads(int(n))


def max_levels(shape):
    return _load().oracle_max_levels(len(shape), _shape_arg(shape))


def _run(name, u, coords, nlevels):
    lib = _load()
    a = np.array(u, dtype=np.float64, order="C", copy=True)
    cp, keep = _coords_arg(a.shape, coords)
    _check(getattr(lib, name)(_dp(a), a.ndim, _shape_arg(a.shape), cp, int(nlevels)))
    del keep
    return a


def decompose(u, coords=None, nlevels=-1):
    """Multilevel decomposition (Sec. II-A, Eq. (1)-(2)) in FP64."""
    return _run("oracle_decompose", u, coords, nlevels)


def recompose(u, coords=None, nlevels=-1):
    """Exact inverse of decompose (Sec. II-A, recomposition)."""
    return _run("oracle_recompose", u, coords, nlevels)


def decompose_adjoint(g, coords=None, nlevels=-1):
    """Transpose of decompose under the Euclidean inner product."""
    return _run("oracle_decompose_adjoint", g, coords, nlevels)


def recompose_adjoint(g, coords=None, nlevels=-1):
    """Transpose of recompose (the inverse transpose of decompose)."""
    return _run("oracle_recompose_adjoint", g, coords, nlevels)


def coefficients_level(u, k, coords=None):
    """Coefficient stage of level step k only (Sec. II-A.1)."""
    return _run("oracle_coefficients_level", u, coords, k)


def level_size(n, k):
    """Nodes of the level-k grid (k steps from the finest) along a dimension
    of n nodes: the multiples of 2^k below n and the last node."""
    return ((n - 2) >> k) + 2


def level_indices(n, k):
    """Full-grid indices of that level grid, in order."""
    return np.minimum(np.arange(level_size(n, k), dtype=np.int64) << k, n - 1)


def load_vector_level(u, k, coords=None):
    """Load vector f = R M vec(C) of level step k, packed (Sec. II-A.2)."""
    lib = _load()
    a = np.ascontiguousarray(u, dtype=np.float64)
    cshape = tuple(level_size(n, k + 1) for n in a.shape)
    f = np.zeros(cshape, dtype=np.float64)
    cp, keep = _coords_arg(a.shape, coords)
    _check(lib.oracle_load_vector_level(_dp(a), _dp(f), a.ndim, _shape_arg(a.shape), cp, int(k)))
    del keep
    return f


def correction_level(f, shape, k, coords=None):
    """Solves M_{l-1} z = f for level step k (Sec. II-A.2); f packed."""
    lib = _load()
    z = np.array(f, dtype=np.float64, order="C", copy=True)
    cp, keep = _coords_arg(tuple(shape), coords)
    _check(lib.oracle_correction_level(_dp(z), len(shape), _shape_arg(shape), cp, int(k)))
    del keep
    return z


def class_map(shape, nlevels=-1):
    """Coefficient class of every node (0 = coarsest values, L = finest)."""
    lib = _load()
    out = np.zeros(tuple(shape), dtype=np.uint8)
    _check(lib.oracle_class_map(len(shape), _shape_arg(shape), int(nlevels),
                                out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))))
    return out


# ---- class-packed layout and progressive recomposition ----------------------
# The paper's use of the refactored data (Sec. I; Sec. II-A, overall
# process): coefficient classes are stored and moved separately, and a
# reader that has only the coarsest classes 0..l reconstructs a lower-
# fidelity approximation.  The layout here: class 0, then class 1, ...,
# class L, each a contiguous segment holding its nodes in C order of their
# grid indices.


def class_offsets(shape, nlevels=-1):
    """Start of each class's segment in the class-packed layout, plus the
    total: offsets[l] .. offsets[l + 1] hold class l (length L + 2)."""
    cm = class_map(shape, nlevels)
    L = max_levels(shape) if nlevels < 0 else nlevels
    counts = [int(np.count_nonzero(cm == l)) for l in range(L + 1)]
    return np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)


def pack_classes(y, nlevels=-1):
    """In-place node-order layout -> class-packed layout (a flat array):
    the values of class 0, then class 1, ..., each in C order (NumPy boolean
    indexing walks the array in C order)."""
    y = np.asarray(y)
    cm = class_map(y.shape, nlevels)
    L = max_levels(y.shape) if nlevels < 0 else nlevels
    return np.concatenate([y[cm == l] for l in range(L + 1)])


def unpack_classes(p, shape, nlevels=-1):
    """Class-packed layout -> in-place node-order layout (inverse of
    pack_classes).  A prefix holding only classes 0..l unpacks with the
    finer classes set to zero."""
    p = np.asarray(p)
    cm = class_map(shape, nlevels)
    L = max_levels(shape) if nlevels < 0 else nlevels
    off = class_offsets(shape, nlevels)
    out = np.zeros(tuple(shape), dtype=p.dtype)
    for l in range(L + 1):
        if off[l + 1] <= p.size:
            out[cm == l] = p[off[l]:off[l + 1]]
    return out


def recompose_level(y, level, coords=None, nlevels=-1):
    """Progressive recomposition (Sec. II-A, overall process): recompose the
    refactored array y with every class finer than `level` omitted (set to
    zero), and return the result at the level-`level` nodes (every index a
    multiple of 2^(L - level)), i.e. the nodal values of Q_level u."""
    y = np.asarray(y, dtype=np.float64)
    L = max_levels(y.shape) if nlevels < 0 else nlevels
    cm = class_map(y.shape, L)
    z = np.where(cm <= level, y, 0.0)
    r = recompose(z, coords, L)
    return np.ascontiguousarray(r[np.ix_(*[level_indices(n, L - level) for n in y.shape])])


# ---- quantisation of the classes (Sec. V, lossy compression) -----------------
# Reading (the paper names the stage, not the quantiser): per-class uniform
# scalar quantiser, code = round-half-even(y / b_class) in the data's own
# precision, clamped to +-(2^31 - 1) (NaN to 0); dequantised value
# code * b_class in that precision.


def _dtype_code(a):
    if a.dtype == np.float32:
        return 0
    if a.dtype == np.float64:
        return 1
    raise TypeError("float32 or float64")


def quant_bins(ndim, nlevels, tol):
    """Bin widths (nlevels + 1) for a max-norm bound tol on the recomposed
    field (derivation in oracle/mgr_oracle.c)."""
    b = np.zeros(nlevels + 1, dtype=np.float64)
    _check(_load().oracle_quant_bins(int(ndim), int(nlevels), float(tol), _dp(b)))
    return b


def quantize(y, bins, nlevels=-1, packed=False, shape=None):
    """Codes (int32, same flat order as y) and the clamped count.  y is the
    in-place layout (its own shape) or, with packed=True, the class-packed
    layout of `shape`."""
    y = np.ascontiguousarray(y)
    shape = tuple(y.shape) if shape is None else tuple(shape)
    b = np.ascontiguousarray(bins, dtype=np.float64)
    q = np.zeros(y.shape, dtype=np.int32)
    nc = ctypes.c_int64(0)
    _check(_load().oracle_quantize(y.ctypes.data, q.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                   _dtype_code(y), len(shape), _shape_arg(shape), int(nlevels), int(bool(packed)),
                                   _dp(b), ctypes.byref(nc)))
    return q, int(nc.value)


def dequantize(q, bins, dtype, nlevels=-1, packed=False, shape=None):
    """Values code * bin in `dtype` (numpy float32 or float64)."""
    q = np.ascontiguousarray(q, dtype=np.int32)
    shape = tuple(q.shape) if shape is None else tuple(shape)
    b = np.ascontiguousarray(bins, dtype=np.float64)
    y = np.zeros(q.shape, dtype=dtype)
    _check(_load().oracle_dequantize(q.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), y.ctypes.data,
                                     _dtype_code(y), len(shape), _shape_arg(shape), int(nlevels), int(bool(packed)),
                                     _dp(b)))
    return y
