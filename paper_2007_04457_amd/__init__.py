"""Multigrid hierarchical data refactoring on MI355X (gfx950).

Implements the multilevel decomposition of Chen et al., "Accelerating
Multigrid-based Hierarchical Scientific Data Refactoring on GPUs" (arXiv
2007.04457, Sec. II-A), its inverse and its adjoint, as HIP kernels behind the
C ABI of include/mgr.h.  This package is a thin binding: tensors must be
contiguous float32/float64 CUDA (HIP) tensors; torch supplies device memory
and the current stream, the library does all the arithmetic.

The C entry points are exposed under their own names (``mgr_decompose`` ...,
taking ``src`` and ``dst`` tensors), with out-of-place conveniences
(``decompose`` ...), an autograd function (``Decompose``) and the batched
work-queue decomposition (``BatchPlan``, over ``mgr_batch_*``).
"""
import numpy as np

from . import _lib
from ._lib import MgrError, MGR_F32, MGR_F64

__all__ = [
    "MgrError", "MGR_F32", "MGR_F64",
    "mgr_decompose", "mgr_recompose", "mgr_decompose_adjoint", "mgr_recompose_adjoint",
    "mgr_decompose_noalloc", "mgr_prepare",
    "mgr_class_map", "class_masks", "mgr_max_levels", "mgr_bench_copy", "mgr_finalize", "mgr_set_tail_max_nodes",
    "mgr_timing_enable", "mgr_timing_disable", "mgr_timing_read", "mgr_kernel_name",
    "decompose", "recompose", "decompose_adjoint", "recompose_adjoint", "Decompose", "Recompose",
    "kernel_classes", "BatchPlan", "batch_queue_check",
    "class_offsets", "pack_classes", "unpack_classes", "recompose_level",
    "quant_bins", "quantize", "dequantize",
]


def _torch():
    import torch
    return torch


def _dtype_code(t):
    torch = _torch()
    if t.dtype == torch.float32:
        return MGR_F32
    if t.dtype == torch.float64:
        return MGR_F64
    raise TypeError(f"unsupported dtype {t.dtype} (float32 or float64)")


def _check(t, name):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _call(fn_name, src, dst, coords, nlevels):
    _check(src, "src")
    _check(dst, "dst")
    if src.shape != dst.shape or src.dtype != dst.dtype or src.device != dst.device:
        raise ValueError("src and dst must have the same shape, dtype and device")
    lib = _lib.load()
    torch = _torch()
    cp, keep = _lib.coords_arg(tuple(src.shape), coords)
    stream = torch.cuda.current_stream(src.device).cuda_stream
    with torch.cuda.device(src.device):
        st = getattr(lib, fn_name)(src.data_ptr(), dst.data_ptr(), _dtype_code(src), src.dim(),
                                   _lib.shape_arg(src.shape), cp, int(nlevels), stream)
    del keep
    _lib.check(st)
    return dst


def mgr_decompose(src, dst, coords=None, nlevels=-1):
    """dst <- decomposition of src (dst may be src).  See include/mgr.h."""
    return _call("mgr_decompose", src, dst, coords, nlevels)


def mgr_decompose_noalloc(src, dst, coords=None, nlevels=-1):
    """mgr_decompose through the library's fixed device scratch array: the
    call allocates no device memory (see include/mgr.h)."""
    return _call("mgr_decompose_noalloc", src, dst, coords, nlevels)


def mgr_recompose(src, dst, coords=None, nlevels=-1):
    """dst <- recomposition of the refactored array src."""
    return _call("mgr_recompose", src, dst, coords, nlevels)


def mgr_decompose_adjoint(src, dst, coords=None, nlevels=-1):
    """dst <- D^T src, the transpose of the decomposition."""
    return _call("mgr_decompose_adjoint", src, dst, coords, nlevels)


def mgr_recompose_adjoint(src, dst, coords=None, nlevels=-1):
    """dst <- R^T src = D^{-T} src, the transpose of the recomposition."""
    return _call("mgr_recompose_adjoint", src, dst, coords, nlevels)


def mgr_prepare(dtype, shape, coords=None, nlevels=-1):
    """Builds tables and workspace ahead of time (before graph capture)."""
    code = _dtype_code(_torch().empty(0, dtype=dtype)) if not isinstance(dtype, int) else dtype
    lib = _lib.load()
    cp, keep = _lib.coords_arg(tuple(shape), coords)
    st = lib.mgr_prepare(code, len(shape), _lib.shape_arg(shape), cp, int(nlevels))
    del keep
    _lib.check(st)


def mgr_max_levels(shape):
    r = _lib.load().mgr_max_levels(len(shape), _lib.shape_arg(shape))
    if r < 0:
        _lib.check(-r)
    return r


def mgr_class_map(shape, nlevels=-1):
    """Class id of every node as a NumPy uint8 array (0 = coarsest)."""
    import ctypes
    import numpy as np
    out = np.zeros(tuple(int(s) for s in shape), dtype=np.uint8)
    lib = _lib.load()
    _lib.check(lib.mgr_class_map(len(shape), _lib.shape_arg(shape), int(nlevels),
                                 out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))))
    return out


def class_masks(shape, nlevels=-1, device=None):
    """One boolean mask per coefficient class of the refactored layout:
    masks[l] is True at the nodes holding class l (0 = the coarsest nodal
    values, L = the finest coefficients), from mgr_class_map.  NumPy arrays,
    or torch tensors on `device` when given."""
    cm = mgr_class_map(shape, nlevels)
    L = mgr_max_levels(shape) if int(nlevels) < 0 else int(nlevels)
    masks = [cm == l for l in range(L + 1)]
    if device is None:
        return masks
    torch = _torch()
    return [torch.from_numpy(m).to(device) for m in masks]


def class_offsets(shape, nlevels=-1):
    """Segment starts of the class-packed layout (L + 2 int64 values):
    class c occupies [offsets[c], offsets[c + 1])."""
    import ctypes
    import numpy as np
    L = mgr_max_levels(shape) if int(nlevels) < 0 else int(nlevels)
    out = np.zeros(L + 2, dtype=np.int64)
    _lib.check(_lib.load().mgr_class_offsets(len(shape), _lib.shape_arg(shape), int(nlevels),
                                             out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
    return out


def _pack_call(name, src, dst, shape, nlevels):
    _check(src, "src")
    _check(dst, "dst")
    if src.numel() != dst.numel() or src.dtype != dst.dtype or src.device != dst.device:
        raise ValueError("src and dst must have the same size, dtype and device")
    torch = _torch()
    stream = torch.cuda.current_stream(src.device).cuda_stream
    with torch.cuda.device(src.device):
        st = getattr(_lib.load(), name)(src.data_ptr(), dst.data_ptr(), _dtype_code(src), len(shape),
                                        _lib.shape_arg(shape), int(nlevels), stream)
    _lib.check(st)
    return dst


def pack_classes(y, nlevels=-1, out=None):
    """Class-packed layout (a flat tensor) of the refactored array y."""
    if out is None:
        out = _torch().empty(y.numel(), dtype=y.dtype, device=y.device)
    return _pack_call("mgr_pack_classes", y, out, tuple(y.shape), nlevels)


def unpack_classes(p, shape, nlevels=-1, out=None):
    """In-place layout of shape `shape` from a class-packed tensor p."""
    if out is None:
        out = _torch().empty(tuple(shape), dtype=p.dtype, device=p.device)
    return _pack_call("mgr_unpack_classes", p, out, tuple(shape), nlevels)


def recompose_level(src, level, shape=None, coords=None, nlevels=-1, packed=False, out=None):
    """Progressive recomposition: the nodal values of Q_level u on the
    level-`level` grid, from the classes 0..level of a refactored array
    (in-place layout of shape `shape`, or a class-packed tensor, of which a
    prefix of offsets[level + 1] elements is enough)."""
    torch = _torch()
    shape = tuple(src.shape) if shape is None else tuple(int(n) for n in shape)
    L = mgr_max_levels(shape) if int(nlevels) < 0 else int(nlevels)
    sub = tuple((n - 1) // 2 ** (L - level) + 1 for n in shape)
    if out is None:
        out = torch.empty(sub, dtype=src.dtype, device=src.device)
    _check(src, "src")
    _check(out, "out")
    need = int(np.prod(shape)) if not packed else int(class_offsets(shape, nlevels)[min(level, L) + 1])
    if src.numel() < need or tuple(out.shape) != sub or out.dtype != src.dtype:
        raise ValueError("src too small, or out of the wrong shape or dtype")
    cp, keep = _lib.coords_arg(shape, coords)
    stream = torch.cuda.current_stream(src.device).cuda_stream
    with torch.cuda.device(src.device):
        st = _lib.load().mgr_recompose_level(src.data_ptr(), out.data_ptr(), _dtype_code(src), len(shape),
                                             _lib.shape_arg(shape), cp, int(nlevels), int(level),
                                             1 if packed else 0, stream)
    del keep
    _lib.check(st)
    return out


def quant_bins(ndim, nlevels, tol):
    """Per-class bin widths (nlevels + 1 doubles) for a bound tol on the
    largest pointwise error of the recomposed field (mgr_quant_bins)."""
    import ctypes
    b = np.zeros(int(nlevels) + 1, dtype=np.float64)
    _lib.check(_lib.load().mgr_quant_bins(int(ndim), int(nlevels), float(tol),
                                          b.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return b


def _bins_arg(bins, L):
    import ctypes
    b = np.ascontiguousarray(np.asarray(bins, dtype=np.float64))
    if b.shape != (L + 1,):
        raise ValueError(f"one bin width per class: {L + 1} values")
    return b, b.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def quantize(y, bins, shape=None, nlevels=-1, packed=False, codes=None, count=True):
    """int32 codes of the classes of a refactored array y (in-place layout,
    or class-packed with packed=True and the field's shape).  Returns
    (codes, clamped) with clamped a one-element int64 GPU tensor holding the
    number of clamped codes (None with count=False)."""
    torch = _torch()
    _check(y, "y")
    shape = tuple(y.shape) if shape is None else tuple(int(n) for n in shape)
    L = mgr_max_levels(shape) if int(nlevels) < 0 else int(nlevels)
    if y.numel() != int(np.prod(shape)):
        raise ValueError("y does not hold prod(shape) elements")
    if codes is None:
        codes = torch.empty(tuple(y.shape), dtype=torch.int32, device=y.device)
    _check(codes, "codes")
    if codes.numel() != y.numel() or codes.dtype != torch.int32 or codes.device != y.device:
        raise ValueError("codes must be int32 with as many elements as y, on its device")
    b, bp = _bins_arg(bins, L)
    clamped = torch.empty(1, dtype=torch.int64, device=y.device) if count else None
    stream = torch.cuda.current_stream(y.device).cuda_stream
    with torch.cuda.device(y.device):
        st = _lib.load().mgr_quantize(y.data_ptr(), codes.data_ptr(), _dtype_code(y), len(shape),
                                      _lib.shape_arg(shape), int(nlevels), 1 if packed else 0, bp,
                                      clamped.data_ptr() if count else None, stream)
    del b
    _lib.check(st)
    return codes, clamped


def dequantize(codes, bins, dtype, shape=None, nlevels=-1, packed=False, out=None):
    """Dequantised classes (code * bin width, in `dtype`) from int32 codes."""
    torch = _torch()
    _check(codes, "codes")
    if codes.dtype != torch.int32:
        raise ValueError("codes must be int32")
    shape = tuple(codes.shape) if shape is None else tuple(int(n) for n in shape)
    L = mgr_max_levels(shape) if int(nlevels) < 0 else int(nlevels)
    if codes.numel() != int(np.prod(shape)):
        raise ValueError("codes does not hold prod(shape) elements")
    if out is None:
        out = torch.empty(tuple(codes.shape), dtype=dtype, device=codes.device)
    _check(out, "out")
    if out.numel() != codes.numel() or out.device != codes.device:
        raise ValueError("out must have as many elements as codes, on its device")
    b, bp = _bins_arg(bins, L)
    stream = torch.cuda.current_stream(codes.device).cuda_stream
    with torch.cuda.device(codes.device):
        st = _lib.load().mgr_dequantize(codes.data_ptr(), out.data_ptr(), _dtype_code(out), len(shape),
                                        _lib.shape_arg(shape), int(nlevels), 1 if packed else 0, bp, stream)
    del b
    _lib.check(st)
    return out


def mgr_bench_copy(src, dst):
    """Single-pass copy kernel (achievable-bandwidth calibration)."""
    _check(src, "src")
    _check(dst, "dst")
    n = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() < n:
        raise ValueError("dst too small")
    torch = _torch()
    stream = torch.cuda.current_stream(src.device).cuda_stream
    _lib.check(_lib.load().mgr_bench_copy(src.data_ptr(), dst.data_ptr(), n, stream))
    return dst


def mgr_set_tail_max_nodes(max_nodes):
    """Level steps with at most max_nodes nodes share one launch; returns
    the previous setting (0 disables)."""
    return _lib.load().mgr_set_tail_max_nodes(int(max_nodes))


def mgr_finalize():
    _lib.load().mgr_finalize()


def mgr_kernel_name(k):
    r = _lib.load().mgr_kernel_name(int(k))
    return None if r is None else r.decode()


def kernel_classes():
    out = {}
    k = 0
    while True:
        n = mgr_kernel_name(k)
        if n is None:
            return out
        out[n] = k
        k += 1


def mgr_timing_enable(kernel, level=-1):
    if isinstance(kernel, str):
        kernel = kernel_classes()[kernel]
    _lib.check(_lib.load().mgr_timing_enable(int(kernel), int(level)))


def mgr_timing_disable():
    _lib.check(_lib.load().mgr_timing_disable())


def mgr_timing_read():
    """(total milliseconds, launch count) of the timed kernel since last read."""
    import ctypes
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    _lib.check(_lib.load().mgr_timing_read(ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def decompose(x, coords=None, nlevels=-1, out=None):
    """Refactored representation of x (a new tensor unless out is given)."""
    if out is None:
        out = _torch().empty_like(x)
    return mgr_decompose(x, out, coords, nlevels)


def recompose(y, coords=None, nlevels=-1, out=None):
    if out is None:
        out = _torch().empty_like(y)
    return mgr_recompose(y, out, coords, nlevels)


def decompose_adjoint(g, coords=None, nlevels=-1, out=None):
    if out is None:
        out = _torch().empty_like(g)
    return mgr_decompose_adjoint(g, out, coords, nlevels)


def recompose_adjoint(g, coords=None, nlevels=-1, out=None):
    if out is None:
        out = _torch().empty_like(g)
    return mgr_recompose_adjoint(g, out, coords, nlevels)


def _make_autograd():
    torch = _torch()

    class Decompose(torch.autograd.Function):
        """y = D x with the hand-written adjoint kernel as backward:
        dL/dx = D^T dL/dy."""

        @staticmethod
        def forward(ctx, x, coords=None, nlevels=-1):
            ctx.coords = coords
            ctx.nlevels = nlevels
            return decompose(x.contiguous(), coords, nlevels)

        @staticmethod
        def backward(ctx, g):
            return decompose_adjoint(g.contiguous(), ctx.coords, ctx.nlevels), None, None

    class Recompose(torch.autograd.Function):
        """x = D^{-1} y with the recomposition's hand-written adjoint as
        backward: dL/dy = D^{-T} dL/dx."""

        @staticmethod
        def forward(ctx, y, coords=None, nlevels=-1):
            ctx.coords = coords
            ctx.nlevels = nlevels
            return recompose(y.contiguous(), coords, nlevels)

        @staticmethod
        def backward(ctx, g):
            return recompose_adjoint(g.contiguous(), ctx.coords, ctx.nlevels), None, None

    return {"Decompose": Decompose, "Recompose": Recompose}


class _LazyFunction:
    _classes = None

    def __init__(self, name):
        self._name = name

    def __getattr__(self, attr):
        if _LazyFunction._classes is None:
            _LazyFunction._classes = _make_autograd()
        return getattr(_LazyFunction._classes[self._name], attr)


Decompose = _LazyFunction("Decompose")
Recompose = _LazyFunction("Recompose")


def batch_queue_check(shapes, dtype_code=MGR_F32, nlevels=None, chunk=8, nthreads=8, poll_limit=0,
                      stall_item=-1, seed=0, nqueues=8):
    """Runs the persistent batch's scheduling protocol for these field shapes
    on host threads (mgr_batch_queue_check; no device needed), with nqueues
    queues.  Returns (items run, items started before their dependencies
    finished, error word, queue positions never taken)."""
    import ctypes
    shapes = [tuple(int(n) for n in s) for s in shapes]
    nf = len(shapes)
    nd = (ctypes.c_int * nf)(*[len(s) for s in shapes])
    shp = [_lib.shape_arg(s) for s in shapes]
    shp_p = (ctypes.POINTER(ctypes.c_int64) * nf)(*[ctypes.cast(a, ctypes.POINTER(ctypes.c_int64)) for a in shp])
    nl = None if nlevels is None else (ctypes.c_int * nf)(*[int(x) for x in nlevels])
    out = (ctypes.c_int64 * 4)()
    _lib.check(_lib.load().mgr_batch_queue_check(nf, nd, shp_p, nl, int(dtype_code), int(chunk), int(nqueues),
                                                 int(nthreads),
                                                 int(poll_limit), int(stall_item), int(seed), out))
    return tuple(int(v) for v in out)


class BatchPlan:
    """Plan for decomposing many independent fields together: one launch per
    wave of work items (``mgr_batch_plan_create`` / ``mgr_batch_decompose``).

    shapes: list of shapes; coords: None or a list (per field) of per-dim
    coordinate arrays or None; nlevels: None or a list of level counts.
    """

    def __init__(self, shapes, dtype=None, coords=None, nlevels=None):
        import ctypes
        torch = _torch()
        dtype = torch.float32 if dtype is None else dtype
        self.dtype = dtype
        self.shapes = [tuple(int(n) for n in s) for s in shapes]
        nf = len(self.shapes)
        lib = _lib.load()
        nd = (ctypes.c_int * nf)(*[len(s) for s in self.shapes])
        shp = [_lib.shape_arg(s) for s in self.shapes]
        shp_p = (ctypes.POINTER(ctypes.c_int64) * nf)(*[ctypes.cast(a, ctypes.POINTER(ctypes.c_int64)) for a in shp])
        keep = []
        cp = None
        if coords is not None:
            arr = (ctypes.POINTER(ctypes.POINTER(ctypes.c_double)) * nf)()
            for f, c in enumerate(coords):
                ptr, k = _lib.coords_arg(self.shapes[f], c)
                keep.append(k)
                arr[f] = ptr if ptr is not None else ctypes.POINTER(ctypes.POINTER(ctypes.c_double))()
            cp = arr
        nl = None if nlevels is None else (ctypes.c_int * nf)(*[int(x) for x in nlevels])
        h = ctypes.c_void_p()
        code = _dtype_code(torch.empty(0, dtype=dtype))
        st = lib.mgr_batch_plan_create(nf, nd, shp_p, cp, nl, code, ctypes.byref(h))
        del keep
        _lib.check(st)
        self._h = h

    def _ptrs(self, ts):
        import ctypes
        for t, s in zip(ts, self.shapes):
            _check(t, "field")
            if tuple(t.shape) != s or t.dtype != self.dtype:
                raise ValueError(f"field of shape {tuple(t.shape)} / {t.dtype}, plan has {s} / {self.dtype}")
        if len(ts) != len(self.shapes):
            raise ValueError("one tensor per field")
        return (ctypes.c_void_p * len(ts))(*[t.data_ptr() for t in ts])

    def decompose(self, srcs, dsts=None):
        """dsts[f] <- decomposition of srcs[f] (new tensors unless given)."""
        torch = _torch()
        if dsts is None:
            dsts = [torch.empty_like(x) for x in srcs]
        stream = torch.cuda.current_stream(srcs[0].device).cuda_stream
        with torch.cuda.device(srcs[0].device):
            _lib.check(_lib.load().mgr_batch_decompose(self._h, self._ptrs(srcs), self._ptrs(dsts), stream))
        return dsts

    def autotune(self, srcs, dsts, top_k=3):
        torch = _torch()
        stream = torch.cuda.current_stream(srcs[0].device).cuda_stream
        _lib.check(_lib.load().mgr_batch_autotune(self._h, self._ptrs(srcs), self._ptrs(dsts), stream, int(top_k)))
        return self.config()

    def config(self):
        """(chunk, launches per call, work items)."""
        import ctypes
        c, w, n = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_int64(0)
        _lib.check(_lib.load().mgr_batch_config(self._h, ctypes.byref(c), ctypes.byref(w), ctypes.byref(n)))
        return c.value, w.value, n.value

    def set_config(self, chunk):
        _lib.check(_lib.load().mgr_batch_set_config(self._h, int(chunk)))

    def tuning(self):
        """(persistent form in use, fitted model per form: {"waves": (a_ms,
        ms_per_byte, ms_per_item, ms_per_depth_plane), "persistent": (...)})
        after autotune."""
        import ctypes
        p = ctypes.c_int(0)
        m = (ctypes.c_double * 8)()
        _lib.check(_lib.load().mgr_batch_tuning(self._h, ctypes.byref(p), m))
        return bool(p.value), {"waves": tuple(m[0:4]), "persistent": tuple(m[4:8])}

    def set_mode(self, persistent, poll_limit=0):
        """persistent=True: one queue-driven launch for all items (see
        mgr_batch_set_mode); poll_limit bounds each dependency wait."""
        _lib.check(_lib.load().mgr_batch_set_mode(self._h, 1 if persistent else 0, int(poll_limit)))

    def tile(self):
        """True when the 3-D streaming items use the wide tile geometry."""
        import ctypes
        w = ctypes.c_int(0)
        _lib.check(_lib.load().mgr_batch_tile(self._h, ctypes.byref(w)))
        return bool(w.value)

    def set_tile(self, wide):
        """Narrow (False) or wide (True) tiles for the 3-D streaming items;
        rebuilds the work items."""
        _lib.check(_lib.load().mgr_batch_set_tile(self._h, 1 if wide else 0))

    def check(self):
        """Synchronises and raises MgrError if the last persistent run
        aborted."""
        _lib.check(_lib.load().mgr_batch_check(self._h))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().mgr_batch_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
