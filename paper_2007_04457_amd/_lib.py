"""ctypes binding of libmgr (include/mgr.h): argument marshalling only.

Every numerical step runs in the library's HIP kernels; this module passes
device pointers, shapes, host coordinates and the current HIP stream.  There
is no CPU fallback: if libmgr.so is missing or cannot load, every call
raises.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmgr.so")

MGR_F32, MGR_F64 = 0, 1

_lib = None


class MgrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(msg)
        self.status = status


def load():
    """Loads libmgr.so (built by paper_2007_04457_amd/build.py)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise MgrError(-1, f"{LIB_PATH} is not built; run paper_2007_04457_amd/build.py "
                           "or __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    i64p = ctypes.POINTER(ctypes.c_int64)
    dpp = ctypes.POINTER(ctypes.POINTER(ctypes.c_double))
    vp = ctypes.c_void_p
    for name in ("mgr_decompose", "mgr_recompose", "mgr_decompose_adjoint", "mgr_recompose_adjoint",
                 "mgr_decompose_noalloc"):
        fn = getattr(lib, name)
        fn.argtypes = [vp, vp, ctypes.c_int, ctypes.c_int, i64p, dpp, ctypes.c_int, vp]
        fn.restype = ctypes.c_int
    lib.mgr_max_levels.argtypes = [ctypes.c_int, i64p]
    lib.mgr_max_levels.restype = ctypes.c_int
    lib.mgr_prepare.argtypes = [ctypes.c_int, ctypes.c_int, i64p, dpp, ctypes.c_int]
    lib.mgr_prepare.restype = ctypes.c_int
    lib.mgr_class_map.argtypes = [ctypes.c_int, i64p, ctypes.c_int, ctypes.POINTER(ctypes.c_uint8)]
    lib.mgr_class_map.restype = ctypes.c_int
    lib.mgr_class_offsets.argtypes = [ctypes.c_int, i64p, ctypes.c_int, i64p]
    lib.mgr_class_offsets.restype = ctypes.c_int
    for name in ("mgr_pack_classes", "mgr_unpack_classes"):
        fn = getattr(lib, name)
        fn.argtypes = [vp, vp, ctypes.c_int, ctypes.c_int, i64p, ctypes.c_int, vp]
        fn.restype = ctypes.c_int
    lib.mgr_recompose_level.argtypes = [vp, vp, ctypes.c_int, ctypes.c_int, i64p, dpp, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_int, vp]
    lib.mgr_recompose_level.restype = ctypes.c_int
    lib.mgr_quant_bins.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.POINTER(ctypes.c_double)]
    lib.mgr_quant_bins.restype = ctypes.c_int
    dp = ctypes.POINTER(ctypes.c_double)
    lib.mgr_quantize.argtypes = [vp, vp, ctypes.c_int, ctypes.c_int, i64p, ctypes.c_int, ctypes.c_int, dp, vp, vp]
    lib.mgr_quantize.restype = ctypes.c_int
    lib.mgr_dequantize.argtypes = [vp, vp, ctypes.c_int, ctypes.c_int, i64p, ctypes.c_int, ctypes.c_int, dp, vp]
    lib.mgr_dequantize.restype = ctypes.c_int
    lib.mgr_status_string.argtypes = [ctypes.c_int]
    lib.mgr_status_string.restype = ctypes.c_char_p
    lib.mgr_last_error.argtypes = []
    lib.mgr_last_error.restype = ctypes.c_char_p
    lib.mgr_finalize.argtypes = []
    lib.mgr_finalize.restype = None
    lib.mgr_set_tail_max_nodes.argtypes = [ctypes.c_int64]
    lib.mgr_set_tail_max_nodes.restype = ctypes.c_int64
    lib.mgr_bench_copy.argtypes = [vp, vp, ctypes.c_size_t, vp]
    lib.mgr_bench_copy.restype = ctypes.c_int
    lib.mgr_timing_enable.argtypes = [ctypes.c_int, ctypes.c_int]
    lib.mgr_timing_enable.restype = ctypes.c_int
    lib.mgr_timing_disable.argtypes = []
    lib.mgr_timing_disable.restype = ctypes.c_int
    lib.mgr_timing_read.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    lib.mgr_timing_read.restype = ctypes.c_int
    lib.mgr_kernel_name.argtypes = [ctypes.c_int]
    lib.mgr_kernel_name.restype = ctypes.c_char_p
    i32p = ctypes.POINTER(ctypes.c_int)
    lib.mgr_batch_plan_create.argtypes = [ctypes.c_int, i32p, ctypes.POINTER(i64p),
                                          ctypes.POINTER(dpp), i32p, ctypes.c_int,
                                          ctypes.POINTER(vp)]
    lib.mgr_batch_plan_create.restype = ctypes.c_int
    vpp = ctypes.POINTER(vp)
    lib.mgr_batch_decompose.argtypes = [vp, vpp, vpp, vp]
    lib.mgr_batch_decompose.restype = ctypes.c_int
    lib.mgr_batch_autotune.argtypes = [vp, vpp, vpp, vp, ctypes.c_int]
    lib.mgr_batch_autotune.restype = ctypes.c_int
    lib.mgr_batch_config.argtypes = [vp, i32p, i32p, ctypes.POINTER(ctypes.c_int64)]
    lib.mgr_batch_config.restype = ctypes.c_int
    lib.mgr_batch_set_config.argtypes = [vp, ctypes.c_int]
    lib.mgr_batch_set_config.restype = ctypes.c_int
    lib.mgr_batch_tuning.argtypes = [vp, i32p, ctypes.POINTER(ctypes.c_double)]
    lib.mgr_batch_tuning.restype = ctypes.c_int
    lib.mgr_batch_set_mode.argtypes = [vp, ctypes.c_int, ctypes.c_uint]
    lib.mgr_batch_set_mode.restype = ctypes.c_int
    lib.mgr_batch_tile.argtypes = [vp, i32p]
    lib.mgr_batch_tile.restype = ctypes.c_int
    lib.mgr_batch_set_tile.argtypes = [vp, ctypes.c_int]
    lib.mgr_batch_set_tile.restype = ctypes.c_int
    lib.mgr_batch_check.argtypes = [vp]
    lib.mgr_batch_check.restype = ctypes.c_int
    lib.mgr_batch_queue_check.argtypes = [ctypes.c_int, i32p, ctypes.POINTER(i64p), i32p, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_int, ctypes.c_int, ctypes.c_uint, ctypes.c_int, ctypes.c_uint64, i64p]
    lib.mgr_batch_queue_check.restype = ctypes.c_int
    lib.mgr_batch_plan_destroy.argtypes = [vp]
    lib.mgr_batch_plan_destroy.restype = None
    _lib = lib
    return lib


def check(status):
    if status != 0:
        lib = load()
        detail = lib.mgr_last_error().decode()
        raise MgrError(status, f"{lib.mgr_status_string(status).decode()}: {detail}")


def shape_arg(shape):
    return (ctypes.c_int64 * len(shape))(*[int(s) for s in shape])


def coords_arg(shape, coords):
    """Host double** for coords (None entries = uniform), plus keep-alive."""
    if coords is None:
        return None, []
    if len(coords) != len(shape):
        raise ValueError("coords needs one entry per dimension")
    ptrs = (ctypes.POINTER(ctypes.c_double) * len(shape))()
    keep = []
    for d, c in enumerate(coords):
        if c is None:
            ptrs[d] = ctypes.POINTER(ctypes.c_double)()
            continue
        a = np.ascontiguousarray(np.asarray(c, dtype=np.float64))
        if a.shape != (int(shape[d]),):
            raise ValueError(f"coords[{d}] must have length {shape[d]}")
        keep.append(a)
        ptrs[d] = a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return ctypes.cast(ptrs, ctypes.POINTER(ctypes.POINTER(ctypes.c_double))), keep
