"""ctypes loader for libttsparse.so (the HIP library).  Argument marshalling only.

The library is built in-tree by ``paper_1908_02721_amd.build``.  Importing this
module never builds or falls back: a missing library raises ``ImportError``.
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch  # noqa: F401  -- load torch's HIP runtime first so the library shares it

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libttsparse.so")

STATUS = {
    0: "TT_OK", 1: "TT_ERR_ARG", 2: "TT_ERR_INDEX", 3: "TT_ERR_DUPLICATE", 4: "TT_ERR_NONFINITE",
    5: "TT_ERR_EMPTY", 6: "TT_ERR_TOO_LARGE", 7: "TT_ERR_NOMEM", 8: "TT_ERR_DEVICE",
}
PRECISION = {"fp64": 0, "fp32": 1, "bf16": 2}
DTYPE_F64, DTYPE_F32 = 0, 1
NUM_STAGES = 6
STAGES = ("ingest", "sort", "sparse_levels", "qr_sweep", "svd_sweep", "total")

_lock = threading.Lock()
_lib = None


class TTError(RuntimeError):
    """A libttsparse call returned a non-OK status."""

    def __init__(self, code: int, msg: str):
        self.code = code
        self.status = STATUS.get(code, f"status {code}")
        super().__init__(f"{self.status}: {msg}")


class tt_options(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int32),
        ("max_rank", ctypes.c_int32),
        ("keep_intermediates", ctypes.c_int32),
        ("sparse_only", ctypes.c_int32),
        ("device_mem_budget", ctypes.c_uint64),
        ("alloc", ctypes.c_void_p),
        ("free", ctypes.c_void_p),
        ("alloc_ctx", ctypes.c_void_p),
        ("dynamic_delta", ctypes.c_int32),
        ("key_bits", ctypes.c_int32),
    ]


EXPORTS = (
    "tt_options_default", "tt_sparse_decompose", "tt_get_ranks", "tt_get_core", "tt_get_info",
    "tt_get_sparse_ranks", "tt_get_sigma", "tt_get_bond_delta", "tt_get_times", "tt_matrix_to_tensor",
    "tt_fasttt_decompose", "tt_get_fasttt_info", "tt_sparse_gram_slice", "tt_get_slice_bond1", "tt_get_slice_x2",
    "tt_get_slice_gram", "tt_fasttt_select_p", "tt_get_level", "tt_get_level_sizes", "tt_cache_trim", "tt_free",
    "tt_eval_entries", "tt_eval_entries_backward", "tt_eval_entries_noalloc", "tt_eval_plan_create", "tt_eval_plan_forward",
    "tt_eval_plan_backward", "tt_eval_plan_free", "tt_status_string", "tt_last_error",
    "tt_kernel_timer_start", "tt_kernel_timer_read",
)


def load():
    """Load and type the library (once).  Raises ImportError when it is missing."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1908_02721_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        i32, i64, f64, vp, u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p, ctypes.c_uint64
        L.tt_options_default.argtypes = [P(tt_options)]
        L.tt_options_default.restype = None
        L.tt_sparse_decompose.argtypes = [i32, P(i64), i64, vp, vp, f64, P(tt_options), vp, P(vp)]
        L.tt_sparse_decompose.restype = ctypes.c_int
        L.tt_get_ranks.argtypes = [vp, P(i64)]
        L.tt_get_ranks.restype = ctypes.c_int
        L.tt_get_core.argtypes = [vp, i32, P(vp), P(i32)]
        L.tt_get_core.restype = ctypes.c_int
        L.tt_get_info.argtypes = [vp, P(i64), P(f64), P(f64)]
        L.tt_get_info.restype = ctypes.c_int
        L.tt_get_sparse_ranks.argtypes = [vp, P(i64), P(i64)]
        L.tt_get_sparse_ranks.restype = ctypes.c_int
        L.tt_get_sigma.argtypes = [vp, i32, P(i64), P(P(f64)), P(f64)]
        L.tt_get_sigma.restype = ctypes.c_int
        L.tt_get_bond_delta.argtypes = [vp, i32, P(f64)]
        L.tt_get_bond_delta.restype = ctypes.c_int
        L.tt_matrix_to_tensor.argtypes = [i32, P(i64), P(i64), i64, vp, vp, vp, vp]
        L.tt_matrix_to_tensor.restype = ctypes.c_int
        L.tt_fasttt_decompose.argtypes = [i32, P(i64), i64, vp, vp, f64, i32, P(tt_options), vp, P(vp)]
        L.tt_fasttt_decompose.restype = ctypes.c_int
        L.tt_sparse_gram_slice.argtypes = [i32, P(i64), i64, vp, vp, P(tt_options), vp, P(vp)]
        L.tt_sparse_gram_slice.restype = ctypes.c_int
        L.tt_get_slice_bond1.argtypes = [vp, P(i64), P(vp), P(vp), P(P(f64))]
        L.tt_get_slice_bond1.restype = ctypes.c_int
        L.tt_get_slice_x2.argtypes = [vp, P(i64), P(vp), P(vp), P(vp), P(i32)]
        L.tt_get_slice_x2.restype = ctypes.c_int
        L.tt_get_slice_gram.argtypes = [vp, P(vp), P(f64), P(i64), P(f64), P(f64)]
        L.tt_get_slice_gram.restype = ctypes.c_int
        L.tt_get_fasttt_info.argtypes = [vp, P(i32), P(i64)]
        L.tt_get_fasttt_info.restype = ctypes.c_int
        L.tt_fasttt_select_p.argtypes = [i32, P(i64), i64, vp, vp, P(f64), P(i32), vp]
        L.tt_fasttt_select_p.restype = ctypes.c_int
        L.tt_get_times.argtypes = [vp, P(f64)]
        L.tt_get_times.restype = ctypes.c_int
        L.tt_get_level.argtypes = [vp, i32, P(i64), P(i64), P(vp), P(vp), P(vp), P(vp), P(vp), P(vp)]
        L.tt_get_level.restype = ctypes.c_int
        L.tt_cache_trim.argtypes = [P(u64)]
        L.tt_cache_trim.restype = ctypes.c_int
        L.tt_get_level_sizes.argtypes = [vp, i32, P(i64)]
        L.tt_get_level_sizes.restype = ctypes.c_int
        L.tt_free.argtypes = [vp]
        L.tt_free.restype = None
        L.tt_eval_entries.argtypes = [i32, P(i64), P(i64), P(vp), i32, i64, vp, vp, vp]
        L.tt_eval_entries.restype = ctypes.c_int
        L.tt_eval_entries_noalloc.argtypes = [i32, P(i64), P(i64), P(vp), i32, i64, vp, vp, vp]
        L.tt_eval_entries_noalloc.restype = ctypes.c_int
        L.tt_eval_entries_backward.argtypes = [i32, P(i64), P(i64), P(vp), i32, i64, vp, vp, P(vp), vp]
        L.tt_eval_entries_backward.restype = ctypes.c_int
        L.tt_eval_plan_create.argtypes = [i32, P(i64), i64, vp, vp, P(vp)]
        L.tt_eval_plan_create.restype = ctypes.c_int
        L.tt_eval_plan_forward.argtypes = [vp, P(i64), P(vp), i32, vp, i32, vp]
        L.tt_eval_plan_forward.restype = ctypes.c_int
        L.tt_eval_plan_backward.argtypes = [vp, P(i64), P(vp), i32, vp, P(vp), i32, vp]
        L.tt_eval_plan_backward.restype = ctypes.c_int
        L.tt_eval_plan_free.argtypes = [vp]
        L.tt_eval_plan_free.restype = None
        L.tt_status_string.argtypes = [ctypes.c_int]
        L.tt_status_string.restype = ctypes.c_char_p
        L.tt_last_error.argtypes = []
        L.tt_last_error.restype = ctypes.c_char_p
        L.tt_kernel_timer_start.argtypes = [ctypes.c_char_p]
        L.tt_kernel_timer_start.restype = ctypes.c_int
        L.tt_kernel_timer_read.argtypes = [P(f64), P(i64), P(f64), P(f64)]
        L.tt_kernel_timer_read.restype = ctypes.c_int
        _ = u64
        _lib = L
        return L


def check(code: int):
    if code != 0:
        msg = load().tt_last_error().decode(errors="replace")
        raise TTError(code, msg)


def kernel_timer_start(family):
    """Time every launch of one kernel family from now on (None stops)."""
    check(load().tt_kernel_timer_start(family.encode() if family else None))


def kernel_timer_read():
    """(total_ms, launches, algorithmic_bytes, algorithmic_flops) since the last start."""
    ms, n, b, f = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
    check(load().tt_kernel_timer_read(ctypes.byref(ms), ctypes.byref(n), ctypes.byref(b), ctypes.byref(f)))
    return ms.value, n.value, b.value, f.value
