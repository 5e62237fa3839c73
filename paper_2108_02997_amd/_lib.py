"""ctypes binding of libprpull.so: the C ABI of include/prpull.h under the same names.

Argument marshalling only: every step of the solve runs in the library's HIP kernels.
PyTorch supplies device memory (tensors) and the stream (its current HIP stream).
torch is imported before the library is opened so that both share torch's HIP runtime.
"""
from __future__ import annotations

import ctypes
import os
import re

import torch  # noqa: F401  (must precede loading libprpull.so: one HIP runtime per process)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libprpull.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "prpull.h")

PR_L1, PR_L2, PR_LINF = 1, 2, 3
PR_FP64, PR_MIXED, PR_FP32 = 0, 1, 2
PR_KERNEL_UPDATE_F64, PR_KERNEL_UPDATE_F32, PR_KERNEL_BATCH_F64, PR_KERNEL_BATCH_F32, PR_KERNEL_MULTI = 0, 1, 2, 3, 4
PR_KERNEL_SWEEP_FOLD = 5
PR_KERNEL_BATCH_F64_W1, PR_KERNEL_BATCH_F32_W1, PR_KERNEL_KINDS = 8, 14, 20
BATCH_ROW_WIDTHS = (1, 2, 4, 8, 12, 16)


def batch_kind(fp32: bool, width: int) -> int:
    """Stats kind of pr_pull_batch updates that ran on rows of `width` values."""
    return (PR_KERNEL_BATCH_F32_W1 if fp32 else PR_KERNEL_BATCH_F64_W1) + BATCH_ROW_WIDTHS.index(width)


MAX_COLS = 16
PR_OK, PR_NOT_CONVERGED, PR_EINVAL, PR_ENOMEM, PR_EDEVICE, PR_EGRAPH = 0, 1, -1, -2, -3, -4
STATUS_NAMES = {0: "PR_OK", 1: "PR_NOT_CONVERGED", -1: "PR_EINVAL", -2: "PR_ENOMEM", -3: "PR_EDEVICE",
                -4: "PR_EGRAPH"}


class pr_result(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32), ("fp32_iters", ctypes.c_int32),
                ("fp64_iters", ctypes.c_int32), ("final_err", ctypes.c_double * 3)]

    def as_dict(self):
        return dict(iterations=self.iterations, converged=bool(self.converged), fp32_iters=self.fp32_iters,
                    fp64_iters=self.fp64_iters, err=tuple(self.final_err))


class pr_problem(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("tau", ctypes.c_double), ("norm", ctypes.c_int32),
                ("max_iter", ctypes.c_int32)]


class pr_graph_problem(ctypes.Structure):
    _fields_ = [("in_offsets", ctypes.c_void_p), ("in_indices", ctypes.c_void_p), ("outdeg", ctypes.c_void_p),
                ("N", ctypes.c_int64), ("E", ctypes.c_int64), ("prep", ctypes.c_void_p), ("alpha", ctypes.c_double),
                ("tau", ctypes.c_double), ("norm", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("init", ctypes.c_void_p), ("ranks", ctypes.c_void_p), ("norm_trace", ctypes.c_void_p)]


class pr_tune_result(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("mid_deg", "grid", "tile", "rows", "mid_deg_batch",
                                              "grid_batch_factor", "tile_batch", "rows_batch", "candidates",
                                              "pad")] + \
               [(n, ctypes.c_double) for n in ("best_us", "default_us", "best_batch_us", "default_batch_us")] + \
               [(n, ctypes.c_int32) for n in ("pair_mid_deg", "seg_grid", "merge_xcd", "seg_candidates")] + \
               [(n, ctypes.c_double) for n in ("best_seg_us", "default_seg_us")]


class PrError(RuntimeError):
    def __init__(self, fn, status, msg):
        super().__init__("%s returned %s: %s" % (fn, STATUS_NAMES.get(status, status), msg))
        self.status = status


_vp, _i64, _i32, _dbl, _sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_size_t

SIGNATURES = {
    "pr_create": ([ctypes.POINTER(_vp), ctypes.c_int], ctypes.c_int),
    "pr_destroy": ([_vp], None),
    "pr_last_error": ([], ctypes.c_char_p),
    "pr_version": ([], ctypes.c_char_p),
    "pr_set_option": ([_vp, ctypes.c_char_p, _i64], ctypes.c_int),
    "pr_get_stats": ([_vp, _i32, ctypes.POINTER(_i64), ctypes.POINTER(_dbl)], ctypes.c_int),
    "pr_reset_stats": ([_vp], ctypes.c_int),
    "pr_prep_bytes": ([_i64, _i64], _sz),
    "pr_prepare": ([_vp, _vp, _vp, _i64, _i64, _vp, _sz], ctypes.c_int),
    "pr_validate_graph": ([_vp, _vp, _vp, _vp, _vp, _i64, _i64, _vp, _sz], ctypes.c_int),
    "pr_segment_count": ([_vp, _vp, _vp, _vp, _i64, _i64, _i32, _vp, _sz, ctypes.POINTER(_i64)], ctypes.c_int),
    "pr_segment_bytes": ([_vp, _i64, _i64, _i32, _i64], _sz),
    "pr_prepare_segmented": ([_vp, _vp, _vp, _vp, _i64, _i64, _i32, _i64, _vp, _sz], ctypes.c_int),
    "pr_relabel_workspace_bytes": ([_vp, _i64, _i64], _sz),
    "pr_relabel": ([_vp, _vp, _vp, _vp, _vp, _i64, _i64, _vp, _vp, _vp, _vp, _vp, _sz], ctypes.c_int),
    "pr_unpermute": ([_vp, _vp, _vp, _i64, _vp, _vp], ctypes.c_int),
    "pr_workspace_bytes": ([_i64, _i64, _i32, _i32], _sz),
    "pr_pull": ([_vp, _vp, _vp, _vp, _vp, _i64, _i64, _vp, _dbl, _dbl, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _sz,
                 ctypes.POINTER(pr_result)], ctypes.c_int),
    "pr_pull_snapshots": ([_vp, _vp, _vp, _vp, _vp, _i64, _i64, _vp, _dbl, _dbl, _i32, _i32, _i32, _vp, _vp, _vp,
                           _i32, _vp, _vp, _vp, _vp, _vp, _sz, ctypes.POINTER(pr_result)], ctypes.c_int),
    "pr_noalloc_max_bytes": ([], _sz),
    "pr_pull_noalloc": ([_vp, _vp, _vp, _vp, _vp, _i64, _i64, _dbl, _dbl, _i32, _i32, _i32, _vp, _vp, _vp,
                         ctypes.POINTER(pr_result)], ctypes.c_int),
    "pr_multi_workspace_bytes": ([_i32, ctypes.POINTER(pr_graph_problem)], _sz),
    "pr_pull_multi": ([_vp, _vp, _i32, ctypes.POINTER(pr_graph_problem), _vp, _sz, ctypes.POINTER(pr_result)],
                      ctypes.c_int),
    "pr_tune_workspace_bytes": ([_i64, _i64, _i32], _sz),
    "pr_autotune": ([_vp, _vp, _vp, _vp, _vp, _i64, _i64, _vp, _vp, _vp, _sz, ctypes.POINTER(pr_tune_result)],
                    ctypes.c_int),
    "pr_mlp_param_count": ([], ctypes.c_int),
    "pr_features": ([_vp, _vp, _vp, _vp, _vp, _i64, _i64, _vp, _vp, _dbl, _vp, _vp, _vp], ctypes.c_int),
    "pr_mlp_forward": ([_vp, _vp, _vp, _vp, _i64, _vp, _vp], ctypes.c_int),
    "pr_mlp_backward_workspace_bytes": ([_i64], _sz),
    "pr_mlp_backward": ([_vp, _vp, _vp, _vp, _vp, _vp, _vp, _i64, _vp, _vp, _sz, ctypes.POINTER(_dbl)], ctypes.c_int),
    "pr_adam_step": ([_vp, _vp, _vp, _vp, _vp, _vp, _i32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                      ctypes.c_float, _i32], ctypes.c_int),
    "pr_warm_start_vector": ([_vp, _vp, _vp, _vp, _i64, _vp, _vp, _sz], ctypes.c_int),
    "pr_l1_distance": ([_vp, _vp, _vp, _vp, _i64, _vp, _sz, ctypes.POINTER(_dbl)], ctypes.c_int),
    "pr_sweep_workspace_bytes": ([_i64, _i64, _i32], _sz),
    "pr_pull_sweep": ([_vp, _vp, _vp, _vp, _vp, _i64, _i64, _vp, _i32, ctypes.POINTER(pr_problem),
                       ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp, _sz, ctypes.POINTER(pr_result)], ctypes.c_int),
    "pr_batch_workspace_bytes": ([_i64, _i64, _i32, _i32, _i32], _sz),
    "pr_pull_batch": ([_vp, _vp, _vp, _vp, _vp, _i64, _i64, _vp, _i32, ctypes.POINTER(pr_problem), _i32,
                       ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp, _sz,
                       ctypes.POINTER(pr_result)], ctypes.c_int),
}

_lib = None


def header_functions(path: str = HEADER):
    """Names of the functions declared in include/prpull.h."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pr_[a-z0-9_]+)\s*\(", text)))


def load():
    """Open libprpull.so; raises if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libprpull.so is missing: build it with `python -m paper_2108_02997_amd.build` "
                               "(or __graft_entry__.build())")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


def last_error() -> str:
    return load().pr_last_error().decode()


def check(fn: str, status: int, allow_not_converged: bool = True) -> int:
    if status < 0 or (status == PR_NOT_CONVERGED and not allow_not_converged):
        raise PrError(fn, status, last_error())
    return status


def ptr(t) -> int | None:
    """Device address of a tensor (None for None)."""
    if t is None:
        return None
    return t.data_ptr()


def stream_handle(device=None) -> int:
    return torch.cuda.current_stream(device).cuda_stream
