"""ctypes binding of libepochlik.so: argument marshalling only.

Every step of the likelihood runs inside the HIP library; this module only
converts numpy arrays to pointers and error codes to exceptions.  If the
library is not built, importing the binding raises.
"""
from __future__ import annotations

import ctypes
import os
import warnings
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libepochlik.so")

EPOCH_OK = 0
EPOCH_ERR_ARG = -1
EPOCH_ERR_STATE = -2
EPOCH_ERR_OOM = -3
EPOCH_ERR_HIP = -4
EPOCH_ERR_NUMERIC = -5
EPOCH_WARN_EIGEN_RESIDUAL = 1
EPOCH_WARN_UNDERFLOW = 2
EPOCH_FP32 = 1
EPOCH_FP64 = 2
EPOCH_GRAD_BRANCH = 0x1
EPOCH_GRAD_Q = 0x2
EPOCH_GRAD_TIME = 0x4
EPOCH_KERNEL_AUTO = 0
EPOCH_KERNEL_GENERIC = 1

# Every symbol include/epochlik.h declares.
EXPORTED = [
    "epoch_last_error", "epoch_version", "epoch_create", "epoch_destroy", "epoch_set_tip_states",
    "epoch_set_pattern_weights", "epoch_set_categories", "epoch_set_root_frequencies",
    "set_epoch_eigensystems", "set_tree_epochs", "update_transition_matrices", "update_partials",
    "root_log_likelihood", "log_likelihood_gradient", "epoch_evaluate", "epoch_get_transition_matrices",
    "epoch_plan_segments", "epoch_set_timing", "epoch_get_timing", "epoch_bandwidth_probe",
    "epoch_batch_create", "epoch_batch_evaluate", "epoch_batch_gradients", "epoch_batch_target_blocks",
    "epoch_batch_destroy", "epoch_set_option", "epoch_plan_walk", "epoch_workspace_bytes",
    "epoch_eigen_residual_noalloc", "epoch_set_branch_rates", "epoch_get_work_counts", "epoch_time_gradient",
    "epoch_set_tip_ambiguities", "epoch_get_kernel_path", "epoch_batch_split_blocks",
]
EPOCH_EVAL_LOGL = 0x1
EPOCH_EVAL_GRAD_BRANCH = 0x2
EPOCH_EVAL_GRAD_Q = 0x4
PHASES = ["transition_matrices", "post_order", "root", "pre_order_dP", "grad_reduce", "grad_Q"]


class EpochConfig(ctypes.Structure):
    _fields_ = [
        ("n_tips", ctypes.c_int32),
        ("n_patterns", ctypes.c_int32),
        ("n_states", ctypes.c_int32),
        ("n_categories", ctypes.c_int32),
        ("n_processes", ctypes.c_int32),
        ("max_intervals", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("kernel_path", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("hbm_budget_bytes", ctypes.c_int64),
        ("stream", ctypes.c_void_p),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_int64),
    ]


class EpochError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"[{code}] {message}")
        self.code = code


_lib = None


def load() -> ctypes.CDLL:
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1309_3075_amd.build`")
    # torch ships its own HIP runtime with the same SONAME as the system one;
    # loading torch first makes the library bind to that single runtime, so
    # torch's streams and device memory are valid inside the library.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i32, u32, dbl = ctypes.c_int32, ctypes.c_uint32, ctypes.c_double
    ip, dp = ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)
    sig = {
        "epoch_last_error": (ctypes.c_char_p, []),
        "epoch_version": (ctypes.c_char_p, []),
        "epoch_create": (i32, [ctypes.POINTER(EpochConfig), ctypes.POINTER(P)]),
        "epoch_destroy": (i32, [P]),
        "epoch_set_tip_states": (i32, [P, ip]),
        "epoch_set_pattern_weights": (i32, [P, dp]),
        "epoch_set_categories": (i32, [P, dp, dp]),
        "epoch_set_root_frequencies": (i32, [P, dp]),
        "set_epoch_eigensystems": (i32, [P, i32, dp, dp, dp, dp, dp, dp]),
        "set_tree_epochs": (i32, [P, ip, dp, dp, i32, dp, ip]),
        "update_transition_matrices": (i32, [P]),
        "update_partials": (i32, [P]),
        "root_log_likelihood": (i32, [P, dp, dp]),
        "log_likelihood_gradient": (i32, [P, dp, dp]),
        "epoch_evaluate": (i32, [P, u32, dp, dp, dp, dp]),
        "epoch_get_transition_matrices": (i32, [P, dp]),
        "epoch_plan_segments": (i32, [i32, ip, dp, i32, dp, ip, i32, i32, ip, ip, dp, ip]),
        "epoch_set_timing": (i32, [P, i32]),
        "epoch_bandwidth_probe": (i32, [ctypes.c_int64, i32, i32, dp]),
        "epoch_batch_create": (i32, [ctypes.POINTER(P), i32, ctypes.c_char_p, ctypes.POINTER(P)]),
        "epoch_batch_evaluate": (i32, [P, u32, dp]),
        "epoch_batch_gradients": (i32, [P, i32, dp, dp]),
        "epoch_batch_target_blocks": (i32, [P, ctypes.POINTER(i32)]),
        "epoch_batch_destroy": (i32, [P]),
        "epoch_get_timing": (i32, [P, dp, ctypes.POINTER(ctypes.c_int64)]),
        "epoch_set_option": (i32, [P, i32, ctypes.c_int64]),
        "epoch_workspace_bytes": (i32, [ctypes.POINTER(EpochConfig), ctypes.POINTER(ctypes.c_int64)]),
        "epoch_plan_walk": (i32, [i32, ip, dp, i32, i32, ip, ip]),
        "epoch_eigen_residual_noalloc": (i32, [i32, i32, P, P, P, P, P, P, P]),
        "epoch_set_branch_rates": (i32, [P, i32, ip, dp]),
        "epoch_get_work_counts": (i32, [P, ctypes.POINTER(ctypes.c_int64)]),
        "epoch_time_gradient": (i32, [P, dp, dp]),
        "epoch_set_tip_ambiguities": (i32, [P, i32, ctypes.POINTER(ctypes.c_uint64)]),
        "epoch_get_kernel_path": (i32, [P, ctypes.POINTER(i32)]),
        "epoch_batch_split_blocks": (i32, [P, ctypes.POINTER(i32)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _dp(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ip(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != tuple(shape):
        a = a.reshape(shape)
    return a


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


class EpochUnderflowWarning(RuntimeWarning):
    """A pattern's likelihood is zero in the working precision: logL is -inf and the state has no gradient."""


def check(code: int, allow_warning: bool = True) -> int:
    if code == EPOCH_WARN_UNDERFLOW and allow_warning:
        warnings.warn(EpochUnderflowWarning(load().epoch_last_error().decode()), stacklevel=3)
        return code
    if code == EPOCH_OK or (allow_warning and code > 0):
        return code
    msg = load().epoch_last_error().decode()
    raise EpochError(code, msg)


def last_error() -> str:
    return load().epoch_last_error().decode()


def plan_segments(parent, height, boundaries, interval_process, n_processes):
    """Host planner segmentation (no GPU needed): (offsets[2N], process[], time[])."""
    lib = load()
    parent = _i32(parent)
    height = _f64(height)
    n_nodes = parent.shape[0]
    n_tips = (n_nodes + 1) // 2
    b = _f64(boundaries) if len(boundaries) else None
    phi = _i32(interval_process)
    off = np.zeros(n_nodes + 1, np.int32)
    nseg = ctypes.c_int32(0)
    cap = n_nodes * (len(phi) + 1)
    proc = np.zeros(cap, np.int32)
    tim = np.zeros(cap, np.float64)
    check(lib.epoch_plan_segments(n_tips, _ip(parent), _dp(height), len(phi), _dp(b), _ip(phi),
                                  n_processes, cap, _ip(off), _ip(proc), _dp(tim), ctypes.byref(nseg)))
    n = nseg.value
    return off, proc[:n].copy(), tim[:n].copy()


EPOCH_OPT_TREE_WALK = 1
EPOCH_OPT_WALK_RECOMPUTE = 2
EPOCH_OPT_WALK_BLOCKS = 3
EPOCH_OPT_WALK_TILES = 4
EPOCH_OPT_LEVEL_MIN_TILES = 5
EPOCH_OPT_SPLIT_BLOCKS = 6
EPOCH_OPT_TARGET_BLOCKS = 7
EPOCH_OPT_CHAIN_SPLIT = 8
EPOCH_OPT_INCREMENTAL = 9
EPOCH_OPT_EIGEN_PRECISION = 10


def plan_walk(parent, height, recompute_tips: int = 2):
    """Host planner (no GPU needed): the 4-state tree-walk programs.
    Returns (post ops [n,4], pre ops [m,4], post stack slots, pre stack slots)."""
    lib = load()
    parent = _i32(parent)
    height = _f64(height)
    n_nodes = parent.shape[0]
    n_tips = (n_nodes + 1) // 2
    counts = np.zeros(4, np.int32)
    cap = 8 * n_nodes + 16
    ops = np.zeros((cap, 4), np.int32)
    check(lib.epoch_plan_walk(n_tips, _ip(parent), _dp(height), int(recompute_tips), cap, _ip(ops), _ip(counts)))
    n_post, n_pre = int(counts[0]), int(counts[1])
    return ops[:n_post].copy(), ops[n_post:n_post + n_pre].copy(), int(counts[2]), int(counts[3])


def bandwidth_probe(nbytes: int = 1 << 31, kind: str = "copy", iters: int = 20) -> float:
    """Measured GB/s of a plain copy / read / write stream on the current device."""
    lib = load()
    out = ctypes.c_double(0.0)
    check(lib.epoch_bandwidth_probe(int(nbytes), {"copy": 0, "read": 1, "write": 2}[kind], iters,
                                    ctypes.byref(out)))
    return out.value
