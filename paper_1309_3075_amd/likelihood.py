"""Thin object wrapper over the C ABI, one method per entry point.

Argument marshalling only: validation and every computation happen inside
libepochlik.so.  The instance runs on torch's current HIP stream when torch
has a GPU, else on the default stream.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np

from . import _abi
from ._abi import _dp, _f64, _i32, _ip, check
from .eigen import eigensystem


def _current_stream():
    try:
        import torch
        if torch.cuda.is_available():
            return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:  # pragma: no cover - torch missing or no device
        pass
    return ctypes.c_void_p(None)


class EpochLikelihood:
    """One likelihood instance (tree size, patterns, states fixed at creation)."""

    def __init__(self, n_tips: int, n_patterns: int, n_states: int, n_categories: int = 1,
                 n_processes: int = 1, max_intervals: int = 1, precision: str = "fp64",
                 grad_branch: bool = False, grad_Q: bool = False, kernel: str = "auto",
                 stream=None, hbm_budget_bytes: int = 0, workspace=None, grad_time: bool = False):
        lib = _abi.load()
        cfg = _abi.EpochConfig()
        cfg.n_tips = n_tips
        cfg.n_patterns = n_patterns
        cfg.n_states = n_states
        cfg.n_categories = n_categories
        cfg.n_processes = n_processes
        cfg.max_intervals = max_intervals
        cfg.precision = {"fp32": _abi.EPOCH_FP32, "fp64": _abi.EPOCH_FP64}[precision]
        cfg.flags = (_abi.EPOCH_GRAD_BRANCH if grad_branch else 0) | (_abi.EPOCH_GRAD_Q if grad_Q else 0) | \
            (_abi.EPOCH_GRAD_TIME if grad_time else 0)
        cfg.kernel_path = {"auto": _abi.EPOCH_KERNEL_AUTO, "generic": _abi.EPOCH_KERNEL_GENERIC}[kernel]
        cfg.reserved = 0
        cfg.hbm_budget_bytes = int(hbm_budget_bytes)
        cfg.stream = stream if stream is not None else _current_stream()
        # caller-owned device memory for the pattern-sized buffers: a torch tensor (kept alive here)
        self._workspace = workspace
        if workspace is not None:
            cfg.workspace = workspace.data_ptr()
            cfg.workspace_bytes = workspace.numel() * workspace.element_size()
        self._cfg = cfg
        h = ctypes.c_void_p()
        check(lib.epoch_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self._lib = lib
        self.n_tips, self.n_patterns, self.n_states = n_tips, n_patterns, n_states
        self.n_categories, self.n_processes = n_categories, n_processes
        self.n_nodes = 2 * n_tips - 1
        self.n_boundaries = 0

    @staticmethod
    def workspace_bytes(n_tips: int, n_patterns: int, n_states: int, n_categories: int = 1,
                        precision: str = "fp64", grad_branch: bool = False, grad_Q: bool = False) -> int:
        """Bytes of the optional caller-owned workspace (epoch_workspace_bytes)."""
        cfg = _abi.EpochConfig()
        cfg.n_tips, cfg.n_patterns, cfg.n_states, cfg.n_categories = n_tips, n_patterns, n_states, n_categories
        cfg.n_processes, cfg.max_intervals = 1, 1
        cfg.precision = {"fp32": _abi.EPOCH_FP32, "fp64": _abi.EPOCH_FP64}[precision]
        cfg.flags = (_abi.EPOCH_GRAD_BRANCH if grad_branch else 0) | (_abi.EPOCH_GRAD_Q if grad_Q else 0)
        out = ctypes.c_int64(0)
        check(_abi.load().epoch_workspace_bytes(ctypes.byref(cfg), ctypes.byref(out)))
        return out.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.epoch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- data ---------------------------------------------------------------
    def set_tip_states(self, states):
        s = _i32(states)
        check(self._lib.epoch_set_tip_states(self._h, _ip(s)))

    def set_tip_ambiguities(self, sets):
        """Ambiguity sets: `sets` is [n_codes][K] 0/1 (or bit masks); tip code K + 1 + a then stands
        for set a.  The tip states must be set again afterwards."""
        arr = np.asarray(sets)
        if arr.ndim == 2:
            arr = np.array([sum(1 << j for j in range(arr.shape[1]) if row[j]) for row in arr], dtype=np.uint64)
        m = np.ascontiguousarray(arr, dtype=np.uint64)
        ptr = m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)) if len(m) else None
        check(self._lib.epoch_set_tip_ambiguities(self._h, int(len(m)), ptr))

    def set_pattern_weights(self, w):
        w = _f64(w)
        check(self._lib.epoch_set_pattern_weights(self._h, _dp(w)))

    def set_categories(self, rates, weights):
        r, w = _f64(rates), _f64(weights)
        check(self._lib.epoch_set_categories(self._h, _dp(r), _dp(w)))

    def set_root_frequencies(self, pi):
        p = _f64(pi)
        check(self._lib.epoch_set_root_frequencies(self._h, _dp(p)))

    def set_eigensystem(self, s: int, V, Vinv, lambda_re, lambda_im=None, Q=None) -> float:
        V, Vi, lr = _f64(V), _f64(Vinv), _f64(lambda_re)
        li = None if lambda_im is None else _f64(lambda_im)
        q = None if Q is None else _f64(Q)
        res = ctypes.c_double(float("nan"))
        check(self._lib.set_epoch_eigensystems(self._h, s, _dp(V), _dp(Vi), _dp(lr), _dp(li), _dp(q),
                                               ctypes.byref(res)))
        return res.value

    def set_rate_matrix(self, s: int, Q, pi=None, check_residual: bool = True) -> float:
        """Decompose Q on the host and hand the eigensystem to the library."""
        e = eigensystem(Q, pi)
        return self.set_eigensystem(s, e.V, e.Vinv, e.lambda_re,
                                    e.lambda_im if e.is_complex else None,
                                    Q if check_residual else None)

    def set_tree(self, parent, height, branch_rate=None, boundaries=(), interval_process=(0,)):
        par, h = _i32(parent), _f64(height)
        r = None if branch_rate is None else _f64(branch_rate)
        b = _f64(boundaries) if len(boundaries) else None
        phi = _i32(interval_process)
        check(self._lib.set_tree_epochs(self._h, _ip(par), _dp(h), _dp(r), len(phi), _dp(b), _ip(phi)))
        self.n_boundaries = len(phi) - 1

    def set_branch_rates(self, nodes, rates):
        """New rates for the branches above `nodes` (epoch_set_branch_rates): the next
        evaluation re-forms only those branches' matrices and their ancestors' partials."""
        n, r = _i32(nodes), _f64(rates)
        check(self._lib.epoch_set_branch_rates(self._h, int(n.shape[0]), _ip(n), _dp(r)))

    def kernel_path(self) -> str:
        """'generic', 'nucleotide' or 'matrix_core64' (epoch_get_kernel_path)."""
        v = ctypes.c_int32(-1)
        check(self._lib.epoch_get_kernel_path(self._h, ctypes.byref(v)))
        return {0: "generic", 1: "nucleotide", 2: "matrix_core64"}[v.value]

    def work_counts(self):
        """(transition matrices, internal-node partials) formed by the last evaluation."""
        out = np.zeros(2, dtype=np.int64)
        check(self._lib.epoch_get_work_counts(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
        return int(out[0]), int(out[1])

    # -- the path -----------------------------------------------------------
    def update_transition_matrices(self):
        check(self._lib.update_transition_matrices(self._h))

    def update_partials(self):
        check(self._lib.update_partials(self._h))

    def root_log_likelihood(self, site: bool = False):
        out = ctypes.c_double(0.0)
        s = np.zeros(self.n_patterns) if site else None
        check(self._lib.root_log_likelihood(self._h, ctypes.byref(out), _dp(s)))
        return (out.value, s) if site else out.value

    def gradient(self, branch: bool = True, Q: bool = False):
        db = np.zeros(self.n_nodes) if branch else None
        dq = np.zeros((self.n_processes, self.n_states, self.n_states)) if Q else None
        check(self._lib.log_likelihood_gradient(self._h, _dp(db), _dp(dq)))
        return db, dq

    def time_gradient(self):
        """(dlogL/dh for every node height [2N-1], dlogL/db for every boundary [M-1])
        (epoch_time_gradient; needs grad_time and a log-likelihood for the current state)."""
        dh = np.zeros(self.n_nodes)
        db = np.zeros(max(self.n_boundaries, 0))
        check(self._lib.epoch_time_gradient(self._h, _dp(dh), _dp(db) if len(db) else None))
        return dh, db

    def evaluate(self, branch: bool = False, Q: bool = False, site: bool = False):
        """One whole evaluation with one host synchronisation (epoch_evaluate):
        returns (logL, site logL or None, dlogL/dl or None, dlogL/dQ or None)."""
        out = ctypes.c_double(0.0)
        s = np.zeros(self.n_patterns) if site else None
        db = np.zeros(self.n_nodes) if branch else None
        dq = np.zeros((self.n_processes, self.n_states, self.n_states)) if Q else None
        what = _abi.EPOCH_EVAL_LOGL | (_abi.EPOCH_EVAL_GRAD_BRANCH if branch else 0) | \
            (_abi.EPOCH_EVAL_GRAD_Q if Q else 0)
        check(self._lib.epoch_evaluate(self._h, what, ctypes.byref(out), _dp(s), _dp(db), _dp(dq)))
        return out.value, s, db, dq

    def transition_matrices(self):
        out = np.zeros((self.n_nodes, self.n_categories, self.n_states, self.n_states))
        check(self._lib.epoch_get_transition_matrices(self._h, _dp(out)))
        return out

    def set_option(self, key: str, value: int):
        """Kernel-selection option (epoch_set_option): 'tree_walk', 'walk_recompute', 'walk_blocks',
        'walk_tiles', 'level_min_tiles', 'split_blocks', 'target_blocks', 'chain_split', 'incremental',
        'eigen_precision'."""
        k = {"tree_walk": _abi.EPOCH_OPT_TREE_WALK, "walk_recompute": _abi.EPOCH_OPT_WALK_RECOMPUTE,
             "walk_blocks": _abi.EPOCH_OPT_WALK_BLOCKS, "walk_tiles": _abi.EPOCH_OPT_WALK_TILES,
             "level_min_tiles": _abi.EPOCH_OPT_LEVEL_MIN_TILES,
             "split_blocks": _abi.EPOCH_OPT_SPLIT_BLOCKS, "target_blocks": _abi.EPOCH_OPT_TARGET_BLOCKS,
             "chain_split": _abi.EPOCH_OPT_CHAIN_SPLIT, "incremental": _abi.EPOCH_OPT_INCREMENTAL,
             "eigen_precision": _abi.EPOCH_OPT_EIGEN_PRECISION}[key]
        check(self._lib.epoch_set_option(self._h, k, int(value)))

    def set_timing(self, enable: bool = True):
        check(self._lib.epoch_set_timing(self._h, 1 if enable else 0))

    def timing(self):
        """{phase: (milliseconds, launch groups)} accumulated since set_timing(True)."""
        ms = np.zeros(len(_abi.PHASES))
        cnt = np.zeros(len(_abi.PHASES), dtype=np.int64)
        check(self._lib.epoch_get_timing(self._h, _dp(ms),
                                         cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
        return {k: (float(m), int(n)) for k, m, n in zip(_abi.PHASES, ms, cnt)}

    def log_likelihood(self, site: bool = False):
        self.update_transition_matrices()
        self.update_partials()
        return self.root_log_likelihood(site)


def from_problem(prob, precision: str = "fp64", grad_branch: bool = False, grad_Q: bool = False,
                 kernel: str = "auto", use_pi: bool = True, options: Optional[dict] = None,
                 hbm_budget_bytes: int = 0, workspace=None, grad_time: bool = False) -> EpochLikelihood:
    """Instance loaded with every input of a generated problem (options: see set_option)."""
    lik = EpochLikelihood(prob.n_tips, prob.n_patterns, prob.n_states, len(prob.cat_rates),
                          prob.n_processes, prob.n_intervals, precision, grad_branch, grad_Q, kernel,
                          hbm_budget_bytes=hbm_budget_bytes, workspace=workspace, grad_time=grad_time)
    for k, v in (options or {}).items():
        lik.set_option(k, v)
    if getattr(prob, "ambiguity", None) is not None:
        lik.set_tip_ambiguities(prob.ambiguity)
    lik.set_tip_states(prob.tips)
    lik.set_pattern_weights(prob.weights)
    lik.set_categories(prob.cat_rates, prob.cat_weights)
    lik.set_root_frequencies(prob.pi_root)
    for s, Q in enumerate(prob.Q):
        pi = prob.pi_process[s] if use_pi else None
        lik.set_rate_matrix(s, Q, pi)
    lik.set_tree(prob.parent, prob.height, prob.branch_rate, prob.boundaries, prob.interval_process)
    return lik


class EpochBatchEvaluator:
    """Many instances evaluated together in one replayed HIP graph (C ABI epoch_batch_*)."""

    def __init__(self, members, tune_cache: Optional[str] = None):
        self._lib = _abi.load()
        self.members = list(members)
        arr = (ctypes.c_void_p * len(self.members))(*[m._h.value for m in self.members])
        h = ctypes.c_void_p()
        check(self._lib.epoch_batch_create(arr, len(self.members),
                                           tune_cache.encode() if tune_cache else None, ctypes.byref(h)))
        self._h = h

    def evaluate(self, grad_branch: bool = True, grad_Q: bool = False) -> np.ndarray:
        what = _abi.EPOCH_EVAL_LOGL | (_abi.EPOCH_EVAL_GRAD_BRANCH if grad_branch else 0) | \
            (_abi.EPOCH_EVAL_GRAD_Q if grad_Q else 0)
        out = np.zeros(len(self.members))
        check(self._lib.epoch_batch_evaluate(self._h, what, _dp(out)))
        return out

    def gradients(self, i: int, branch: bool = True, Q: bool = False):
        m = self.members[i]
        db = np.zeros(m.n_nodes) if branch else None
        dq = np.zeros((m.n_processes, m.n_states, m.n_states)) if Q else None
        check(self._lib.epoch_batch_gradients(self._h, i, _dp(db), _dp(dq)))
        return db, dq

    def target_blocks(self) -> int:
        v = ctypes.c_int32(0)
        check(self._lib.epoch_batch_target_blocks(self._h, ctypes.byref(v)))
        return v.value

    def split_blocks(self) -> int:
        v = ctypes.c_int32(0)
        check(self._lib.epoch_batch_split_blocks(self._h, ctypes.byref(v)))
        return v.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.epoch_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
