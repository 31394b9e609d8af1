"""Host-side checks of the C ABI: exports, argument validation, the planner.

None of these launch a kernel; they run without a GPU.
"""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import epoch_oracle as O
from paper_1309_3075_amd import _abi
from paper_1309_3075_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "epochlik.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\**(\w+)\s*\(", text, flags=re.M)))


def test_library_exports_every_declared_symbol():
    lib = _abi.load()
    names = header_functions()
    assert len(names) >= 16
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(_abi.EXPORTED) == names
    assert b"epochlik" in lib.epoch_version()


def test_header_constants_match_the_binding():
    """Every EPOCH_* integer constant the header defines has the same value in the binding."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    defs = dict(re.findall(r"^#define\s+(EPOCH_\w+)\s+\(?(-?(?:0x[0-9a-fA-F]+|\d+))u?\)?", text, flags=re.M))
    assert {"EPOCH_WARN_UNDERFLOW", "EPOCH_ERR_NUMERIC", "EPOCH_OPT_INCREMENTAL"} <= set(defs)
    for name, val in defs.items():
        if hasattr(_abi, name):
            assert getattr(_abi, name) == int(val, 0), name
    assert _abi.EPOCH_WARN_UNDERFLOW > 0 > _abi.EPOCH_ERR_NUMERIC


def _cfg(**kw):
    c = _abi.EpochConfig()
    c.n_tips, c.n_patterns, c.n_states, c.n_categories = 4, 10, 4, 1
    c.n_processes, c.max_intervals, c.precision, c.flags = 1, 1, _abi.EPOCH_FP64, 0
    c.kernel_path, c.reserved, c.stream = 0, 0, None
    for k, v in kw.items():
        setattr(c, k, v)
    return c


@pytest.mark.parametrize("bad", [dict(n_tips=1), dict(n_patterns=0), dict(n_states=1), dict(n_states=65),
                                 dict(n_categories=0), dict(n_categories=9), dict(n_processes=0),
                                 dict(max_intervals=0), dict(precision=3), dict(flags=0x10),
                                 dict(kernel_path=7), dict(reserved=1), dict(hbm_budget_bytes=-1),
                                 dict(hbm_budget_bytes=1 << 20, flags=0x2),  # 4-state walk budget without dQ
                                 # budgets below one chunk of min(64, P) patterns: 64-state, generic paths
                                 dict(hbm_budget_bytes=7799, n_states=61, precision=_abi.EPOCH_FP32),
                                 dict(hbm_budget_bytes=7799, n_states=20),
                                 dict(hbm_budget_bytes=1079, kernel_path=1)])
def test_create_rejects_bad_config_before_touching_the_device(bad):
    lib = _abi.load()
    h = ctypes.c_void_p()
    rc = lib.epoch_create(ctypes.byref(_cfg(**bad)), ctypes.byref(h))
    assert rc == _abi.EPOCH_ERR_ARG
    assert lib.epoch_last_error().decode()
    assert not h.value


def test_null_arguments():
    lib = _abi.load()
    assert lib.epoch_create(None, None) == _abi.EPOCH_ERR_ARG
    assert lib.update_partials(None) == _abi.EPOCH_ERR_ARG
    assert lib.epoch_destroy(None) == _abi.EPOCH_OK


@pytest.mark.parametrize("seed,n_tips,n_int,tip_h", [(1, 5, 1, 0.0), (2, 9, 3, 0.3), (3, 30, 6, 0.5),
                                                    (4, 64, 48, 0.0)])
def test_planner_segments_match_oracle_segmentation(seed, n_tips, n_int, tip_h):
    rng = np.random.default_rng(seed)
    prob = W.random_problem(rng, n_tips, 3, 1, n_intervals=n_int, n_processes=min(n_int, 4),
                            tip_height_max=tip_h)
    off, proc, tim = _abi.plan_segments(prob.parent, prob.height, prob.boundaries,
                                        prob.interval_process, prob.n_processes)
    for v in range(prob.parent.shape[0] - 1):
        want = O.branch_segments(prob.height[prob.parent[v]], prob.height[v], prob.boundaries,
                                 prob.interval_process)
        got = list(zip(proc[off[v]:off[v + 1]], tim[off[v]:off[v + 1]]))
        assert [s for s, _ in got] == [s for s, _ in want]
        np.testing.assert_allclose([t for _, t in got], [t for _, t in want], rtol=1e-15, atol=1e-15)
        assert np.isclose(sum(t for _, t in got), prob.height[prob.parent[v]] - prob.height[v],
                          rtol=1e-13)
    root = prob.parent.shape[0] - 1
    assert off[root] == off[root + 1]


def test_planner_node_on_boundary_and_zero_length_branch():
    # tips 0,1,2; node 3 joins 0,1 at 0.5 (exactly a boundary); root 4 at 1.0
    parent = [3, 3, 4, 4, -1]
    height = [0.0, 0.5, 0.0, 0.5, 1.0]     # tip 1 sits at its parent's height: zero-length
    off, proc, tim = _abi.plan_segments(parent, height, [0.25, 0.5, 0.75], [0, 1, 2, 3], 4)
    assert off[1] == off[2]                  # zero-length branch: no segment
    assert list(proc[off[0]:off[1]]) == [1, 0]
    assert list(proc[off[3]:off[4]]) == [3, 2]  # 1.0 -> 0.5: [0.75, 1.0) then [0.5, 0.75)
    np.testing.assert_allclose(tim[off[3]:off[4]], [0.25, 0.25])


@pytest.mark.parametrize("parent,height,msg", [
    ([3, 3, 3, 4, -1], [0, 0, 0, 1, 2], "more than two children"),
    ([3, 3, 4, 4, 4], [0, 0, 0, 1, 2], "own parent"),
    ([3, 3, 4, 4, -1], [0, 0, 0, 1.5, 1.0], "younger"),
    ([3, 3, 4, 4, -1], [0, 0, np.nan, 1, 2], "not finite"),
    ([3, 3, 4, -1, -1], [0, 0, 0, 1, 2], "more than one root"),
    ([2, 3, 4, 4, -1], [0, 0, 0, 1, 2], "parent must be an internal node"),
])
def test_planner_rejects_bad_trees(parent, height, msg):
    with pytest.raises(_abi.EpochError) as ei:
        _abi.plan_segments(parent, height, [], [0], 1)
    assert ei.value.code == _abi.EPOCH_ERR_ARG
    assert msg in str(ei.value)


def test_planner_rejects_bad_epochs():
    parent, height = [3, 3, 4, 4, -1], [0, 0, 0, 1, 2]
    with pytest.raises(_abi.EpochError, match="ascending"):
        _abi.plan_segments(parent, height, [0.5, 0.5], [0, 0, 0], 1)
    with pytest.raises(_abi.EpochError, match="interval_process out of range"):
        _abi.plan_segments(parent, height, [0.5], [0, 2], 2)


def test_generator_invariants_and_determinism():
    for idx in (1, 2, 3):
        p = W.make_config(idx, n_tips=12, n_patterns=40)
        for Q, pi in zip(p.Q, p.pi_process):
            np.testing.assert_allclose(Q.sum(axis=1), 0.0, atol=1e-12)
            np.testing.assert_allclose(np.dot(pi, np.diag(Q)), -1.0, rtol=1e-12)
            # detailed balance
            np.testing.assert_allclose(pi[:, None] * Q, (pi[:, None] * Q).T, atol=1e-14)
        q = W.make_config(idx, n_tips=12, n_patterns=40)
        assert np.array_equal(p.tips, q.tips) and np.array_equal(p.height, q.height)
        assert p.tips.shape == (12, 40) and p.weights.shape == (40,)
        assert len(np.unique(p.tips.T, axis=0)) == 40
    c4 = W.make_config(4, n_tips=20)
    assert len(c4.Q) == 12 and c4.n_intervals == 48
    for Q in c4.Q:
        np.testing.assert_allclose(Q.sum(axis=1), 0.0, atol=1e-12)
        np.testing.assert_allclose(-np.trace(Q) / 40, 1.0, rtol=1e-12)
    rates, w = W.discrete_gamma(0.5, 4)
    np.testing.assert_allclose(np.dot(rates, w), 1.0, rtol=1e-12)
    assert np.all(np.diff(rates) > 0)
    assert len(W.sense_codons()[0]) == 61


def test_host_eigensystem_real_form():
    from paper_1309_3075_amd.eigen import eigensystem
    rng = np.random.default_rng(3)
    Q = W.sparse_asymmetric(12, 0.4, rng)
    e = eigensystem(Q)
    B = np.diag(e.lambda_re)
    j = 0
    while j < 12:
        if e.lambda_im[j] > 0:
            a, b = e.lambda_re[j], e.lambda_im[j]
            B[j:j + 2, j:j + 2] = [[a, b], [-b, a]]
            j += 2
        else:
            j += 1
    np.testing.assert_allclose(e.V @ B @ e.Vinv, Q, atol=1e-10)
    pi = rng.dirichlet(np.ones(4))
    Q2 = W.gtr(rng.dirichlet(np.ones(6)), pi)
    e2 = eigensystem(Q2, pi)
    np.testing.assert_allclose(e2.V @ np.diag(e2.lambda_re) @ e2.Vinv, Q2, atol=1e-13)


def test_workspace_bytes_covers_the_pattern_sized_buffers():
    lib = _abi.load()
    out = ctypes.c_int64(0)
    c = _cfg(n_tips=10, n_patterns=1000, n_states=4, n_categories=4, flags=_abi.EPOCH_GRAD_BRANCH)
    assert lib.epoch_workspace_bytes(ctypes.byref(c), ctypes.byref(out)) == _abi.EPOCH_OK
    N, P, C, R = 10, 1000, 4, 8
    need = N * P + 8 * P + R * P + 2 * (N - 1) * C * P * 4 * R + 4 * (N - 1) * P + 8 * P
    assert need <= out.value <= need + 7 * 256
    c.flags = 0
    small = ctypes.c_int64(0)
    assert lib.epoch_workspace_bytes(ctypes.byref(c), ctypes.byref(small)) == _abi.EPOCH_OK
    assert small.value < out.value  # no outside vectors without gradients
    assert lib.epoch_workspace_bytes(ctypes.byref(_cfg(n_states=65)), ctypes.byref(out)) == _abi.EPOCH_ERR_ARG


def test_workspace_too_small_or_misaligned_is_refused_before_the_device():
    lib = _abi.load()
    c = _cfg(n_tips=6, n_patterns=100)
    need = ctypes.c_int64(0)
    assert lib.epoch_workspace_bytes(ctypes.byref(c), ctypes.byref(need)) == _abi.EPOCH_OK
    h = ctypes.c_void_p()
    for ws, nbytes in [(1 << 20, need.value - 1), ((1 << 20) + 8, need.value), (1 << 20, need.value)]:
        c.workspace, c.workspace_bytes = ws, nbytes
        c.hbm_budget_bytes = 1 << 30 if nbytes == need.value and ws == 1 << 20 else 0
        assert lib.epoch_create(ctypes.byref(c), ctypes.byref(h)) == _abi.EPOCH_ERR_ARG
        assert not h.value
