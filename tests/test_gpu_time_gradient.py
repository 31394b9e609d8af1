"""Node-height and epoch-boundary gradients (epoch_time_gradient) against the FP64 oracle:
every kernel path (4-state level kernels, 64-state, generic, matrix-core P stages with real
and complex eigensystems), dated tips, several categories, long epoch chains, and nodes
exactly on boundaries (one-sided derivatives)."""
import numpy as np
import pytest

from oracle import epoch_oracle as O
from paper_1309_3075_amd import _abi
from paper_1309_3075_amd import workloads as W
from paper_1309_3075_amd.likelihood import EpochLikelihood, from_problem
from tolerances import TOL_GRAD, assert_grad

pytestmark = pytest.mark.gpu


def _rand(seed, n, K, P, C, M, S, rev, th=0.2):
    rng = np.random.default_rng(seed)
    return W.random_problem(rng, n, K, P, n_categories=C, n_intervals=M, n_processes=S, reversible=rev,
                            tip_height_max=th, branch_rate_spread=0.25, missing_frac=0.03)


CASES = {
    "K4_C4": lambda: _rand(201, 24, 4, 500, 4, 4, 3, True),
    "K4_asym_C2": lambda: _rand(202, 15, 4, 300, 2, 3, 2, False),
    "K3_C3": lambda: _rand(203, 11, 3, 200, 3, 3, 2, False),
    "K20_C2": lambda: _rand(204, 13, 20, 120, 2, 3, 3, True),
    "K40_asym": lambda: _rand(205, 12, 40, 40, 1, 6, 4, False, 0.0),
    "K61_codon": lambda: W.make_config(3, n_tips=40, n_patterns=300),
    "C4_shape_160": lambda: W.make_config(4, n_tips=160),
}


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("name", list(CASES))
def test_time_gradient_against_oracle(name, precision):
    prob = CASES[name]()
    use_pi = prob.pi_process[0] is not None
    with from_problem(prob, precision, grad_time=True, use_pi=use_pi) as lik:
        lik.log_likelihood()
        dh, db = lik.time_gradient()
        # the branch-gradient pass it ran gives the usual branch gradient too
        g, _ = lik.gradient()
    want_h, want_b = O.time_gradient(prob)
    assert_grad(dh, want_h, TOL_GRAD[precision], "dlogL/dh")
    if len(want_b):
        assert_grad(db, want_b, TOL_GRAD[precision], "dlogL/db")
    ref_g, _ = O.gradient(prob, wrt=("branch",))
    assert_grad(g, ref_g, TOL_GRAD[precision], "dlogL/dl")


def test_time_gradient_at_ties():
    """A tip and an internal node exactly on boundaries: the library gives the oracle's upward
    one-sided derivatives (the oracle's are pinned by one-sided differences)."""
    Q0 = np.array([[-1.0, 0.6, 0.4], [0.3, -0.5, 0.2], [0.5, 0.5, -1.0]])
    Q1 = np.array([[-0.4, 0.1, 0.3], [1.2, -1.5, 0.3], [0.2, 0.9, -1.1]])
    parent = np.array([4, 4, 5, 6, 5, 6, -1], np.int32)
    height = np.array([0.0, 0.1, 0.25, 0.0, 0.6, 0.8, 1.0])
    tips = np.array([[0, 1, 2, 0, 1, 3], [1, 1, 0, 2, 2, 0], [2, 0, 1, 1, 3, 2], [0, 2, 2, 1, 0, 1]], np.int32)
    prob = W.Problem(name="ties", parent=parent, height=height,
                     branch_rate=np.array([1.1, 0.9, 1.0, 1.2, 0.8, 1.0, 1.0]),
                     boundaries=np.array([0.25, 0.6]), interval_process=np.array([0, 1, 0], np.int32),
                     Q=[Q0, Q1], pi_process=[None, None], pi_root=np.array([0.3, 0.3, 0.4]),
                     cat_rates=np.array([0.5, 1.5]), cat_weights=np.array([0.5, 0.5]), tips=tips,
                     weights=np.ones(6))
    want_h, want_b = O.time_gradient(prob)
    for precision in ("fp64", "fp32"):
        with from_problem(prob, precision, grad_time=True, use_pi=False) as lik:
            lik.log_likelihood()
            dh, db = lik.time_gradient()
        assert_grad(dh, want_h, TOL_GRAD[precision], f"{precision} dlogL/dh")
        assert_grad(db, want_b, TOL_GRAD[precision], f"{precision} dlogL/db")


def test_time_gradient_C2_tree_level_kernels():
    """The 512-taxon C2 tree and model with 3,000 patterns in FP32: the 4-state level kernels'
    branch adjoints feed the time gradient."""
    prob = W.make_config(2, n_patterns=3000)
    with from_problem(prob, "fp32", grad_time=True) as lik:
        logL, _, _, _ = lik.evaluate(branch=True)
        dh, db = lik.time_gradient()
    want_h, want_b = O.time_gradient(prob)
    assert_grad(dh, want_h, TOL_GRAD["fp32"], "dlogL/dh")
    assert_grad(db, want_b, TOL_GRAD["fp32"], "dlogL/db")


def test_time_gradient_call_rules():
    prob = _rand(206, 6, 4, 20, 1, 2, 2, True)
    with from_problem(prob, "fp64", grad_branch=True) as lik:
        lik.log_likelihood()
        with pytest.raises(_abi.EpochError) as e:
            lik.time_gradient()
        assert e.value.code == _abi.EPOCH_ERR_STATE
    with from_problem(prob, "fp64", grad_time=True) as lik:
        with pytest.raises(_abi.EpochError) as e:
            lik.time_gradient()
        assert e.value.code == _abi.EPOCH_ERR_STATE
        lik.log_likelihood()
        a = lik.time_gradient()
        b = lik.time_gradient()  # the branch adjoints are reused, the result is the same
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    with pytest.raises(_abi.EpochError) as e:
        EpochLikelihood(prob.n_tips, prob.n_patterns, 4, 1, 2, 2, "fp32", grad_time=True, hbm_budget_bytes=1 << 20)
    assert e.value.code == _abi.EPOCH_ERR_ARG
