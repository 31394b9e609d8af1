"""A pattern whose likelihood leaves the working precision's range (EPOCH_WARN_UNDERFLOW).

Partials are rescaled per pattern by a power of two shared by the rate categories. On a tree
whose root joins a subtree where one pattern is constant (the slow category dominates there by
about 4^120) and a subtree where the same pattern varies at every tip (the fast category dominates
by far more), each category is flushed to zero in the other subtree in FP32, so that pattern's
likelihood is zero at the root: FP32 returns logL = -inf with the warning, while FP64, whose range
holds both ratios, matches the oracle."""
import warnings

import numpy as np
import pytest

from oracle import epoch_oracle as O
from paper_1309_3075_amd import _abi
from paper_1309_3075_amd import workloads as W
from paper_1309_3075_amd.likelihood import EpochBatchEvaluator, from_problem
from tolerances import TOL_LOGL, rel

pytestmark = pytest.mark.gpu


def _ladder(tips, h_lo, h_hi, parent, height, next_id):
    """Caterpillar over `tips` with internal heights evenly from h_lo to h_hi; returns its root."""
    node = tips[0]
    hs = np.linspace(h_lo, h_hi, len(tips) - 1)
    for t, h in zip(tips[1:], hs):
        parent[node] = parent[t] = next_id[0]
        height[next_id[0]] = h
        node = next_id[0]
        next_id[0] += 1
    return node


def _two_subtree_problem(n_a=120, n_b=40, seed=5):
    N = n_a + n_b
    parent = np.full(2 * N - 1, -1, np.int32)
    height = np.zeros(2 * N - 1)
    nxt = [N]
    ra = _ladder(list(range(n_a)), 0.5, 0.6, parent, height, nxt)
    rb = _ladder(list(range(n_a, N)), 0.5, 0.6, parent, height, nxt)
    root = nxt[0]
    parent[ra] = parent[rb] = root
    height[root] = 1.0
    rng = np.random.default_rng(seed)
    tips = np.zeros((N, 3), np.int32)
    tips[:n_a, 0] = 0                                   # constant in subtree A ...
    tips[n_a:, 0] = np.arange(n_b) % 4                  # ... varying at every tip of subtree B
    tips[:, 1] = rng.integers(0, 4, N)                  # ordinary patterns
    tips[:, 2] = rng.integers(0, 2, N)
    Q0 = np.full((4, 4), 1.0 / 3.0)
    np.fill_diagonal(Q0, -1.0)
    Q1 = np.array([[-1.0, 0.2, 0.6, 0.2], [0.2, -1.0, 0.2, 0.6], [0.6, 0.2, -1.0, 0.2], [0.2, 0.6, 0.2, -1.0]])
    pi = np.full(4, 0.25)
    return W.Problem(name="two_subtrees", parent=parent, height=height, branch_rate=np.ones(2 * N - 1),
                     boundaries=np.array([0.5]), interval_process=np.array([0, 1], np.int32), Q=[Q0, Q1],
                     pi_process=[pi, pi], pi_root=pi, cat_rates=np.array([0.001, 10.0]),
                     cat_weights=np.array([0.5, 0.5]), tips=tips, weights=np.array([1.0, 2.0, 1.0]))


@pytest.mark.parametrize("kernel,options", [("auto", {"tree_walk": 0}), ("auto", {"tree_walk": 1}),
                                            ("generic", {})])
def test_fp32_underflow_is_a_warning_and_fp64_matches_the_oracle(kernel, options):
    prob = _two_subtree_problem()
    want_site = O.site_log_likelihoods(prob)
    assert np.all(np.isfinite(want_site))
    with from_problem(prob, "fp64", grad_branch=True, kernel=kernel, options=options) as lik:
        with warnings.catch_warnings():
            warnings.simplefilter("error")
            logL, site, db, _ = lik.evaluate(branch=True, site=True)
    assert rel(logL, float(np.dot(prob.weights, want_site))) <= TOL_LOGL["fp64"]
    assert np.all(np.isfinite(db))

    with from_problem(prob, "fp32", grad_branch=True, kernel=kernel, options=options) as lik:
        lik.update_transition_matrices()
        lik.update_partials()
        with pytest.warns(_abi.EpochUnderflowWarning):
            logL, site = lik.root_log_likelihood(site=True)
        assert logL == -np.inf and site[0] == -np.inf
        np.testing.assert_allclose(site[1:], want_site[1:], rtol=TOL_LOGL["fp32"] * 10)
        with pytest.raises(_abi.EpochError) as e:
            lik.gradient()
        assert e.value.code == _abi.EPOCH_ERR_NUMERIC
        with pytest.warns(_abi.EpochUnderflowWarning):
            logL2, _, db2, _ = lik.evaluate(branch=True)
        assert logL2 == -np.inf and np.all(np.isnan(db2))


def test_batch_member_underflow():
    bad = _two_subtree_problem()
    good = _two_subtree_problem()
    good.tips[:, 0] = good.tips[:, 1]
    want = float(np.dot(good.weights, O.site_log_likelihoods(good)))
    liks = [from_problem(p, "fp32", grad_branch=True) for p in (good, bad)]
    try:
        batch = EpochBatchEvaluator(liks)
        with pytest.warns(_abi.EpochUnderflowWarning):
            out = batch.evaluate(grad_branch=True)
        assert rel(out[0], want) <= TOL_LOGL["fp32"] and out[1] == -np.inf
        db, _ = batch.gradients(0)
        assert np.all(np.isfinite(db))
        with pytest.raises(_abi.EpochError) as e:
            batch.gradients(1)
        assert e.value.code == _abi.EPOCH_ERR_NUMERIC
        batch.close()
    finally:
        for lik in liks:
            lik.close()
