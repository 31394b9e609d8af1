"""Batched evaluation in one replayed HIP graph (C ABI epoch_batch_*)."""
import os
import tempfile

import numpy as np
import pytest

from oracle import epoch_oracle as O
from paper_1309_3075_amd import workloads as W
from paper_1309_3075_amd import _abi
from paper_1309_3075_amd.likelihood import EpochBatchEvaluator, from_problem
from tolerances import TOL_GRAD, TOL_LOGL, assert_grad, rel

pytestmark = pytest.mark.gpu


def _members(probs, precision="fp32"):
    return [from_problem(p, precision, grad_branch=True, grad_Q=True) for p in probs]


def test_codon_batch_matches_oracle_and_single_instances():
    probs = W.make_batch(5, scale=0.08)
    members = _members(probs)
    cache = os.path.join(tempfile.mkdtemp(), "tune.json")
    batch = EpochBatchEvaluator(members, tune_cache=cache)
    logL = batch.evaluate(grad_branch=True, grad_Q=True)
    assert os.path.exists(cache) and batch.target_blocks() > 0
    for i, p in enumerate(probs):
        want = O.log_likelihood(p)
        assert abs(logL[i] - want) / abs(want) <= 1e-5, (i, logL[i], want)
        db, dq = batch.gradients(i, branch=True, Q=True)
        ref_b, ref_q = O.gradient(p)
        assert np.linalg.norm(db - ref_b) / np.linalg.norm(ref_b) <= 1e-3
        assert np.linalg.norm(dq - ref_q) / np.linalg.norm(ref_q) <= 1e-3
    # replays give the same bits
    again = batch.evaluate(grad_branch=True, grad_Q=True)
    assert np.array_equal(again, logL)
    # a tree change forces a new capture and stays correct
    p0 = probs[0]
    p0.branch_rate = p0.branch_rate * 1.3
    members[0].set_tree(p0.parent, p0.height, p0.branch_rate, p0.boundaries, p0.interval_process)
    l2 = batch.evaluate(grad_branch=True)
    assert abs(l2[0] - O.log_likelihood(p0)) / abs(l2[0]) <= 1e-5
    assert np.array_equal(l2[1:], logL[1:])
    # the tuned shape is read back from the cache by a new batch
    b2 = EpochBatchEvaluator(members, tune_cache=cache)
    b2.evaluate(grad_branch=False)
    assert b2.target_blocks() == batch.target_blocks() and b2.split_blocks() == batch.split_blocks()
    b2.close()
    batch.close()
    for m in members:
        m.close()


def test_nucleotide_batch_unmerged_path():
    probs = [W.make_config(2, replicate=r, n_tips=20 + 7 * r, n_patterns=300 + 211 * r) for r in range(3)]
    members = _members(probs)
    batch = EpochBatchEvaluator(members)
    for step in range(2):
        if step == 1:
            # options on a member (level kernels with one tile per wavefront: more gradient slots,
            # a larger slot buffer) make the batch capture its graph again
            for m in members:
                m.set_option("tree_walk", 0)
            members[0].set_option("level_min_tiles", 1)
        logL = batch.evaluate(grad_branch=True)
        for i, p in enumerate(probs):
            want = O.log_likelihood(p)
            assert abs(logL[i] - want) / abs(want) <= 1e-5, (step, i)
            db, _ = batch.gradients(i)
            ref_b, _ = O.gradient(p, wrt=("branch",))
            assert np.linalg.norm(db - ref_b) / np.linalg.norm(ref_b) <= 1e-3, (step, i)
    batch.close()
    for m in members:
        m.close()


def test_members_on_concurrent_branches_match_single_evaluations():
    """Members that run their own launches are captured on concurrent branches: eleven members
    of three kernel families (4-state walk and level kernels, generic 20-state with dlogL/dQ, a
    40-state member) give the bits of their single evaluations, on every replay."""
    rng = np.random.default_rng(77)
    probs, opts = [], []
    for r in range(6):
        probs.append(W.make_config(1, replicate=r, n_tips=int(rng.integers(10, 40)), n_patterns=int(rng.integers(50, 900))))
        opts.append({"tree_walk": r % 2})
    for r in range(4):
        probs.append(W.random_problem(np.random.default_rng(300 + r), 12 + r, 20, 40 + 10 * r, n_categories=2,
                                      n_intervals=3, reversible=True))
        opts.append({})
    probs.append(W.make_config(4, n_tips=40))
    opts.append({})
    members = [from_problem(p, "fp32", grad_branch=True, grad_Q=True, kernel="auto" if i < 6 else "generic",
                            use_pi=i < 10, options=o) for i, (p, o) in enumerate(zip(probs, opts))]
    try:
        single = [m.evaluate(branch=True, Q=True) for m in members]
        batch = EpochBatchEvaluator(members)
        for _ in range(3):
            logL = batch.evaluate(grad_branch=True, grad_Q=True)
            for i in range(len(members)):
                assert logL[i] == single[i][0], i
                db, dq = batch.gradients(i, branch=True, Q=True)
                assert np.array_equal(db, single[i][2]) and np.array_equal(dq, single[i][3]), i
        for i in (0, 7, 10):
            assert rel(logL[i], O.log_likelihood(probs[i])) <= TOL_LOGL["fp32"], i
        batch.close()
    finally:
        for m in members:
            m.close()


def test_batch_with_a_pattern_chunked_codon_member():
    """A 64-state member under an HBM budget (pattern chunks) leaves the merged launches and is
    evaluated on its own inside the batch; every member still matches the oracle."""
    probs = W.make_batch(3, scale=0.05)
    p0 = probs[0]
    nm1 = p0.n_tips - 1
    budget = (nm1 * (64 * 4 + 4) + nm1 * 64 * 4 + 2 * nm1 * 64 * 64 * 4 // 64) * 64  # chunks of 64 patterns
    members = [from_problem(p0, "fp32", grad_branch=True, hbm_budget_bytes=budget)] + \
              [from_problem(p, "fp32", grad_branch=True) for p in probs[1:]]
    batch = EpochBatchEvaluator(members)
    logL = batch.evaluate(grad_branch=True)
    again = batch.evaluate(grad_branch=True)
    assert np.array_equal(logL, again)
    for i, p in enumerate(probs):
        want = O.log_likelihood(p)
        assert abs(logL[i] - want) / abs(want) <= 1e-5, (i, logL[i], want)
        db, _ = batch.gradients(i)
        ref_b, _ = O.gradient(p, wrt=("branch",))
        assert np.linalg.norm(db - ref_b) / np.linalg.norm(ref_b) <= 1e-3
    batch.close()
    for m in members:
        m.close()


def test_one_member_batch_splits_chains_and_recaptures_after_an_option():
    """A batch of one 40-state member runs that member's own P stage inside the graph (long epoch
    chains cut into parts); changing an option on the member (here the chain split, which rebuilds
    its chain work lists) makes the batch capture its graph again.  Every evaluation, and its
    replay, matches the oracle."""
    prob = W.make_config(4, n_tips=160)
    want = O.log_likelihood(prob)
    ref_b, ref_q = O.gradient(prob)
    with from_problem(prob, "fp64", grad_branch=True, grad_Q=True, use_pi=False,
                      options={"chain_split": 7}) as lik:
        batch = EpochBatchEvaluator([lik])
        for split in (7, 2, 0):
            lik.set_option("chain_split", split)
            logL = batch.evaluate(grad_branch=True, grad_Q=True)
            again = batch.evaluate(grad_branch=True, grad_Q=True)
            assert np.array_equal(logL, again)
            db, dq = batch.gradients(0, branch=True, Q=True)
            assert abs(logL[0] - want) / abs(want) <= 1e-12, (split, logL[0], want)
            assert np.linalg.norm(db - ref_b) / np.linalg.norm(ref_b) <= 1e-6, split
            assert np.linalg.norm(dq - ref_q) / np.linalg.norm(ref_q) <= 1e-6, split
        batch.close()


def test_logL_only_codon_batch_tunes_and_matches_oracle():
    """A merged 64-state batch whose members keep no gradient buffers: the first evaluation tunes
    the launch shape with log-likelihood-only replays, every member matches the oracle, and a
    gradient request is refused."""
    probs = W.make_batch(4, scale=0.05)
    members = [from_problem(p, "fp32") for p in probs]
    cache = os.path.join(tempfile.mkdtemp(), "tune.json")  # empty cache: the tuner runs
    batch = EpochBatchEvaluator(members, tune_cache=cache)
    logL = batch.evaluate(grad_branch=False)
    assert os.path.exists(cache)
    for i, p in enumerate(probs):
        assert rel(logL[i], O.log_likelihood(p)) <= TOL_LOGL["fp32"], i
    assert np.array_equal(batch.evaluate(grad_branch=False), logL)
    with pytest.raises(_abi.EpochError) as e:
        batch.evaluate(grad_branch=True)
    assert e.value.code == _abi.EPOCH_ERR_STATE
    batch.close()
    for m in members:
        m.close()


@pytest.fixture(scope="module")
def full_c5():
    """The full batched codon workload (64 GY94 problems, 64-256 taxa, 1,000-20,000 patterns
    each) in the configuration bench.py times, evaluated once with branch and rate-matrix
    gradients."""
    probs = W.make_batch(64)
    members = [from_problem(p, "fp32", grad_branch=True, grad_Q=True) for p in probs]
    batch = EpochBatchEvaluator(members, tune_cache=os.path.join(tempfile.mkdtemp(), "tune.json"))
    logL = batch.evaluate(grad_branch=True, grad_Q=True)
    grads = [batch.gradients(i, branch=True, Q=True) for i in range(len(probs))]
    yield probs, members, batch, logL, grads
    batch.close()
    for m in members:
        m.close()


def test_full_C5_batch_every_member_sites(full_c5):
    """Every member of the full batch: its root log-likelihood, formed again from the partials
    the batched launches left, reproduces the batch's logL, and its per-site log-likelihoods on
    sampled patterns (first, last and random) match the oracle on those patterns."""
    import dataclasses
    probs, members, _, logL, _ = full_c5
    rng = np.random.default_rng(5)
    for i, (p, m) in enumerate(zip(probs, members)):
        again, site = m.root_log_likelihood(site=True)
        assert again == logL[i], (i, again, logL[i])
        idx = np.unique(np.concatenate([[0, p.n_patterns - 1], rng.choice(p.n_patterns, 24, replace=False)]))
        sub = dataclasses.replace(p, tips=p.tips[:, idx], weights=p.weights[idx])
        want = O.site_log_likelihoods(sub)
        np.testing.assert_allclose(site[idx], want, rtol=TOL_LOGL["fp32"] * 10, atol=0, err_msg=f"member {i}")


def _checked_members(probs):
    size = [p.n_tips * p.n_patterns for p in probs]
    order = np.argsort(size)
    # the largest, the smallest and six spread between them
    return sorted({int(order[-1]), int(order[0])} | {int(order[k]) for k in np.linspace(1, len(probs) - 2, 6).astype(int)})


def test_full_C5_batch_logL_of_eight_members(full_c5):
    probs, _, _, logL, _ = full_c5
    for i in _checked_members(probs):
        want = O.log_likelihood(probs[i])
        assert rel(logL[i], want) <= TOL_LOGL["fp32"], (i, logL[i], want)


@pytest.mark.parametrize("half", [0, 1])
def test_full_C5_batch_gradients_of_eight_members(full_c5, half):
    """Branch and per-epoch rate-matrix gradients (through which torch forms the omega
    gradients) of eight members including the largest, against the oracle."""
    probs, _, _, _, grads = full_c5
    chosen = _checked_members(probs)
    for i in chosen[half::2]:
        ref_b, ref_q = O.gradient(probs[i])
        db, dq = grads[i]
        assert_grad(db, ref_b, TOL_GRAD["fp32"], f"member {i} dlogL/dl")
        assert_grad(dq, ref_q, TOL_GRAD["fp32"], f"member {i} dlogL/dQ")
