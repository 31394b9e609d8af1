"""Batched evaluation in one replayed HIP graph (C ABI epoch_batch_*)."""
import os
import tempfile

import numpy as np
import pytest

from oracle import epoch_oracle as O
from paper_1309_3075_amd import workloads as W
from paper_1309_3075_amd.likelihood import EpochBatchEvaluator, from_problem

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
    assert b2.target_blocks() == batch.target_blocks()
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
