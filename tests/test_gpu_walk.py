"""4-state tree-walk kernels (an opt-in alternative to the level kernels)
against the FP64 oracle, through the C ABI: every category packing, ragged
pattern tiles, recomputation thresholds, strided tiles, deep (caterpillar) and
balanced trees; the level kernels under their tiling option; and evaluation
under an HBM budget (4-state recomputation, 64-state pattern chunks)."""
import dataclasses

import numpy as np
import pytest

from oracle import epoch_oracle as O
from paper_1309_3075_amd import workloads as W
from paper_1309_3075_amd.likelihood import from_problem

pytestmark = pytest.mark.gpu

TOL_LOGL = {"fp64": 1e-12, "fp32": 1e-5}
TOL_GRAD = {"fp64": 1e-6, "fp32": 1e-3}


def _check(prob, precision, options=None, grad_Q=False):
    options = {"tree_walk": 1, **(options or {})}
    with from_problem(prob, precision, grad_branch=True, grad_Q=grad_Q, options=options) as lik:
        logL, site, db, dq = lik.evaluate(branch=True, Q=grad_Q, site=True)
    want_site = O.site_log_likelihoods(prob)
    want = float(np.dot(prob.weights, want_site))
    assert abs(logL - want) <= TOL_LOGL[precision] * abs(want), (logL, want)
    assert np.max(np.abs(site - want_site)) <= TOL_LOGL[precision] * 10 * np.max(np.abs(want_site))
    ref_b, ref_q = O.gradient(prob, wrt=("branch", "Q") if grad_Q else ("branch",))
    assert np.linalg.norm(db - ref_b) <= TOL_GRAD[precision] * np.linalg.norm(ref_b), \
        np.linalg.norm(db - ref_b) / np.linalg.norm(ref_b)
    if grad_Q:
        assert np.linalg.norm(dq - ref_q) <= TOL_GRAD[precision] * np.linalg.norm(ref_q)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("C", [1, 2, 4, 5])
@pytest.mark.parametrize("P", [1, 17, 100])
def test_walk_categories_and_tiles(C, P, precision):
    rng = np.random.default_rng(5000 + 10 * C + P)
    prob = W.random_problem(rng, 19, 4, P, n_categories=C, n_intervals=3, reversible=False, missing_frac=0.05)
    _check(prob, precision)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("recompute", [3, 8, 40])
def test_walk_recompute_thresholds(recompute, precision):
    rng = np.random.default_rng(5100 + recompute)
    prob = W.random_problem(rng, 40, 4, 70, n_categories=4, n_intervals=3, reversible=True,
                            tip_height_max=0.2, missing_frac=0.05)
    _check(prob, precision, options={"walk_recompute": recompute})


@pytest.mark.parametrize("tiles", [1, 2])
@pytest.mark.parametrize("blocks", [1, 3])
def test_walk_strided_tiles(blocks, tiles):
    """Fewer blocks than tiles: each wavefront walks several groups of tiles in turn."""
    rng = np.random.default_rng(5200 + blocks)
    prob = W.random_problem(rng, 25, 4, 300, n_categories=4, n_intervals=2)
    _check(prob, "fp32", options={"walk_blocks": blocks, "walk_tiles": tiles})


@pytest.mark.parametrize("C", [1, 3, 8])
def test_walk_one_tile_per_wavefront(C):
    rng = np.random.default_rng(5250 + C)
    prob = W.random_problem(rng, 33, 4, 150, n_categories=C, n_intervals=3, reversible=False, missing_frac=0.05)
    _check(prob, "fp32", options={"walk_tiles": 1})


def _shaped(parent, seed, P=60, C=4):
    rng = np.random.default_rng(seed)
    n = len(parent)
    N = (n + 1) // 2
    prob = W.random_problem(rng, N, 4, P, n_categories=C, n_intervals=3, reversible=False)
    height = np.zeros(n)
    for u in range(N, n):
        height[u] = 1.0 + max(height[v] for v in range(n) if parent[v] == u)
    return dataclasses.replace(prob, parent=np.asarray(parent, np.int32), height=height / height[-1])


def test_walk_caterpillar_tree():
    N = 60
    parent = [-1] * (2 * N - 1)
    parent[0] = parent[1] = N
    for k in range(2, N):
        parent[k] = N + k - 1
        parent[N + k - 2] = N + k - 1
    _check(_shaped(parent, 5300), "fp32")
    _check(_shaped(parent, 5301), "fp64")


def test_walk_balanced_tree():
    N = 64
    parent = [-1] * (2 * N - 1)
    level, nxt = list(range(N)), N
    while len(level) > 1:
        new = []
        for i in range(0, len(level), 2):
            parent[level[i]] = parent[level[i + 1]] = nxt
            new.append(nxt)
            nxt += 1
        level = new
    _check(_shaped(parent, 5400), "fp32")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("min_tiles", [1, 8, 64])
def test_level_kernels_still_match(precision, min_tiles):
    rng = np.random.default_rng(5500)
    prob = W.random_problem(rng, 30, 4, 2000, n_categories=4, n_intervals=3, reversible=False, missing_frac=0.05)
    _check(prob, precision, options={"tree_walk": 0, "level_min_tiles": min_tiles})


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_walk_post_with_rate_matrix_gradient(precision):
    """dlogL/dQ takes the level pre-order kernels on the walk's stored partials."""
    rng = np.random.default_rng(5600)
    prob = W.random_problem(rng, 30, 4, 90, n_categories=4, n_intervals=3, reversible=False)
    _check(prob, precision, grad_Q=True)


def test_walk_and_level_agree_at_c2_shape():
    """The same 512-taxon problem through both 4-state paths (FP32)."""
    prob = W.make_config(2, n_patterns=3000)
    with from_problem(prob, "fp32", grad_branch=True, options={"tree_walk": 1}) as lik:
        a = lik.evaluate(branch=True)
    with from_problem(prob, "fp32", grad_branch=True, options={"tree_walk": 0}) as lik:
        b = lik.evaluate(branch=True)
    assert abs(a[0] - b[0]) <= 1e-5 * abs(b[0])
    assert np.linalg.norm(a[2] - b[2]) <= 1e-3 * np.linalg.norm(b[2])


def _budget_for(prob, precision, n_stored):
    """Bytes the library needs to store n_stored partials (plus its root scale row and gradient rows)."""
    P, C = prob.n_patterns, len(prob.cat_rates)
    R = 8 if precision == "fp64" else 4
    n_nodes = 2 * prob.n_tips - 1
    cp = 1 if C <= 1 else (2 if C <= 2 else (4 if C <= 4 else 8))
    tiles = -(-P // (64 // cp))
    rows = -(-(tiles * n_nodes * R) // 256) * 256 + 32 * n_nodes * 8
    return n_stored * P * C * 4 * R + 4 * P + rows


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("n_stored", [1, 4, 12])
def test_hbm_budget_recomputes_partials(n_stored, precision):
    """Under an HBM budget only the partials of the largest subtrees are stored; the
    gradient pass recomputes the rest from the tip states.  Results match the oracle
    and the unbudgeted instance."""
    rng = np.random.default_rng(5700 + n_stored)
    prob = W.random_problem(rng, 48, 4, 400, n_categories=4, n_intervals=3, reversible=False, missing_frac=0.05)
    budget = _budget_for(prob, precision, n_stored)
    with from_problem(prob, precision, grad_branch=True, hbm_budget_bytes=budget) as lik:
        logL, site, db, _ = lik.evaluate(branch=True, site=True)
        logL2, _, db2, _ = lik.evaluate(branch=True)  # a second evaluation reuses the compact slots
    with from_problem(prob, precision, grad_branch=True, options={"tree_walk": 1}) as lik:
        ref_logL, _, ref_db, _ = lik.evaluate(branch=True)
    want = O.log_likelihood(prob)
    assert abs(logL - want) <= TOL_LOGL[precision] * abs(want)
    assert logL2 == logL and np.array_equal(db, db2)
    ob, _ = O.gradient(prob, wrt=("branch",))
    assert np.linalg.norm(db - ob) <= TOL_GRAD[precision] * np.linalg.norm(ob)
    assert abs(logL - ref_logL) <= TOL_LOGL[precision] * abs(want)
    assert np.linalg.norm(db - ref_db) <= TOL_GRAD[precision] * np.linalg.norm(ob)


def test_hbm_budget_too_small_is_refused():
    rng = np.random.default_rng(5800)
    prob = W.random_problem(rng, 20, 4, 300, n_categories=4, n_intervals=2)
    with pytest.raises(Exception, match="hbm_budget_bytes"):
        from_problem(prob, "fp32", grad_branch=True, hbm_budget_bytes=_budget_for(prob, "fp32", 1) - 1)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_caller_owned_workspace(precision):
    """Pattern-sized buffers inside a torch tensor give the same results as library-owned ones."""
    import torch
    from paper_1309_3075_amd.likelihood import EpochLikelihood
    rng = np.random.default_rng(5900)
    prob = W.random_problem(rng, 30, 4, 700, n_categories=4, n_intervals=3, reversible=False)
    nbytes = EpochLikelihood.workspace_bytes(prob.n_tips, prob.n_patterns, 4, 4, precision, grad_branch=True)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    with from_problem(prob, precision, grad_branch=True, workspace=ws) as lik:
        a = lik.evaluate(branch=True, site=True)
    torch.cuda.synchronize()
    with from_problem(prob, precision, grad_branch=True) as lik:
        b = lik.evaluate(branch=True, site=True)
    assert a[0] == b[0] and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


def _codon_budget(prob, patterns_per_chunk, grad=True):
    """Budget that gives the 64-state path chunks of patterns_per_chunk patterns (a multiple of 64)."""
    nm1 = prob.n_tips - 1
    per = nm1 * (64 * 4 + 4) + (nm1 * 64 * 4 + 2 * nm1 * 64 * 64 * 4 // 64 if grad else 0)
    return per * patterns_per_chunk


@pytest.mark.parametrize("split_blocks", [256, 0])
@pytest.mark.parametrize("chunk", [64, 192])
def test_codon_hbm_budget_streams_pattern_chunks(chunk, split_blocks):
    """Under a budget the 64-state path evaluates the patterns in chunks (the last one
    ragged); the gradient call forms each chunk's partials again.  Results match the
    oracle and the unbudgeted instance, through the separate calls and the single call,
    with the pre-order levels on the side-split kernel (the default here) or all on the
    four-wavefront kernel (split_blocks 0); both zero the slots of blocks past a short chunk."""
    prob = W.make_config(3, n_patterns=700)
    budget = _codon_budget(prob, chunk)
    with from_problem(prob, "fp32", grad_branch=True, grad_Q=True, hbm_budget_bytes=budget,
                      options={"split_blocks": split_blocks}) as lik:
        logL, site = lik.log_likelihood(site=True)
        db, dq = lik.gradient(branch=True, Q=True)
        one = lik.evaluate(branch=True, Q=True, site=True)
        again = lik.evaluate(branch=True, Q=True, site=True)
    with from_problem(prob, "fp32", grad_branch=True, grad_Q=True) as lik:
        ref = lik.evaluate(branch=True, Q=True, site=True)
    want = O.log_likelihood(prob)
    ob, oq = O.gradient(prob)
    assert abs(logL - want) <= TOL_LOGL["fp32"] * abs(want)
    assert np.linalg.norm(db - ob) <= TOL_GRAD["fp32"] * np.linalg.norm(ob)
    assert np.linalg.norm(dq - oq) <= TOL_GRAD["fp32"] * np.linalg.norm(oq)
    # the same FP32 partials; only the FP64 sums over chunks are ordered differently
    assert abs(logL - ref[0]) <= 1e-13 * abs(want) and abs(one[0] - logL) <= 1e-13 * abs(want)
    assert np.array_equal(site, ref[1]) and np.array_equal(one[1], ref[1])
    assert np.linalg.norm(db - ref[2]) <= 1e-12 * np.linalg.norm(ob)
    assert np.linalg.norm(dq - ref[3]) <= 1e-12 * np.linalg.norm(oq)
    assert np.linalg.norm(one[2] - db) <= 1e-12 * np.linalg.norm(ob)
    assert again[0] == one[0] and np.array_equal(again[2], one[2]) and np.array_equal(again[3], one[3])


def test_codon_hbm_budget_logL_only_and_large_budget():
    prob = W.make_config(3, n_patterns=300)
    with from_problem(prob, "fp32", hbm_budget_bytes=_codon_budget(prob, 128, grad=False)) as lik:
        logL = lik.log_likelihood()
    with from_problem(prob, "fp32", grad_branch=True, hbm_budget_bytes=1 << 40) as lik:  # one chunk
        big = lik.evaluate(branch=True)
    want = O.log_likelihood(prob)
    assert abs(logL - want) <= TOL_LOGL["fp32"] * abs(want)
    assert abs(big[0] - want) <= TOL_LOGL["fp32"] * abs(want)


def test_codon_hbm_budget_too_small_is_refused():
    prob = W.make_config(3, n_patterns=300)
    with pytest.raises(Exception, match="hbm_budget_bytes"):
        from_problem(prob, "fp32", grad_branch=True, hbm_budget_bytes=_codon_budget(prob, 64) - 1)


def _generic_budget(prob, precision, patterns_per_chunk, grad=True):
    """Budget that gives the generic path chunks of patterns_per_chunk patterns (a multiple of 64)."""
    K = prob.n_states
    kp = 4 if K <= 4 else (8 if K <= 8 else -(-K // 16) * 16)
    row = len(prob.cat_rates) * kp * (8 if precision == "fp64" else 4)
    return (prob.n_tips - 1) * (row * (2 if grad else 1) + 4) * patterns_per_chunk


@pytest.mark.parametrize("K,C,kernel,precision", [(20, 2, "auto", "fp64"), (20, 2, "auto", "fp32"),
                                                  (4, 4, "generic", "fp32"), (61, 1, "auto", "fp64")])
def test_generic_hbm_budget_streams_pattern_chunks(K, C, kernel, precision):
    """The generic path under a budget: chunks of 64 patterns (the last one ragged), partials
    formed again chunk by chunk in the gradient call; logL, site logL and both gradients match
    the oracle and the unbudgeted instance."""
    rng = np.random.default_rng(6000 + K + C)
    prob = W.random_problem(rng, 20, K, 300, n_categories=C, n_intervals=3, reversible=False, missing_frac=0.05)
    budget = _generic_budget(prob, precision, 64)
    kw = dict(grad_branch=True, grad_Q=True, kernel=kernel)
    with from_problem(prob, precision, hbm_budget_bytes=budget, **kw) as lik:
        logL, site = lik.log_likelihood(site=True)
        db, dq = lik.gradient(branch=True, Q=True)
        one = lik.evaluate(branch=True, Q=True, site=True)
        path = lik.kernel_path()
    with from_problem(prob, precision, **kw) as lik:
        ref = lik.evaluate(branch=True, Q=True, site=True)
        same_kernels = lik.kernel_path() == path
    want = O.log_likelihood(prob)
    ob, oq = O.gradient(prob)
    assert abs(logL - want) <= TOL_LOGL[precision] * abs(want)
    assert np.linalg.norm(db - ob) <= TOL_GRAD[precision] * np.linalg.norm(ob)
    assert np.linalg.norm(dq - oq) <= TOL_GRAD[precision] * np.linalg.norm(oq)
    assert np.array_equal(one[1], site)
    if not same_kernels:
        # several categories of 17-32 states: without a budget the matrix-core kernels take them
        # (they take a budget with one category only), so the two instances round differently
        np.testing.assert_allclose(site, ref[1], rtol=TOL_LOGL[precision] * 10)
        return
    # per-pattern values are those of the unbudgeted instance; only sums over chunks regroup
    assert np.array_equal(site, ref[1])
    assert abs(logL - ref[0]) <= 1e-13 * abs(want) and abs(one[0] - logL) <= 1e-13 * abs(want)
    tol = 1e-12 if precision == "fp64" else 1e-5
    assert np.linalg.norm(db - ref[2]) <= tol * np.linalg.norm(ob)
    assert np.linalg.norm(dq - ref[3]) <= tol * np.linalg.norm(oq)
    assert np.array_equal(one[2], db) and np.array_equal(one[3], dq)


def test_generic_hbm_budget_too_small_is_refused():
    rng = np.random.default_rng(6100)
    prob = W.random_problem(rng, 12, 20, 200)
    with pytest.raises(Exception, match="hbm_budget_bytes"):
        from_problem(prob, "fp64", grad_branch=True, hbm_budget_bytes=_generic_budget(prob, "fp64", 64) - 1)
