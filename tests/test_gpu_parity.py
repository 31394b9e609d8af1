"""Parity of the HIP path (through the C ABI) against the FP64 oracle.

Tolerances: |dlogL|/|logL| <= 1e-12 (FP64) and <= 1e-5 (FP32); per-site
log-likelihoods to 10x that relative bound plus an absolute floor of the bound
times the largest |site logL|; gradients ||dg||_2 / ||g||_2 <= 1e-6 (FP64) and
<= 1e-3 (FP32) and componentwise (tests/tolerances.py); transition matrices
entrywise to 1e-12 (FP64) / 2e-6 (FP32).
"""
import numpy as np
import pytest

from oracle import epoch_oracle as O
from paper_1309_3075_amd import _abi
from paper_1309_3075_amd import workloads as W
from paper_1309_3075_amd.likelihood import EpochLikelihood, from_problem
from tolerances import TOL_GRAD, TOL_LOGL, TOL_P, assert_grad, grad_rel, rel  # noqa: F401

pytestmark = pytest.mark.gpu


RANDOM_CASES = [
    # seed, tips, K, patterns, C, intervals, processes, reversible, tip_h, missing
    (101, 5, 2, 37, 1, 2, 2, True, 0.0, 0.0),
    (102, 9, 3, 300, 3, 3, 2, False, 0.2, 0.05),
    (103, 24, 4, 777, 4, 4, 3, True, 0.1, 0.02),
    (104, 7, 5, 65, 2, 2, 2, False, 0.0, 0.0),
    (105, 13, 20, 130, 2, 3, 3, True, 0.3, 0.0),
    (106, 11, 40, 19, 1, 6, 4, False, 0.0, 0.0),
    (107, 10, 61, 70, 1, 4, 4, True, 0.0, 0.0),
    (108, 6, 64, 33, 2, 2, 1, True, 0.0, 0.1),
    # 4-state cases for every category-group width of the specialised kernels
    (109, 17, 4, 200, 1, 2, 2, True, 0.1, 0.0),
    (110, 8, 4, 150, 2, 3, 2, False, 0.0, 0.05),
    (111, 12, 4, 333, 3, 2, 2, True, 0.2, 0.0),
    (112, 10, 4, 70, 5, 3, 3, True, 0.0, 0.0),
    (113, 9, 4, 90, 8, 2, 2, False, 0.1, 0.1),
]
GRAD_CASES = RANDOM_CASES


def _prob(case):
    seed, n, K, P, C, M, S, rev, th, miss = case
    rng = np.random.default_rng(seed)
    return W.random_problem(rng, n, K, P, n_categories=C, n_intervals=M, n_processes=S,
                            reversible=rev, tip_height_max=th, missing_frac=miss,
                            branch_rate_spread=0.25)


@pytest.mark.parametrize("use_pi", [False, True], ids=["eig", "sym"])
@pytest.mark.parametrize("kernel", ["generic", "auto"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", RANDOM_CASES, ids=[f"K{c[2]}_n{c[1]}_P{c[3]}" for c in RANDOM_CASES])
def test_random_problem_logL_and_P(case, precision, kernel, use_pi):
    prob = _prob(case)
    if use_pi and prob.pi_process[0] is None:
        pytest.skip("asymmetric model: no symmetric form")
    with from_problem(prob, precision, kernel=kernel, use_pi=use_pi) as lik:
        logL, site = lik.log_likelihood(site=True)
        P = lik.transition_matrices()
    want_site = O.site_log_likelihoods(prob)
    want = float(np.dot(prob.weights, want_site))
    assert rel(logL, want) <= TOL_LOGL[precision], (logL, want)
    np.testing.assert_allclose(site, want_site, rtol=TOL_LOGL[precision] * 10,
                               atol=TOL_LOGL[precision] * np.abs(want_site).max())
    Pw = O.transition_matrices(prob)
    Pw[-1] = 0.0
    np.testing.assert_allclose(P, Pw, rtol=0, atol=TOL_P[precision] * max(1.0, prob.n_states / 8))


@pytest.mark.parametrize("kernel", ["generic", "auto"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_C1_full_size(precision, kernel):
    prob = W.make_config(1)
    with from_problem(prob, precision, kernel=kernel) as lik:
        logL = lik.log_likelihood()
    want = O.log_likelihood(prob)
    assert rel(logL, want) <= TOL_LOGL[precision]


@pytest.mark.parametrize("kernel", ["generic", "auto"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", GRAD_CASES, ids=[f"K{c[2]}_n{c[1]}_C{c[4]}" for c in GRAD_CASES])
def test_gradients_against_oracle(case, precision, kernel):
    prob = _prob(case)
    with from_problem(prob, precision, grad_branch=True, grad_Q=True, kernel=kernel, use_pi=False) as lik:
        lik.log_likelihood()
        db, dq = lik.gradient(branch=True, Q=True)
    ref_b, ref_q = O.gradient(prob)
    assert_grad(db, ref_b, TOL_GRAD[precision])
    assert_grad(dq, ref_q, TOL_GRAD[precision])
    assert db[-1] == 0.0


def test_call_order_and_argument_errors():
    prob = _prob(RANDOM_CASES[0])
    lik = EpochLikelihood(prob.n_tips, prob.n_patterns, prob.n_states, 1, prob.n_processes,
                          prob.n_intervals, "fp64", grad_branch=True)
    with pytest.raises(_abi.EpochError) as e:
        lik.update_transition_matrices()
    assert e.value.code == _abi.EPOCH_ERR_STATE
    with pytest.raises(_abi.EpochError) as e:
        lik.update_partials()
    assert e.value.code == _abi.EPOCH_ERR_STATE
    bad = prob.tips.copy()
    bad[0, 0] = prob.n_states + 1
    with pytest.raises(_abi.EpochError) as e:
        lik.set_tip_states(bad)
    assert e.value.code == _abi.EPOCH_ERR_ARG
    with pytest.raises(_abi.EpochError):
        lik.set_categories([1.0], [0.5])
    with pytest.raises(_abi.EpochError):
        lik.set_root_frequencies(np.full(prob.n_states, 0.3))
    lik.close()
    lik = from_problem(prob, "fp64")
    lik.log_likelihood()
    with pytest.raises(_abi.EpochError) as e:
        lik.gradient()
    assert e.value.code == _abi.EPOCH_ERR_STATE
    lik.close()


def test_eigensystem_residual_warning():
    prob = _prob(RANDOM_CASES[2])
    with from_problem(prob, "fp64", use_pi=False) as lik:
        from paper_1309_3075_amd.eigen import eigensystem
        e = eigensystem(prob.Q[0])
        res = lik.set_eigensystem(0, e.V, e.Vinv, e.lambda_re, None, prob.Q[0])
        assert res < 1e-12
        wrong = e.lambda_re.copy()
        wrong[0] += 0.1
        res_bad = lik.set_eigensystem(0, e.V, e.Vinv, wrong, None, prob.Q[0])
        assert res_bad > 1e-3


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_C2_tree_reduced_patterns(precision):
    """The full 512-taxon C2 tree and model, 3000 simulated patterns, logL + branch gradients."""
    prob = W.make_config(2, n_patterns=3000)
    with from_problem(prob, precision, grad_branch=True) as lik:
        logL = lik.log_likelihood()
        db, _ = lik.gradient()
    want = O.log_likelihood(prob)
    ref_b, _ = O.gradient(prob, wrt=("branch",))
    assert rel(logL, want) <= TOL_LOGL[precision], rel(logL, want)
    assert_grad(db, ref_b, TOL_GRAD[precision])


def test_C2_full_tree_fp32_level_kernels_gradient():
    """The benchmarked 4-state kernels on the full 512-taxon C2 tree and model: FP32, level
    kernels (more than 1,024 tiles of 16 patterns, so the automatic choice is the level path
    that bench.py times), 30,000 simulated patterns; logL and all 1,022 branch gradients
    against the oracle on the same patterns."""
    prob = W.make_config(2, n_patterns=30000)
    with from_problem(prob, "fp32", grad_branch=True, options={"tree_walk": 0}) as lik:
        logL, _, db, _ = lik.evaluate(branch=True)
    want = O.log_likelihood(prob)
    ref_b, _ = O.gradient(prob, wrt=("branch",))
    assert rel(logL, want) <= TOL_LOGL["fp32"], rel(logL, want)
    assert_grad(db, ref_b, TOL_GRAD["fp32"], "dlogL/dl")


def test_repeat_evaluations_are_bitwise_identical():
    """No float atomics: the same inputs give the same bits on every evaluation."""
    prob = W.make_config(2, n_tips=64, n_patterns=5000)
    with from_problem(prob, "fp32", grad_branch=True) as lik:
        out = []
        for _ in range(3):
            lik.update_transition_matrices()
            lik.update_partials()
            logL = lik.root_log_likelihood()
            db, _ = lik.gradient()
            out.append((logL, db.copy()))
    for logL, db in out[1:]:
        assert logL == out[0][0]
        assert np.array_equal(db, out[0][1])


@pytest.mark.parametrize("kernel", ["auto", "generic"])
def test_codon_C3_tree(kernel):
    """GY94 61-state (padded to 64), 4 epochs, the full 128-taxon tree, 700 patterns
    (11 tiles of 64 with a ragged tail): logL, branch and rate-matrix gradients in FP32."""
    prob = W.make_config(3, n_patterns=700)
    with from_problem(prob, "fp32", grad_branch=True, grad_Q=True, kernel=kernel) as lik:
        logL = lik.log_likelihood()
        db, dq = lik.gradient(branch=True, Q=True)
    want = O.log_likelihood(prob)
    ref_b, ref_q = O.gradient(prob)
    assert rel(logL, want) <= TOL_LOGL["fp32"], rel(logL, want)
    assert_grad(db, ref_b, TOL_GRAD["fp32"])
    assert_grad(dq, ref_q, TOL_GRAD["fp32"])


def _codon_eval(prob, options):
    with from_problem(prob, "fp32", grad_branch=True, grad_Q=True, options=options) as lik:
        logL = lik.log_likelihood()
        db, dq = lik.gradient(branch=True, Q=True)
    return logL, db, dq


@pytest.mark.parametrize("n_patterns", [20, 700])
def test_codon_side_split_pre_order_matches_oracle(n_patterns):
    """Pre-order levels with each child branch on its own wavefronts (all levels, the
    default narrow ones, none) match the oracle and give the same bits."""
    prob = W.make_config(3, n_patterns=n_patterns)
    want = O.log_likelihood(prob)
    ref_b, ref_q = O.gradient(prob)
    out = [_codon_eval(prob, {"split_blocks": v}) for v in (0, 256, 1 << 30)]
    for logL, db, dq in out:
        assert rel(logL, want) <= TOL_LOGL["fp32"], rel(logL, want)
        assert_grad(db, ref_b, TOL_GRAD["fp32"])
        assert_grad(dq, ref_q, TOL_GRAD["fp32"])
    for logL, db, dq in out[1:]:
        assert logL == out[0][0] and np.array_equal(db, out[0][1]) and np.array_equal(dq, out[0][2])


@pytest.mark.parametrize("target_blocks", [64, 4096])
def test_codon_target_blocks_option(target_blocks):
    """Fewer or more blocks per 64-state level launch (more or fewer tiles per block) still
    match the oracle."""
    prob = W.make_config(3, n_patterns=2000)
    logL, db, dq = _codon_eval(prob, {"target_blocks": target_blocks})
    want = O.log_likelihood(prob)
    ref_b, ref_q = O.gradient(prob)
    assert rel(logL, want) <= TOL_LOGL["fp32"]
    assert_grad(db, ref_b, TOL_GRAD["fp32"])
    assert_grad(dq, ref_q, TOL_GRAD["fp32"])


def test_codon_side_split_several_tiles_per_block():
    """5000 patterns put several 64-pattern tiles on each block of the wide levels; the
    side-split kernel on every level gives the bits of the four-wavefront kernel."""
    prob = W.make_config(3, n_patterns=5000)
    a = _codon_eval(prob, {"split_blocks": 0})
    b = _codon_eval(prob, {"split_blocks": 1 << 30})
    assert a[0] == b[0] and np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


def test_codon_fp64_generic_C3_tree():
    prob = W.make_config(3, n_patterns=300)
    with from_problem(prob, "fp64", grad_branch=True) as lik:
        logL = lik.log_likelihood()
        db, _ = lik.gradient()
    assert rel(logL, O.log_likelihood(prob)) <= TOL_LOGL["fp64"]
    ref_b, _ = O.gradient(prob, wrt=("branch",))
    assert_grad(db, ref_b, TOL_GRAD["fp64"])


@pytest.mark.parametrize("kernel", ["auto", "generic"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_trait_C4_shape(precision, kernel):
    """40-state asymmetric CTMC (padded to 48), 12 processes cycled over 48 intervals,
    160-taxon tree: branches near the root cross up to dozens of intervals, so the
    epoch-product chains and their adjoints are long; logL, branch and Q gradients."""
    prob = W.make_config(4, n_tips=160)
    with from_problem(prob, precision, grad_branch=True, grad_Q=True, kernel=kernel, use_pi=False) as lik:
        logL = lik.log_likelihood()
        db, dq = lik.gradient(branch=True, Q=True)
    want = O.log_likelihood(prob)
    ref_b, ref_q = O.gradient(prob)
    assert rel(logL, want) <= TOL_LOGL[precision], rel(logL, want)
    assert_grad(db, ref_b, TOL_GRAD[precision])
    assert_grad(dq, ref_q, TOL_GRAD[precision])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("chain_split", [0, 2, 7])
def test_split_epoch_chains(precision, chain_split):
    """Epoch-product chains cut into two halves that run in parallel (every chain of at least
    chain_split segments; 0 = none): P, dP/dl (through the branch gradient), the stored forward
    products of the dlogL/dQ adjoint and its backward chain all match the oracle, and the
    unsplit evaluation to rounding."""
    prob = W.make_config(4, n_tips=160)
    opts = {"chain_split": chain_split}
    with from_problem(prob, precision, grad_branch=True, grad_Q=True, use_pi=False, options=opts) as lik:
        logL, _, db, dq = lik.evaluate(branch=True, Q=True)
        P = lik.transition_matrices()
    want = O.log_likelihood(prob)
    ref_b, ref_q = O.gradient(prob)
    assert rel(logL, want) <= TOL_LOGL[precision], rel(logL, want)
    assert_grad(db, ref_b, TOL_GRAD[precision])
    assert_grad(dq, ref_q, TOL_GRAD[precision])
    ref_P = O.transition_matrices(prob)
    ref_P[-1] = 0.0
    np.testing.assert_allclose(P, ref_P, rtol=0, atol=TOL_P[precision] * max(1.0, prob.n_states / 8))


def test_chain_split_option_between_evaluations():
    """Changing the chain split invalidates the state: the gradient is refused until the path
    runs again, and the new evaluation matches the oracle."""
    prob = W.make_config(4, n_tips=160)
    want = O.log_likelihood(prob)
    ref_b, ref_q = O.gradient(prob)
    with from_problem(prob, "fp64", grad_branch=True, grad_Q=True, use_pi=False, options={"chain_split": 2}) as lik:
        first = lik.evaluate(branch=True, Q=True)
        lik.set_option("chain_split", 7)
        with pytest.raises(Exception):
            lik.gradient(branch=True, Q=True)
        logL, _, db, dq = lik.evaluate(branch=True, Q=True)
    for l, b, q in ((first[0], first[2], first[3]), (logL, db, dq)):
        assert rel(l, want) <= TOL_LOGL["fp64"]
        assert_grad(b, ref_b, TOL_GRAD["fp64"])
        assert_grad(q, ref_q, TOL_GRAD["fp64"])


def test_trait_C4_full_size():
    """The full 2000-taxon 40-state workload in the benchmarked configuration (FP32,
    automatic kernels): logL and every gradient against the oracle."""
    prob = W.make_config(4)
    with from_problem(prob, "fp32", grad_branch=True, grad_Q=True, use_pi=False) as lik:
        logL = lik.log_likelihood()
        db, dq = lik.gradient(branch=True, Q=True)
    assert rel(logL, O.log_likelihood(prob)) <= TOL_LOGL["fp32"]
    ref_b, ref_q = O.gradient(prob)
    assert_grad(db, ref_b, TOL_GRAD["fp32"])
    assert_grad(dq, ref_q, TOL_GRAD["fp32"])


def _pattern_subset(prob, idx):
    import dataclasses
    return dataclasses.replace(prob, tips=prob.tips[:, idx], weights=prob.weights[idx])


@pytest.mark.parametrize("config", [2, 3])
def test_full_size_sampled_sites(config):
    """Full-size workloads in the benchmarked configuration (FP32, automatic kernels):
    site log-likelihoods of a sample of patterns (first, last and random ones, so the
    ragged last tile is included) against the oracle on those patterns alone."""
    prob = W.make_config(config)
    with from_problem(prob, "fp32", grad_branch=True, grad_Q=config == 3) as lik:
        _, site = lik.log_likelihood(site=True)
    rng = np.random.default_rng(7)
    idx = np.unique(np.concatenate([[0, prob.n_patterns - 1],
                                    rng.choice(prob.n_patterns, 150, replace=False)]))
    want = O.site_log_likelihoods(_pattern_subset(prob, idx))
    np.testing.assert_allclose(site[idx], want, rtol=TOL_LOGL["fp32"] * 10, atol=0)


@pytest.mark.parametrize("config", [2, 3])
def test_full_size_gradient_directional(config):
    """Full-size gradients checked by a property that holds at any size: the FP64 library
    logL along a random branch-length direction has central difference <dlogL/dl, d>."""
    prob = W.make_config(config)
    n = prob.parent.shape[0]
    tau = np.zeros(n)
    for v in range(n):
        if prob.parent[v] >= 0:
            tau[v] = prob.height[prob.parent[v]] - prob.height[v]
    rng = np.random.default_rng(11)
    # relative perturbations: coalescent tip branches can be ~1e-5 long
    d = prob.branch_rate * tau * rng.standard_normal(n)
    d[prob.parent < 0] = 0.0
    with from_problem(prob, "fp64", grad_branch=True) as lik:
        lik.log_likelihood()
        db, _ = lik.gradient()
        h = 1e-6
        vals = []
        for sgn in (1.0, -1.0):
            # l_v = r_v tau_v, so l + s h d is the rate r_v + s h d_v / tau_v
            rate = prob.branch_rate + np.where(tau > 0, sgn * h * d / np.where(tau > 0, tau, 1.0), 0.0)
            lik.set_tree(prob.parent, prob.height, rate, prob.boundaries, prob.interval_process)
            vals.append(lik.log_likelihood())
    fd = (vals[0] - vals[1]) / (2 * h)
    assert abs(fd - float(np.dot(db, d))) <= 1e-6 * abs(fd) + 1e-9 * np.linalg.norm(db * d), (fd, np.dot(db, d))


@pytest.mark.parametrize("case", [RANDOM_CASES[2], RANDOM_CASES[6], RANDOM_CASES[10]],
                         ids=lambda c: f"K{c[2]}_n{c[1]}")
def test_single_call_evaluation_matches_separate_calls(case):
    """epoch_evaluate (one host synchronisation) gives the same bits as the four
    separate calls, and its errors follow the same rules."""
    prob = _prob(case)
    with from_problem(prob, "fp32", grad_branch=True, grad_Q=True, use_pi=False) as lik:
        lik.update_transition_matrices()
        lik.update_partials()
        logL, site = lik.root_log_likelihood(site=True)
        db, dq = lik.gradient(branch=True, Q=True)
        l2, s2, db2, dq2 = lik.evaluate(branch=True, Q=True, site=True)
        l3, _, db3, dq3 = lik.evaluate()
    assert l2 == logL and l3 == logL
    assert np.array_equal(s2, site) and np.array_equal(db2, db) and np.array_equal(dq2, dq)
    assert db3 is None and dq3 is None
    with from_problem(prob, "fp32", grad_branch=True, use_pi=False) as lik:
        with pytest.raises(_abi.EpochError) as e:
            lik.evaluate(branch=True, Q=True)
        assert e.value.code == _abi.EPOCH_ERR_STATE
