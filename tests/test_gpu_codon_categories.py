"""Rate categories (discrete Gamma, text after Eq. 4) on the matrix-core 64-state kernels: each
category runs as a problem of its own and the root reduction combines them with per-category
scale exponents. Against the FP64 oracle: logL, site log-likelihoods, branch, rate-matrix and time
gradients; ambiguous tips; incremental proposals; a merged batch of members with different
category counts."""
import dataclasses

import numpy as np
import pytest

from oracle import epoch_oracle as O
from paper_1309_3075_amd import workloads as W
from paper_1309_3075_amd.likelihood import EpochBatchEvaluator, from_problem
from tolerances import TOL_GRAD, TOL_LOGL, assert_grad, rel

pytestmark = pytest.mark.gpu


def _with_gamma(prob, alpha, n_cat):
    rates, wts = W.discrete_gamma(alpha, n_cat)
    return dataclasses.replace(prob, cat_rates=np.asarray(rates), cat_weights=np.asarray(wts))


def _rand(seed, K, C, n=14, P=250, amb=0.0):
    rng = np.random.default_rng(seed)
    return W.random_problem(rng, n, K, P, n_categories=C, n_intervals=3, reversible=True, tip_height_max=0.2,
                            missing_frac=0.03, branch_rate_spread=0.2, ambiguous_frac=amb, n_ambiguity_sets=5)


CASES = {
    "codon_gamma4": lambda: _with_gamma(W.make_config(3, n_tips=40, n_patterns=400), 0.5, 4),
    "codon_gamma2": lambda: _with_gamma(W.make_config(3, n_tips=24, n_patterns=300), 1.0, 2),
    "K20_gamma3": lambda: _rand(401, 20, 3),
    "K61_gamma8_ambiguous": lambda: _rand(402, 61, 8, amb=0.1),
    "K32_gamma2": lambda: _rand(403, 32, 2),
}


@pytest.mark.parametrize("name", list(CASES))
def test_categories_on_matrix_cores_against_oracle(name):
    prob = CASES[name]()
    assert len(prob.cat_rates) > 1
    with from_problem(prob, "fp32", grad_branch=True, grad_Q=True, grad_time=True) as lik:
        assert lik.kernel_path() == "matrix_core64"
        logL, site, db, dq = lik.evaluate(branch=True, Q=True, site=True)
        dh, dbound = lik.time_gradient()
    want_site = O.site_log_likelihoods(prob)
    want = float(np.dot(prob.weights, want_site))
    assert rel(logL, want) <= TOL_LOGL["fp32"], (logL, want)
    np.testing.assert_allclose(site, want_site, rtol=TOL_LOGL["fp32"] * 10,
                               atol=TOL_LOGL["fp32"] * np.abs(want_site).max())
    ref_b, ref_q = O.gradient(prob)
    assert_grad(db, ref_b, TOL_GRAD["fp32"], "dlogL/dl")
    assert_grad(dq, ref_q, TOL_GRAD["fp32"], "dlogL/dQ")
    want_h, want_bd = O.time_gradient(prob)
    assert_grad(dh, want_h, TOL_GRAD["fp32"], "dlogL/dh")
    if np.any(want_bd != 0):
        assert_grad(dbound, want_bd, TOL_GRAD["fp32"], "dlogL/db")
    else:  # one process on both sides of every boundary: moving it changes nothing
        assert np.all(np.abs(dbound) <= TOL_GRAD["fp32"] * np.abs(want_h).max())


def test_categories_split_and_level_kernels_agree():
    """Every pre-order level on the side-split kernel gives the bits of the level kernel."""
    prob = CASES["codon_gamma4"]()
    out = []
    for split in (0, 1 << 30):
        with from_problem(prob, "fp32", grad_branch=True, options={"split_blocks": split}) as lik:
            out.append(lik.evaluate(branch=True))
    assert out[0][0] == out[1][0] and np.array_equal(out[0][2], out[1][2])


def test_categories_incremental_proposal():
    prob = CASES["codon_gamma2"]()
    with from_problem(prob, "fp32") as lik:
        lik.log_likelihood()
        cur = dataclasses.replace(prob, branch_rate=prob.branch_rate.copy())
        cur.branch_rate[5] *= 1.3
        lik.set_branch_rates([5], [cur.branch_rate[5]])
        logL = lik.log_likelihood()
        assert lik.work_counts()[0] == len(prob.cat_rates)  # one branch x its categories
    with from_problem(cur, "fp32") as fresh:
        assert fresh.log_likelihood() == logL
    assert rel(logL, O.log_likelihood(cur)) <= TOL_LOGL["fp32"]


def test_batch_members_with_categories():
    probs = [CASES["codon_gamma4"](), W.make_config(3, n_tips=30, n_patterns=200), CASES["codon_gamma2"]()]
    liks = [from_problem(p, "fp32", grad_branch=True) for p in probs]
    try:
        single = [lik.evaluate(branch=True) for lik in liks]
        batch = EpochBatchEvaluator(liks)
        out = batch.evaluate(grad_branch=True)
        for i, p in enumerate(probs):
            assert out[i] == single[i][0]  # the post-order pass does not depend on the launch shape
            db, _ = batch.gradients(i)
            ref_b, _ = O.gradient(p, wrt=("branch",))
            assert_grad(db, ref_b, TOL_GRAD["fp32"], f"member {i} dlogL/dl")
        batch.close()
    finally:
        for lik in liks:
            lik.close()
