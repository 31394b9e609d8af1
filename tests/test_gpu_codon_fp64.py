"""FP64 instances of 49-64 and 17-32 states on the matrix-core 64-state kernels (FP64 matrix
cores), with one or several rate categories, against the FP64 oracle at the FP64 tolerances:
logL, site log-likelihoods, branch, rate-matrix and time gradients; ambiguous tips; a merged
batch; an incremental proposal."""
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


def _rand(seed, K, C, n=14, P=250, amb=0.0, rev=True):
    rng = np.random.default_rng(seed)
    return W.random_problem(rng, n, K, P, n_categories=C, n_intervals=3, reversible=rev, tip_height_max=0.2,
                            missing_frac=0.03, branch_rate_spread=0.2, ambiguous_frac=amb, n_ambiguity_sets=5)


CASES = {
    "codon": lambda: W.make_config(3, n_tips=40, n_patterns=400),
    "codon_gamma4": lambda: _with_gamma(W.make_config(3, n_tips=24, n_patterns=300), 0.5, 4),
    "K20_gamma3": lambda: _rand(501, 20, 3),
    "K61_gamma2_ambiguous": lambda: _rand(502, 61, 2, amb=0.1),
    "K50_asymmetric": lambda: _rand(503, 50, 1, rev=False),
}


@pytest.mark.parametrize("name", list(CASES))
def test_fp64_on_matrix_cores_against_oracle(name):
    prob = CASES[name]()
    use_pi = prob.pi_process[0] is not None
    with from_problem(prob, "fp64", grad_branch=True, grad_Q=True, grad_time=True, use_pi=use_pi) as lik:
        assert lik.kernel_path() == "matrix_core64"
        logL, site, db, dq = lik.evaluate(branch=True, Q=True, site=True)
        dh, dbound = lik.time_gradient()
    want_site = O.site_log_likelihoods(prob)
    want = float(np.dot(prob.weights, want_site))
    assert rel(logL, want) <= TOL_LOGL["fp64"], (logL, want)
    np.testing.assert_allclose(site, want_site, rtol=TOL_LOGL["fp64"] * 10,
                               atol=TOL_LOGL["fp64"] * np.abs(want_site).max())
    ref_b, ref_q = O.gradient(prob)
    assert_grad(db, ref_b, TOL_GRAD["fp64"], "dlogL/dl")
    assert_grad(dq, ref_q, TOL_GRAD["fp64"], "dlogL/dQ")
    want_h, want_bd = O.time_gradient(prob)
    assert_grad(dh, want_h, TOL_GRAD["fp64"], "dlogL/dh")
    if np.any(want_bd != 0):
        assert_grad(dbound, want_bd, TOL_GRAD["fp64"], "dlogL/db")


def test_fp64_batch_and_incremental():
    probs = [CASES["codon"](), CASES["codon_gamma4"](), CASES["K20_gamma3"]()]
    liks = [from_problem(p, "fp64", grad_branch=True) for p in probs]
    try:
        single = [lik.evaluate(branch=True) for lik in liks]
        batch = EpochBatchEvaluator(liks)
        out = batch.evaluate(grad_branch=True)
        for i, p in enumerate(probs):
            assert out[i] == single[i][0]
            db, _ = batch.gradients(i)
            assert_grad(db, O.gradient(p, wrt=("branch",))[0], TOL_GRAD["fp64"], f"member {i} dlogL/dl")
        batch.close()
    finally:
        for lik in liks:
            lik.close()
    prob = CASES["codon_gamma4"]()
    with from_problem(prob, "fp64") as lik:
        lik.log_likelihood()
        cur = dataclasses.replace(prob, branch_rate=prob.branch_rate.copy())
        cur.branch_rate[6] *= 0.7
        lik.set_branch_rates([6], [cur.branch_rate[6]])
        logL = lik.log_likelihood()
        assert lik.work_counts()[0] == len(prob.cat_rates)
    with from_problem(cur, "fp64") as fresh:
        assert fresh.log_likelihood() == logL
    assert rel(logL, O.log_likelihood(cur)) <= TOL_LOGL["fp64"]
