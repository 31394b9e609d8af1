"""17- to 32-state models (a 20-state amino-acid-sized model) in FP32 with one category run on the
matrix-core kernels, padded to 32 states; against the FP64 oracle: logL, site
log-likelihoods, branch, rate-matrix and time gradients, ambiguous tips and incremental proposals."""
import dataclasses

import numpy as np
import pytest

from oracle import epoch_oracle as O
from paper_1309_3075_amd import workloads as W
from paper_1309_3075_amd.likelihood import from_problem
from tolerances import TOL_GRAD, TOL_LOGL, assert_grad, rel

pytestmark = pytest.mark.gpu


def _rand(seed, K, n=15, P=300, M=3, amb=0.0):
    rng = np.random.default_rng(seed)
    return W.random_problem(rng, n, K, P, n_categories=1, n_intervals=M, reversible=True, tip_height_max=0.2,
                            missing_frac=0.03, branch_rate_spread=0.2, ambiguous_frac=amb, n_ambiguity_sets=5)


CASES = {
    "K20_tree": lambda: W.make_config(6, n_tips=60, n_patterns=700),
    "K17": lambda: _rand(301, 17),
    "K32": lambda: _rand(302, 32),
    "K20_ambiguous": lambda: _rand(303, 20, amb=0.1),
}


@pytest.mark.parametrize("name", list(CASES))
def test_states20_on_matrix_cores_against_oracle(name):
    prob = CASES[name]()
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
    assert_grad(dbound, want_bd, TOL_GRAD["fp32"], "dlogL/db")


def test_states20_incremental_proposal():
    prob = W.make_config(6, n_tips=60, n_patterns=700)
    with from_problem(prob, "fp32") as lik:
        assert lik.kernel_path() == "matrix_core64"
        lik.log_likelihood()
        cur = dataclasses.replace(prob, branch_rate=prob.branch_rate.copy())
        cur.branch_rate[7] *= 1.4
        lik.set_branch_rates([7], [cur.branch_rate[7]])
        logL = lik.log_likelihood()
        assert lik.work_counts()[0] == 1
    with from_problem(cur, "fp32") as fresh:
        assert fresh.log_likelihood() == logL
    assert rel(logL, O.log_likelihood(cur)) <= TOL_LOGL["fp32"]
