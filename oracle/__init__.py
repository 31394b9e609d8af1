"""FP64 CPU oracle for the epoch-model likelihood.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the library's product path.
"""
from .epoch_oracle import (branch_segments, epoch_P, homogeneous_P, transition_matrices,
                           post_order, site_log_likelihoods, log_likelihood, branch_adjoints,
                           adjoint_frechet_exp, gradient)

__all__ = ["branch_segments", "epoch_P", "homogeneous_P", "transition_matrices", "post_order",
           "site_log_likelihoods", "log_likelihood", "branch_adjoints", "adjoint_frechet_exp",
           "gradient"]
