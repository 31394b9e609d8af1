"""torch.autograd binding of the epoch likelihood.

``EpochLogLikelihood.apply(model, branch_lengths, Q_0, ..., Q_{S-1})`` returns
logL as a 0-d float64 tensor.  The forward pass hands the eigensystems of the
rate matrices (decomposed on the host, as the caller of the library does) and
the branch rates r_v = l_v / tau_v to the library; the backward pass returns
the library's dlogL/dl and dlogL/dQ_s.  Rate matrices built from model
parameters with differentiable torch code (see ``gy94_q``, ``hky_q``,
``gtr_q``) receive gradients for kappa, omega, exchangeabilities, ...
"""
from __future__ import annotations

import functools
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import workloads as W
from .likelihood import EpochLikelihood


class EpochModel:
    """Fixed structure of a likelihood problem: tree heights, epochs, data."""

    def __init__(self, prob: W.Problem, precision: str = "fp64", kernel: str = "auto",
                 reversible_pi: Optional[Sequence[Optional[np.ndarray]]] = None):
        self.prob = prob
        self.lik = EpochLikelihood(prob.n_tips, prob.n_patterns, prob.n_states, len(prob.cat_rates),
                                   prob.n_processes, prob.n_intervals, precision, grad_branch=True,
                                   grad_Q=True, kernel=kernel)
        self.lik.set_tip_states(prob.tips)
        self.lik.set_pattern_weights(prob.weights)
        self.lik.set_categories(prob.cat_rates, prob.cat_weights)
        self.lik.set_root_frequencies(prob.pi_root)
        self.reversible_pi = list(reversible_pi) if reversible_pi is not None else [None] * prob.n_processes
        self.tree_set = False  # the tree is planned once; later forwards only set branch rates
        n = prob.parent.shape[0]
        self.tau = np.zeros(n)
        for v in range(n):
            if prob.parent[v] >= 0:
                self.tau[v] = prob.height[prob.parent[v]] - prob.height[v]
        self.branches = np.nonzero(prob.parent >= 0)[0].astype(np.int32)

    def branch_lengths(self) -> torch.Tensor:
        """l_v = r_v * tau_v of the generated problem (root entry 0)."""
        return torch.tensor(self.prob.branch_rate * self.tau, dtype=torch.float64)

    def close(self):
        self.lik.close()


class EpochLogLikelihood(torch.autograd.Function):
    @staticmethod
    def forward(ctx, model: EpochModel, branch_lengths: torch.Tensor, *Qs: torch.Tensor):
        prob = model.prob
        ell = branch_lengths.detach().cpu().double().numpy()
        rate = np.ones_like(ell)
        mask = model.tau > 0
        rate[mask] = ell[mask] / model.tau[mask]
        if np.any(rate[mask] <= 0):
            raise ValueError("branch lengths must be positive")
        for s, Q in enumerate(Qs):
            model.lik.set_rate_matrix(s, Q.detach().cpu().double().numpy(), model.reversible_pi[s])
        if not model.tree_set:
            model.lik.set_tree(prob.parent, prob.height, rate, prob.boundaries, prob.interval_process)
            model.tree_set = True
        else:
            model.lik.set_branch_rates(model.branches, rate[model.branches])
        # The library instance is shared by every forward on this model, so the gradients of
        # this forward are formed now (one evaluation, one host synchronisation) and kept with
        # its context: a later forward cannot overwrite them before this backward runs.
        want = any(ctx.needs_input_grad[1:])
        logL, _, db, dq = model.lik.evaluate(branch=want, Q=want)
        ctx.grads = (db, dq)
        ctx.n_q = len(Qs)
        ctx.devices = [branch_lengths.device] + [Q.device for Q in Qs]
        return torch.tensor(logL, dtype=torch.float64)

    @staticmethod
    def backward(ctx, grad_out: torch.Tensor):
        db, dq = ctx.grads
        g = float(grad_out)
        grads: List[Optional[torch.Tensor]] = [None]
        grads.append(torch.tensor(g * db, dtype=torch.float64, device=ctx.devices[0]))
        for s in range(ctx.n_q):
            grads.append(torch.tensor(g * dq[s], dtype=torch.float64, device=ctx.devices[1 + s]))
        return tuple(grads)


# ---------------------------------------------------------------------------
# Differentiable rate-matrix builders (torch, float64), normalised so that
# sum_i pi_i q_ii = -1 (Methods, rate normalisation).
# ---------------------------------------------------------------------------


def _normalise(Q: torch.Tensor, pi: torch.Tensor) -> torch.Tensor:
    off = Q - torch.diag(torch.diagonal(Q))
    Q = off - torch.diag(off.sum(dim=1))
    mu = -(pi * torch.diagonal(Q)).sum()
    return Q / mu


def hky_q(kappa: torch.Tensor, pi: torch.Tensor) -> torch.Tensor:
    ts = torch.tensor(W._IS_TRANSITION, dtype=torch.float64)
    R = torch.ones(4, 4, dtype=torch.float64) + ts * (kappa - 1.0)
    return _normalise(R * pi[None, :], pi)


def gtr_q(exch: torch.Tensor, pi: torch.Tensor) -> torch.Tensor:
    iu = torch.triu_indices(4, 4, 1)
    R = torch.zeros(4, 4, dtype=torch.float64)
    R = R.index_put((iu[0], iu[1]), exch)
    R = R + R.T
    return _normalise(R * pi[None, :], pi)


@functools.lru_cache(maxsize=1)
def _gy94_masks():
    """Sense-codon pairs one nucleotide apart, and which of those are transitions and which change
    the amino acid (universal code): fixed by the genetic code, so built once."""
    codons, aas = W.sense_codons()
    K = len(codons)
    single = np.zeros((K, K), bool)
    trans = np.zeros((K, K), bool)
    nonsyn = np.zeros((K, K), bool)
    for i in range(K):
        for j in range(K):
            diff = [p for p in range(3) if codons[i][p] != codons[j][p]]
            if i != j and len(diff) == 1:
                single[i, j] = True
                p = diff[0]
                trans[i, j] = W._IS_TRANSITION[codons[i][p], codons[j][p]]
                nonsyn[i, j] = aas[i] != aas[j]
    return tuple(torch.tensor(m, dtype=torch.float64) for m in (single, trans, nonsyn))


def gy94_q(kappa: torch.Tensor, omega: torch.Tensor, pi_codon: torch.Tensor) -> torch.Tensor:
    S, Tm, Nm = _gy94_masks()
    R = S * (1.0 + Tm * (kappa - 1.0)) * (1.0 + Nm * (omega - 1.0))
    return _normalise(R * pi_codon[None, :], pi_codon)
