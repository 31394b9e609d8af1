"""Seeded synthetic inputs for the epoch-model likelihood.

This module builds inputs only: trees, rate matrices, among-site rate
categories, tip states and pattern weights.  It holds none of the likelihood
arithmetic (no matrix exponentials, no pruning): sequences are simulated with
a jump-by-jump (Gillespie) walk of the continuous-time Markov chain, switching
rate matrix whenever the walk crosses an epoch boundary, which is the
generative process of the change-point model (Methods, "Relaxing
time-homogeneity").  Both the GPU path and the FP64 oracle consume what it
returns.

Conventions (shared by the library ABI):
  * Node indices: tips 0..N-1, internal nodes N..2N-2 in order of creation,
    root = 2N-2.  Every parent index is larger than its children's, so
    increasing index order is a valid post-order.
  * Times are heights (time before the youngest tip).  Epoch interval k covers
    heights [b_k, b_{k+1}) with b_0 = -inf and b_M = +inf; interval 0 is the
    youngest.  ``interval_process[k]`` names the rate matrix active there.
  * Rate matrices are row-major, rows index the earlier (parent-side) state.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np
from scipy import special, stats

SEED_BASE = 13093075

# ---------------------------------------------------------------------------
# Trees
# ---------------------------------------------------------------------------


def coalescent_tree(n_tips: int, rng: np.random.Generator, root_height: float = 1.0,
                    tip_heights: Optional[np.ndarray] = None):
    """Kingman coalescent tree (heterochronous when ``tip_heights`` is given).

    Returns (parent[2N-1] int32 with -1 at the root, height[2N-1] float64).
    Heights are rescaled so that the root sits at ``root_height``.
    """
    n = int(n_tips)
    if n < 2:
        raise ValueError("need at least 2 tips")
    if tip_heights is None:
        tip_heights = np.zeros(n)
    tip_heights = np.asarray(tip_heights, dtype=np.float64)
    order = np.argsort(tip_heights, kind="stable")
    parent = np.full(2 * n - 1, -1, dtype=np.int32)
    height = np.zeros(2 * n - 1, dtype=np.float64)
    height[:n] = tip_heights
    active: List[int] = []
    next_tip = 0
    t = 0.0
    # enter all tips sampled at (or before) time zero
    while next_tip < n and tip_heights[order[next_tip]] <= t:
        active.append(int(order[next_tip]))
        next_tip += 1
    new_node = n
    while new_node < 2 * n - 1:
        k = len(active)
        rate = k * (k - 1) / 2.0
        wait = rng.exponential(1.0 / rate) if k >= 2 else math.inf
        if next_tip < n and tip_heights[order[next_tip]] <= t + wait:
            t = float(tip_heights[order[next_tip]])
            active.append(int(order[next_tip]))
            next_tip += 1
            continue
        t += wait
        i, j = rng.choice(k, size=2, replace=False)
        a, b = active[i], active[j]
        for idx in sorted((i, j), reverse=True):
            active.pop(idx)
        parent[a] = new_node
        parent[b] = new_node
        height[new_node] = t
        active.append(new_node)
        new_node += 1
    scale = root_height / height[2 * n - 2]
    height *= scale
    return parent, height


# ---------------------------------------------------------------------------
# Rate matrices
# ---------------------------------------------------------------------------

NUC = "ACGT"
# transitions are A<->G and C<->T
_IS_TRANSITION = np.zeros((4, 4), dtype=bool)
for _a, _b in ((0, 2), (2, 0), (1, 3), (3, 1)):
    _IS_TRANSITION[_a, _b] = True


def _normalise_reversible(Q: np.ndarray, pi: np.ndarray) -> np.ndarray:
    np.fill_diagonal(Q, 0.0)
    np.fill_diagonal(Q, -Q.sum(axis=1))
    mu = -float(np.dot(pi, np.diag(Q)))
    return Q / mu


def hky(kappa: float, pi: Sequence[float]) -> np.ndarray:
    """HKY85 rate matrix with sum_i pi_i q_ii = -1 (Methods, rate normalisation)."""
    pi = np.asarray(pi, dtype=np.float64)
    Q = np.tile(pi, (4, 1))
    Q[_IS_TRANSITION] *= kappa
    return _normalise_reversible(Q, pi)


def gtr(exch: Sequence[float], pi: Sequence[float]) -> np.ndarray:
    """GTR rate matrix; ``exch`` holds (AC, AG, AT, CG, CT, GT)."""
    pi = np.asarray(pi, dtype=np.float64)
    R = np.zeros((4, 4))
    iu = np.triu_indices(4, 1)
    R[iu] = np.asarray(exch, dtype=np.float64)
    R = R + R.T
    Q = R * pi[None, :]
    return _normalise_reversible(Q, pi)


# Standard genetic code, bases in T,C,A,G order at each position.
_CODE_TCAG = "FFLLSSSSYY**CC*WLLLLPPPPHHQQRRRRIIIMTTTTNNKKSSRRVVVVAAAADDEEGGGG"
_TCAG_TO_ACGT = {"T": 3, "C": 1, "A": 0, "G": 2}


def _genetic_code_acgt():
    aa = {}
    bases = "TCAG"
    for i, b1 in enumerate(bases):
        for j, b2 in enumerate(bases):
            for k, b3 in enumerate(bases):
                key = (_TCAG_TO_ACGT[b1], _TCAG_TO_ACGT[b2], _TCAG_TO_ACGT[b3])
                aa[key] = _CODE_TCAG[16 * i + 4 * j + k]
    return aa


def sense_codons():
    """The 61 sense codons as (n1, n2, n3) in ACGT order, and their amino acids."""
    code = _genetic_code_acgt()
    codons, aas = [], []
    for n1 in range(4):
        for n2 in range(4):
            for n3 in range(4):
                a = code[(n1, n2, n3)]
                if a != "*":
                    codons.append((n1, n2, n3))
                    aas.append(a)
    return codons, aas


def f3x4_frequencies(pos_freqs: np.ndarray) -> np.ndarray:
    """Codon frequencies from per-position nucleotide frequencies [3][4]."""
    codons, _ = sense_codons()
    f = np.array([pos_freqs[0, a] * pos_freqs[1, b] * pos_freqs[2, c] for a, b, c in codons])
    return f / f.sum()


def gy94(kappa: float, omega: float, pi_codon: np.ndarray) -> np.ndarray:
    """Goldman-Yang 1994 codon rate matrix over the 61 sense codons.

    q_ij = 0 when codons differ at more than one position; otherwise
    pi_j * (kappa if the change is a transition) * (omega if non-synonymous).
    """
    codons, aas = sense_codons()
    K = len(codons)
    Q = np.zeros((K, K))
    for i in range(K):
        for j in range(K):
            if i == j:
                continue
            diff = [p for p in range(3) if codons[i][p] != codons[j][p]]
            if len(diff) != 1:
                continue
            p = diff[0]
            r = pi_codon[j]
            if _IS_TRANSITION[codons[i][p], codons[j][p]]:
                r *= kappa
            if aas[i] != aas[j]:
                r *= omega
            Q[i, j] = r
    return _normalise_reversible(Q, pi_codon)


def sparse_asymmetric(K: int, density: float, rng: np.random.Generator) -> np.ndarray:
    """Asymmetric CTMC with ~``density`` nonzero lognormal(0,1) off-diagonal rates.

    Normalised so the mean exit rate over states is 1 (-(1/K) sum_i q_ii = 1),
    which does not need a unique stationary distribution.
    """
    mask = rng.random((K, K)) < density
    np.fill_diagonal(mask, False)
    rates = np.exp(rng.normal(0.0, 1.0, size=(K, K)))
    Q = np.where(mask, rates, 0.0)
    np.fill_diagonal(Q, -Q.sum(axis=1))
    return Q / (-np.trace(Q) / K)


def discrete_gamma(alpha: float, n_cat: int):
    """Discrete-gamma among-site rates (mean of each equal-probability category).

    Returns (rates[C], weights[C]) with mean rate 1.
    """
    if n_cat == 1:
        return np.ones(1), np.ones(1)
    q = stats.gamma.ppf(np.arange(1, n_cat) / n_cat, a=alpha, scale=1.0 / alpha)
    edges = np.concatenate([[0.0], q * alpha, [np.inf]])
    upper = special.gammainc(alpha + 1.0, edges)
    rates = np.diff(upper) * n_cat
    return rates, np.full(n_cat, 1.0 / n_cat)


# ---------------------------------------------------------------------------
# Simulation (Gillespie walk of the change-point CTMC)
# ---------------------------------------------------------------------------


def _walk(states, remaining, Q, rng):
    """Advance each site's CTMC state by ``remaining`` time units under Q."""
    K = Q.shape[0]
    exit_rate = -np.diag(Q)
    jump = np.where(np.eye(K, dtype=bool), 0.0, Q)
    with np.errstate(invalid="ignore", divide="ignore"):
        jump = jump / exit_rate[:, None]
    jump = np.nan_to_num(jump)
    cum = np.cumsum(jump, axis=1)
    idx = np.arange(states.shape[0])
    rem = remaining.copy()
    while idx.size:
        x = states[idx]
        rate = exit_rate[x]
        with np.errstate(divide="ignore"):
            wait = rng.exponential(1.0, size=idx.size) / rate
        go = wait < rem[idx]
        idx = idx[go]
        if not idx.size:
            break
        rem[idx] -= wait[go]
        u = rng.random(idx.size)
        new = (cum[states[idx]] < u[:, None]).sum(axis=1)
        states[idx] = np.minimum(new, K - 1)
    return states


def simulate_sites(parent, height, branch_rate, boundaries, interval_process, Qs, pi_root,
                   cat_rates, cat_weights, n_sites, rng):
    """Simulate ``n_sites`` independent sites down the tree; returns tips [N][n_sites]."""
    n_nodes = parent.shape[0]
    n_tips = (n_nodes + 1) // 2
    K = Qs[0].shape[0]
    states = np.zeros((n_nodes, n_sites), dtype=np.int32)
    root = n_nodes - 1
    states[root] = rng.choice(K, size=n_sites, p=pi_root / pi_root.sum())
    cat = rng.choice(len(cat_rates), size=n_sites, p=cat_weights)
    site_rate = np.asarray(cat_rates)[cat]
    b = np.asarray(boundaries, dtype=np.float64)
    for v in range(n_nodes - 2, -1, -1):  # parents have larger indices
        u = parent[v]
        x = states[u].copy()
        h = height[u]
        while h > height[v]:
            # interval holding the stretch just below height h: count of boundaries < h
            k = int(np.searchsorted(b, h, side="left"))
            lo = b[k - 1] if k > 0 else -np.inf
            h_next = max(lo, height[v])
            dt = (h - h_next) * branch_rate[v]
            if dt > 0:
                x = _walk(x, dt * site_rate, Qs[interval_process[k]], rng)
            h = h_next
        states[v] = x
    return states[:n_tips]


def unique_patterns(sites: np.ndarray):
    """Unique site columns in order of first appearance, with their counts."""
    cols = np.ascontiguousarray(sites.T)
    _, first, inverse, counts = np.unique(cols, axis=0, return_index=True,
                                          return_inverse=True, return_counts=True)
    order = np.argsort(first)
    return cols[first[order]].T.copy(), counts[order].astype(np.float64)


# ---------------------------------------------------------------------------
# Problems
# ---------------------------------------------------------------------------


@dataclasses.dataclass
class Problem:
    """One likelihood problem: tree, epoch model, categories and data."""
    name: str
    parent: np.ndarray          # [2N-1] int32, -1 at root
    height: np.ndarray          # [2N-1] float64
    branch_rate: np.ndarray     # [2N-1] float64 (rate of the branch above each node)
    boundaries: np.ndarray      # [M-1] ascending heights
    interval_process: np.ndarray  # [M] int32
    Q: List[np.ndarray]         # S rate matrices [K][K]
    pi_process: List[Optional[np.ndarray]]  # stationary distribution per process (reversible) or None
    pi_root: np.ndarray         # [K]
    cat_rates: np.ndarray       # [C]
    cat_weights: np.ndarray     # [C]
    tips: np.ndarray            # [N][P] int32, value K = missing, K + 1 + a = ambiguity set a
    weights: np.ndarray         # [P] float64
    seed: int = 0
    ambiguity: Optional[np.ndarray] = None  # [A][K] 0/1 state sets of the tip codes K + 1 + a

    @property
    def n_tips(self):
        return (self.parent.shape[0] + 1) // 2

    @property
    def n_states(self):
        return self.Q[0].shape[0]

    @property
    def n_patterns(self):
        return self.tips.shape[1]

    @property
    def n_processes(self):
        return len(self.Q)

    @property
    def n_intervals(self):
        return len(self.interval_process)


def simulate_patterns(tree, boundaries, phi, Qs, pi_root, cat_rates, cat_weights, n_patterns,
                      rng, weights_mode="counts", max_rounds=64):
    parent, height = tree
    rate = np.ones(parent.shape[0])
    pats, counts = None, None
    batch = max(n_patterns, 64)
    seen = {}
    order = []
    for _ in range(max_rounds):
        sites = simulate_sites(parent, height, rate, boundaries, phi, Qs, pi_root,
                               cat_rates, cat_weights, batch, rng)
        cols = np.ascontiguousarray(sites.T.astype(np.uint8 if Qs[0].shape[0] < 256 else np.int32))
        for c in cols:
            key = c.tobytes()
            if key in seen:
                seen[key][1] += 1
            else:
                seen[key] = [c, 1]
                order.append(key)
        if len(order) >= n_patterns:
            break
    if len(order) < n_patterns:
        raise RuntimeError("could not simulate enough unique patterns")
    keep = order[:n_patterns]
    pats = np.stack([seen[k][0] for k in keep], axis=1).astype(np.int32)
    counts = np.array([seen[k][1] for k in keep], dtype=np.float64)
    if weights_mode == "counts":
        w = counts
    else:
        w = rng.integers(1, 6, size=n_patterns).astype(np.float64)
    return pats, w


def _dirichlet(rng, alpha, k):
    return rng.dirichlet(np.full(k, float(alpha)))


def make_config(index: int, replicate: int = 0, *, n_tips=None, n_patterns=None,
                tip_height_max: float = 0.0) -> Problem:
    """The five workloads (index 1..5 as C1..C5) and a 20-state variant (index 6), optionally
    shrunk for tests.

    C5 returns one problem per call; use :func:`make_batch` for the batch.
    """
    seed = SEED_BASE + 100 * index + replicate
    rng = np.random.default_rng(seed)
    if index == 1:
        N = n_tips or 16
        P = n_patterns or 1000
        pi = _dirichlet(rng, 5.0, 4)
        Qs = [hky(2.0, pi), hky(8.0, pi)]
        pis = [pi, pi]
        bounds = np.array([0.5])
        phi = np.array([0, 1], dtype=np.int32)
        rates, wts = discrete_gamma(0.5, 4)
        pi_root = pi
        weights_mode = "uniform15"
    elif index == 2:
        N = n_tips or 512
        P = n_patterns or 100_000
        Qs, pis = [], []
        for _ in range(3):
            ex = _dirichlet(rng, 1.0, 6)
            pi = _dirichlet(rng, 1.0, 4)
            Qs.append(gtr(ex, pi))
            pis.append(pi)
        bounds = np.array([1.0 / 3.0, 2.0 / 3.0])
        phi = np.array([0, 1, 2], dtype=np.int32)
        rates, wts = discrete_gamma(0.5, 4)
        pi_root = pis[-1]
        weights_mode = "counts"
    elif index in (3, 5):
        if index == 5:
            N = n_tips or int(rng.integers(64, 257))
            P = n_patterns or int(rng.integers(1000, 20001))
        else:
            N = n_tips or 128
            P = n_patterns or 10_000
        pos = np.stack([_dirichlet(rng, 10.0, 4) for _ in range(3)])
        pic = f3x4_frequencies(pos)
        omegas = [0.2, 1.0, 2.5, 0.5]
        Qs = [gy94(3.0, w, pic) for w in omegas]
        pis = [pic] * 4
        bounds = np.array([0.25, 0.5, 0.75])
        phi = np.array([0, 1, 2, 3], dtype=np.int32)
        rates, wts = np.ones(1), np.ones(1)
        pi_root = pic
        weights_mode = "counts"
    elif index == 6:
        # 20-state (amino-acid-sized) variant of the codon workload: random reversible
        # rates per epoch (exchangeabilities Dir(1), frequencies Dir(5)), 4 epochs, 128 taxa
        N = n_tips or 128
        P = n_patterns or 10_000
        Qs, pis = [], []
        for _ in range(4):
            pi = _dirichlet(rng, 5.0, 20)
            R = rng.dirichlet(np.ones(190))
            Rm = np.zeros((20, 20))
            Rm[np.triu_indices(20, 1)] = R
            Rm = Rm + Rm.T
            Qs.append(_normalise_reversible(Rm * pi[None, :], pi))
            pis.append(pi)
        bounds = np.array([0.25, 0.5, 0.75])
        phi = np.array([0, 1, 2, 3], dtype=np.int32)
        rates, wts = np.ones(1), np.ones(1)
        pi_root = pis[-1]
        weights_mode = "counts"
    elif index == 4:
        N = n_tips or 2000
        P = n_patterns or 1
        K = 40
        Qs = [sparse_asymmetric(K, 0.2, rng) for _ in range(12)]
        pis = [None] * 12
        M = 48
        bounds = np.arange(1, M) / M
        phi = (np.arange(M) % 12).astype(np.int32)
        rates, wts = np.ones(1), np.ones(1)
        pi_root = np.full(K, 1.0 / K)
        weights_mode = None
    else:
        raise ValueError(index)

    tip_h = None
    if tip_height_max > 0:
        tip_h = rng.uniform(0.0, tip_height_max, size=N)
    parent, height = coalescent_tree(N, rng, 1.0, tip_h)
    K = Qs[0].shape[0]
    if weights_mode is None:
        tips = rng.integers(0, K, size=(N, P)).astype(np.int32)
        weights = np.ones(P)
    else:
        tips, weights = simulate_patterns((parent, height), bounds, phi, Qs, pi_root, rates, wts,
                                          P, rng, weights_mode)
    return Problem(name=f"C{index}", parent=parent, height=height,
                   branch_rate=np.ones(parent.shape[0]), boundaries=bounds,
                   interval_process=phi, Q=Qs, pi_process=pis, pi_root=pi_root,
                   cat_rates=np.asarray(rates, dtype=np.float64),
                   cat_weights=np.asarray(wts, dtype=np.float64), tips=tips,
                   weights=weights, seed=seed)


def make_batch(n_problems: int = 64, replicate: int = 0, scale: float = 1.0) -> List[Problem]:
    """The batched codon workload: independent C3-type problems of uneven size."""
    rng = np.random.default_rng(SEED_BASE + 500 + replicate)
    out = []
    for i in range(n_problems):
        N = int(rng.integers(64, 257))
        P = int(rng.integers(1000, 20001))
        if scale != 1.0:
            N = max(4, int(N * scale))
            P = max(8, int(P * scale))
        out.append(make_config(5, replicate=1000 * replicate + i + 1, n_tips=N, n_patterns=P))
    return out


def random_problem(rng: np.random.Generator, n_tips: int, n_states: int, n_patterns: int,
                   n_categories: int = 1, n_intervals: int = 2, n_processes: Optional[int] = None,
                   reversible: bool = True, tip_height_max: float = 0.0, missing_frac: float = 0.0,
                   branch_rate_spread: float = 0.0, root_height: float = 1.0,
                   ambiguous_frac: float = 0.0, n_ambiguity_sets: int = 3) -> Problem:
    """Small random problem for tests: random Q's, random (not simulated) tip states."""
    K = n_states
    S = n_processes or n_intervals
    Qs, pis = [], []
    for _ in range(S):
        if reversible:
            pi = _dirichlet(rng, 2.0, K)
            R = rng.exponential(1.0, size=(K, K))
            R = (R + R.T) / 2
            Q = R * pi[None, :]
            Qs.append(_normalise_reversible(Q, pi))
            pis.append(pi)
        else:
            Qs.append(sparse_asymmetric(K, 0.6, rng))
            pis.append(None)
    tip_h = rng.uniform(0, tip_height_max, size=n_tips) if tip_height_max > 0 else None
    parent, height = coalescent_tree(n_tips, rng, root_height, tip_h)
    bounds = np.sort(rng.uniform(0.05, 0.95, size=n_intervals - 1)) * root_height
    phi = rng.integers(0, S, size=n_intervals).astype(np.int32)
    if n_categories > 1:
        rates, wts = discrete_gamma(0.7, n_categories)
    else:
        rates, wts = np.ones(1), np.ones(1)
    tips = rng.integers(0, K, size=(n_tips, n_patterns)).astype(np.int32)
    if missing_frac > 0:
        tips[rng.random(tips.shape) < missing_frac] = K
    amb = None
    if ambiguous_frac > 0:
        # partially observed tips: random state sets of 2 .. K-1 states (K >= 3), codes K + 1 + a
        amb = np.zeros((n_ambiguity_sets, K), dtype=np.int32)
        for a in range(n_ambiguity_sets):
            size = int(rng.integers(2, max(3, K)))
            amb[a, rng.choice(K, size=min(size, K), replace=False)] = 1
        sel = rng.random(tips.shape) < ambiguous_frac
        tips[sel] = K + 1 + rng.integers(0, n_ambiguity_sets, size=int(sel.sum()))
    weights = rng.integers(1, 6, size=n_patterns).astype(np.float64)
    br = np.exp(rng.normal(0.0, branch_rate_spread, size=parent.shape[0])) if branch_rate_spread else np.ones(parent.shape[0])
    pi_root = _dirichlet(rng, 3.0, K)
    return Problem(name="random", parent=parent, height=height, branch_rate=br,
                   boundaries=bounds, interval_process=phi, Q=Qs, pi_process=pis,
                   pi_root=pi_root, cat_rates=np.asarray(rates, float),
                   cat_weights=np.asarray(wts, float), tips=tips, weights=weights, ambiguity=amb)
