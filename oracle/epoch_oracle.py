"""FP64 CPU oracle for the epoch-model phylogenetic likelihood.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import this module.  It shares no code
with the GPU library: it takes rate matrices Q (never eigensystems), forms
every transition matrix with a library matrix exponential, and evaluates the
likelihood the slow, plain way in float64.

What it computes, with the passage each step follows (Bielejec et al.,
"Inferring heterogeneous evolutionary processes through time"):

* Transition probabilities over a homogeneous stretch: P = exp(r t Q), rows
  indexed by the earlier state (Methods, Eq. 1 and Eq. 3).
* Change-point (epoch) process: rate matrix Q_phi(m) active in interval m
  between fixed boundaries (Methods, "Relaxing time-homogeneity").  A branch
  that crosses boundaries gets the ordered product of the per-interval
  exponentials, the interval holding the parent first and the one holding the
  child last (Eq. 5-7, Fig. 1).  Reading used for the garbled terms of Eq. 7:
  interior factors span whole intervals, the last factor spans from the last
  boundary crossed down to the child.
* Felsenstein pruning over nodes in post-order (Eq. 4), tips set to 0/1
  indicators with all-ones for missing data, root likelihood sum_i pi_i L(i),
  conditional independence over sites and rate categories (text after Eq. 4).
* Per-(node, pattern) rescaling by the maximum over categories and states,
  log-scales kept in float64 (an addition the paper does not describe; exact
  up to rounding).
* Gradient (an addition): derivative of the same log-likelihood with respect
  to each rate-scaled branch length l_b = r_b * tau_b with the per-interval
  fractions held fixed, and with respect to every entry of every Q_s.  A
  pre-order ("outside") pass gives dlogL/dP_b; the chain rule through the
  ordered product and the exponential uses the Van Loan block-matrix identity
  for the adjoint Frechet derivative of exp.
* Time gradient (an addition; the paper fixes the transition times and names
  estimating them as the next step, Discussion): derivatives with respect to
  every node height and every epoch boundary, branch rates held fixed.  Heights
  and boundaries enter only through the stretch durations of Eq. 7.  At a tie
  (a node exactly on a boundary) the stretch structure changes, and the
  derivative given is the one-sided derivative for an increasing height or
  boundary, which is the side the half-open intervals assign the tie to.

Times are heights (time before the youngest tip); interval k covers heights
[b_k, b_{k+1}) with b_0 = -inf, b_M = +inf, interval 0 the youngest.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import expm

LN2 = float(np.log(2.0))


# ---------------------------------------------------------------------------
# Branch segmentation (Methods, "Relaxing time-homogeneity"; Eq. 7)
# ---------------------------------------------------------------------------


def branch_segments(h_parent, h_child, boundaries, interval_process):
    """Ordered (process, duration) list for a branch, parent side first.

    Walks down in height from the parent to the child; every stretch between
    consecutive boundaries contributes one factor.  Zero-length stretches are
    dropped (exp(0) = I).
    """
    b = [float(x) for x in boundaries]
    edges = [-np.inf] + b + [np.inf]
    segs = []
    for k in range(len(edges) - 2, -1, -1):   # oldest interval first
        lo, hi = edges[k], edges[k + 1]
        top = min(h_parent, hi)
        bot = max(h_child, lo)
        if top > bot:
            segs.append((int(interval_process[k]), top - bot))
    return segs


# ---------------------------------------------------------------------------
# Transition matrices (Eq. 3, Eq. 6, Eq. 7)
# ---------------------------------------------------------------------------


def homogeneous_P(Q, t):
    """P(t) = exp(t Q) (Eq. 3 with the rate scalar folded into t)."""
    return expm(np.asarray(Q, dtype=np.float64) * float(t))


def epoch_P(Qs, segments, scale):
    """Ordered product of per-interval exponentials (Eq. 6 and Eq. 7).

    ``scale`` multiplies every duration (branch rate times category rate).
    """
    K = Qs[0].shape[0]
    P = np.eye(K)
    for s, dt in segments:
        P = P @ homogeneous_P(Qs[s], scale * dt)
    return P


def transition_matrices(prob):
    """P[node][c] for every non-root node (the branch above it)."""
    n_nodes = prob.parent.shape[0]
    K = prob.Q[0].shape[0]
    C = len(prob.cat_rates)
    P = np.zeros((n_nodes, C, K, K))
    for v in range(n_nodes - 1):
        u = prob.parent[v]
        segs = branch_segments(prob.height[u], prob.height[v], prob.boundaries,
                               prob.interval_process)
        for c in range(C):
            P[v, c] = epoch_P(prob.Q, segs, prob.branch_rate[v] * prob.cat_rates[c])
    return P


# ---------------------------------------------------------------------------
# Pruning (Eq. 4) and the root likelihood
# ---------------------------------------------------------------------------


def tip_partials(states, K, ambiguity=None):
    """0/1 indicator vectors [P][K] of the possible states (text after Eq. 4:
    a (partially) observed tip): code < K one state, K every state (missing),
    K + 1 + a the states of ambiguity set a."""
    states = np.asarray(states)
    L = np.zeros((states.shape[0], K))
    for p, st in enumerate(states):
        if st < K:
            L[p, st] = 1.0
        elif st == K:
            L[p, :] = 1.0
        else:
            L[p, :] = np.asarray(ambiguity)[st - K - 1]
    return L


def _children(parent):
    ch = [[] for _ in range(parent.shape[0])]
    for v, u in enumerate(parent):
        if u >= 0:
            ch[u].append(v)
    return ch


def post_order(prob, P=None, rescale=True):
    """Inside partials for every node, per category.

    Returns (partials[node] -> array [C][P][K], logscale[node] -> [P]) where
    the stored partial equals the true one times exp(-logscale).
    """
    if P is None:
        P = transition_matrices(prob)
    n_nodes = prob.parent.shape[0]
    N = prob.n_tips
    K = prob.Q[0].shape[0]
    C = len(prob.cat_rates)
    npat = prob.tips.shape[1]
    ch = _children(prob.parent)
    part = [None] * n_nodes
    logscale = [np.zeros(npat) for _ in range(n_nodes)]
    for t in range(N):
        L = tip_partials(prob.tips[t], K, getattr(prob, "ambiguity", None))
        part[t] = np.broadcast_to(L, (C, npat, K)).copy()
    for u in range(N, n_nodes):      # children have smaller indices
        v, w = ch[u]
        x = np.empty((C, npat, K))
        for c in range(C):
            # sum_j p_ij L_v(j) for every pattern: rows of P index the parent state
            left = part[v][c] @ P[v, c].T
            right = part[w][c] @ P[w, c].T
            x[c] = left * right
        ls = logscale[v] + logscale[w]
        if rescale:
            m = x.max(axis=(0, 2))
            m = np.where(m > 0, m, 1.0)
            x /= m[None, :, None]
            ls = ls + np.log(m)
        part[u] = x
        logscale[u] = ls
    return part, logscale


def site_log_likelihoods(prob, P=None, rescale=True):
    """log L_p per pattern: root sum over pi and categories, plus log-scales."""
    part, logscale = post_order(prob, P, rescale)
    root = prob.parent.shape[0] - 1
    per_cat = part[root] @ prob.pi_root            # [C][P]
    Lp = prob.cat_weights @ per_cat                 # [P]
    return np.log(Lp) + logscale[root]


def log_likelihood(prob, P=None, rescale=True):
    """sum_p w_p log L_p (text after Eq. 4: independent sites aggregate)."""
    return float(np.dot(prob.weights, site_log_likelihoods(prob, P, rescale)))


# ---------------------------------------------------------------------------
# Gradient (not in the paper; exact derivative of the same logL)
# ---------------------------------------------------------------------------


def adjoint_frechet_exp(A, G):
    """L_exp(A)^*[G]: adjoint (Frobenius) of the Frechet derivative of exp at A.

    Van Loan (1978): exp([[X, E], [0, X]]) has L_exp(X)[E] as its top-right
    block, and the adjoint at A equals the derivative at A^T.
    """
    K = A.shape[0]
    M = np.zeros((2 * K, 2 * K))
    M[:K, :K] = A.T
    M[K:, K:] = A.T
    M[:K, K:] = G
    return expm(M)[:K, K:]


def branch_adjoints(prob, P=None):
    """G[v][c] = dlogL/dP_{v,c} (elementwise), from a pre-order pass.

    For the branch above v (parent u, sibling w):
      dL_p/dP_v(i, j) = w_c * qt_v(i) * L_v(j),  qt_v = q_u * (P_w L_w)
    where q_u is the outside vector at u (pi at the root) and L the inside
    partials.  Scale factors of q and L cancel in the ratio with L_p.
    """
    if P is None:
        P = transition_matrices(prob)
    part, logscale = post_order(prob, P, rescale=True)
    n_nodes = prob.parent.shape[0]
    N = prob.n_tips
    K = prob.Q[0].shape[0]
    C = len(prob.cat_rates)
    npat = prob.tips.shape[1]
    ch = _children(prob.parent)
    root = n_nodes - 1
    # outside vectors q[u] [C][P][K], with their own log-scales
    q = [None] * n_nodes
    qscale = [None] * n_nodes
    q[root] = np.broadcast_to(prob.pi_root, (C, npat, K)).copy()
    qscale[root] = np.zeros(npat)
    # full site likelihood (scaled to match each node below)
    per_cat = part[root] @ prob.pi_root
    Lp_root = prob.cat_weights @ per_cat                 # times exp(-logscale[root])
    logLp = np.log(Lp_root) + logscale[root]
    G = np.zeros((n_nodes, C, K, K))
    for u in range(n_nodes - 1, N - 1, -1):             # parents before children
        for v, w in (tuple(ch[u]), tuple(ch[u])[::-1]):
            qt = np.empty((C, npat, K))
            for c in range(C):
                qt[c] = q[u][c] * (part[w][c] @ P[w, c].T)
            # qt * exp(qscale_u + logscale_w) and part[v] * exp(logscale_v) are true values
            log_factor = qscale[u] + logscale[w] + logscale[v] - logLp
            coef = prob.weights * np.exp(log_factor)      # w_p / L_p with scales restored
            for c in range(C):
                G[v, c] += prob.cat_weights[c] * (qt[c] * coef[:, None]).T @ part[v][c]
            if v >= N:
                qv = np.empty((C, npat, K))
                for c in range(C):
                    qv[c] = qt[c] @ P[v, c]              # q_v(j) = sum_i qt(i) p_ij
                m = qv.max(axis=(0, 2))
                m = np.where(m > 0, m, 1.0)
                q[v] = qv / m[None, :, None]
                qscale[v] = qscale[u] + logscale[w] + np.log(m)
    return G


def gradient(prob, wrt=("branch", "Q")):
    """(dlogL/dl_b per child node [2N-1] with root entry 0, dlogL/dQ_s [S][K][K]).

    ``wrt`` selects which of the two to form (the other is returned as zeros).

    l_b = r_b * tau_b; the per-interval fractions of the branch stay fixed, so
    the factor of interval k is exp(rho_c * l_b * f_bk * Q_s).
    """
    P = transition_matrices(prob)
    G = branch_adjoints(prob, P)
    n_nodes = prob.parent.shape[0]
    K = prob.Q[0].shape[0]
    C = len(prob.cat_rates)
    S = len(prob.Q)
    d_branch = np.zeros(n_nodes)
    d_Q = np.zeros((S, K, K))
    for v in range(n_nodes - 1):
        u = prob.parent[v]
        segs = branch_segments(prob.height[u], prob.height[v], prob.boundaries,
                               prob.interval_process)
        tau = prob.height[u] - prob.height[v]
        for c in range(C):
            scale = prob.branch_rate[v] * prob.cat_rates[c]
            F = [homogeneous_P(prob.Q[s], scale * dt) for s, dt in segs]
            m = len(F)
            for k in range(m):
                A = np.eye(K)
                for i in range(k):
                    A = A @ F[i]
                B = np.eye(K)
                for i in range(k + 1, m):
                    B = B @ F[i]
                Gk = A.T @ G[v, c] @ B.T                 # dlogL/dF_k
                s, dt = segs[k]
                # d F_k / d l_b = rho_c * (dt / tau) * Q_s F_k
                dF = prob.cat_rates[c] * (dt / tau) * (prob.Q[s] @ F[k])
                if "branch" in wrt:
                    d_branch[v] += float(np.sum(Gk * dF))
                # d F_k / d Q_s [E] = L_exp(scale*dt*Q_s)[scale*dt*E]
                if "Q" in wrt:
                    d_Q[s] += scale * dt * adjoint_frechet_exp(scale * dt * prob.Q[s], Gk)
    return d_branch, d_Q


# ---------------------------------------------------------------------------
# Time gradient (an addition; Methods, "Relaxing time-homogeneity", Eq. 7)
# ---------------------------------------------------------------------------


def interval_of(h, boundaries):
    """Index of the interval holding height h.  Intervals are half-open,
    [b_{k-1}, b_k), so a height exactly on a boundary belongs to the interval
    above it, and the stretch just above any height h lies in this interval."""
    return int(np.searchsorted(np.asarray(boundaries, dtype=np.float64), h, side="right"))


def time_gradient(prob):
    """(dlogL/dh [2N-1] for every node height, dlogL/db [M-1] for every boundary).

    Branch rates stay fixed.  With G = dlogL/dP from the outside pass and
    x = r_b * rho_c:
    * raising the parent height h_u lengthens the branch at its top by a stretch
      of the interval holding h_u: dP/dh_u = x Q_top P;
    * raising the child height h_v shortens it at its bottom, in the interval
      holding h_v: dP/dh_v = -x P Q_bottom;
    * raising boundary b_m (between interval m below and m + 1 above) moves
      time of every branch spanning it (h_v <= b_m < h_u) from interval m + 1 to
      interval m: with X the product of the factors above b_m and Y of those
      below, dP/db_m = x X (Q_phi(m) - Q_phi(m+1)) Y.
    """
    P = transition_matrices(prob)
    G = branch_adjoints(prob, P)
    n_nodes = prob.parent.shape[0]
    C = len(prob.cat_rates)
    b = np.asarray(prob.boundaries, dtype=np.float64)
    phi = prob.interval_process
    d_h = np.zeros(n_nodes)
    d_b = np.zeros(len(b))
    for v in range(n_nodes):
        u = prob.parent[v]
        if u < 0:
            continue
        hu, hv = prob.height[u], prob.height[v]
        Q_top = prob.Q[phi[interval_of(hu, b)]]
        Q_bot = prob.Q[phi[interval_of(hv, b)]]
        for c in range(C):
            x = prob.branch_rate[v] * prob.cat_rates[c]
            d_h[u] += x * float(np.sum(G[v, c] * (Q_top @ P[v, c])))
            d_h[v] -= x * float(np.sum(G[v, c] * (P[v, c] @ Q_bot)))
            for m, bm in enumerate(b):
                if hv <= bm < hu:
                    X = epoch_P(prob.Q, branch_segments(hu, bm, b, phi), x)
                    Y = epoch_P(prob.Q, branch_segments(bm, hv, b, phi), x)
                    D = prob.Q[phi[m]] - prob.Q[phi[m + 1]]
                    d_b[m] += x * float(np.sum(G[v, c] * (X @ D @ Y)))
    return d_h, d_b
