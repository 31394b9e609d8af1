"""The 4-state tree-walk programs from the library's host planner (no GPU).

A small interpreter runs the two programs in FP64 over every pattern at once,
with the oracle's transition matrices, and checks what they compute against
the oracle: the post-order program must give the log-likelihood, and the
pre-order program's per-branch outer products must add up to the oracle's
dlogL/dP.  The interpreter also checks the stack discipline: every slot read
holds the vector the operation expects, no slot index reaches the reported
slot count, and every partial read from memory was stored by the post-order
program.
"""
import numpy as np
import pytest

from oracle import epoch_oracle as O
from paper_1309_3075_amd import _abi
from paper_1309_3075_amd import workloads as W

PRE, ROOT, STORE = 1, 2, 4
TIP, HBM, STACK = 0, 1, 2


def decode(info):
    info = int(info) & 0xFFFFFFFF
    return dict(pre=bool(info & PRE), root=bool(info & ROOT), store=bool(info & STORE),
                ka=(info >> 3) & 3, kb=(info >> 5) & 3, s_a=(info >> 8) & 63, s_b=(info >> 14) & 63,
                s_q=(info >> 20) & 63, s_qb=(info >> 26) & 63)


def normalise(x):
    m = x.max(axis=(0, 2))
    e = np.where(m > 0, np.frexp(np.where(m > 0, m, 1.0))[1], 0)
    return x * np.exp2(-e)[None, :, None], e


def run_programs(prob, recompute_tips):
    post, pre, post_slots, pre_slots = _abi.plan_walk(prob.parent, prob.height, recompute_tips)
    P = O.transition_matrices(prob)
    N, K, C = prob.n_tips, prob.Q[0].shape[0], len(prob.cat_rates)
    npat = prob.tips.shape[1]
    n_nodes = prob.parent.shape[0]
    root = n_nodes - 1
    wc = np.asarray(prob.cat_weights)

    def tip_vec(v):
        return np.broadcast_to(O.tip_partials(prob.tips[v], K), (C, npat, K))

    def apply(M, x):  # [C][K][K] x [C][P][K] -> [C][P][K]
        return np.einsum("cij,cpj->cpi", M, x)

    # post-order program
    stack, owner, stored = {}, {}, {}
    E = np.zeros(npat)
    logL = None
    assert post.shape[0] == N - 1
    for info, a, b, u in post:
        d = decode(info)
        assert not d["pre"]
        xs = []
        for k, s, v in ((d["ka"], d["s_a"], a), (d["kb"], d["s_b"], b)):
            if k == TIP:
                assert v < N
                xs.append(tip_vec(v))
            else:
                assert k == STACK and s < post_slots and owner.get(s) == ("x", v)
                xs.append(stack[s])
                owner.pop(s)
        y, e = normalise(apply(P[a], xs[0]) * apply(P[b], xs[1]))
        E += e
        if d["store"]:
            stored[u] = y
        if d["root"]:
            assert u == root and d["store"] and d["s_q"] == post_slots  # discarded output
            Lp = wc @ (y @ prob.pi_root)
            logL = float(np.dot(prob.weights, np.log(Lp) + E * np.log(2.0)))
        else:
            assert d["s_q"] < post_slots
            stack[d["s_q"]] = y
            owner[d["s_q"]] = ("x", u)
    assert logL is not None

    # pre-order program
    stack, owner = {}, {}
    G = np.zeros((n_nodes, C, K, K))
    visited = set()
    for info, a, b, u in pre:
        d = decode(info)
        if not d["pre"]:  # recomputation of a subtree that is not stored
            assert not d["store"] and not d["root"]
            xs = []
            for k, s, v in ((d["ka"], d["s_a"], a), (d["kb"], d["s_b"], b)):
                if k == TIP:
                    xs.append(tip_vec(v))
                else:
                    assert k == STACK and s < pre_slots and owner.get(s) == ("x", v)
                    xs.append(stack[s])
                    owner.pop(s)
            y, _ = normalise(apply(P[a], xs[0]) * apply(P[b], xs[1]))
            assert d["s_q"] < pre_slots and d["s_q"] not in owner
            stack[d["s_q"]] = y
            owner[d["s_q"]] = ("x", u)
            continue
        assert u not in visited
        visited.add(u)
        if d["root"]:
            assert u == root
            q = np.broadcast_to(prob.pi_root, (C, npat, K))
        else:
            assert owner.get(d["s_q"]) == ("q", u)
            q = stack[d["s_q"]]
            owner.pop(d["s_q"])
        xs = []
        for k, s, v in ((d["ka"], d["s_a"], a), (d["kb"], d["s_b"], b)):
            if k == TIP:
                assert v < N
                xs.append(tip_vec(v))
            elif k == HBM:
                assert v in stored
                xs.append(stored[v])
            else:
                assert k == STACK and s < pre_slots and owner.get(s) == ("x", v)
                xs.append(stack[s])
                owner.pop(s)
        Sa, Sb = apply(P[a], xs[0]), apply(P[b], xs[1])
        lp = np.einsum("c,cpi->p", wc, q * Sa * Sb)
        f = (prob.weights / lp)[None, :] * wc[:, None]  # [C][P]
        ta, tb = q * Sb, q * Sa
        G[a] += np.einsum("cp,cpi,cpj->cij", f, ta, xs[0])
        G[b] += np.einsum("cp,cpi,cpj->cij", f, tb, xs[1])
        for k, v, t, slot in ((d["ka"], a, ta, d["s_q"]), (d["kb"], b, tb, d["s_qb"])):
            if k != TIP:
                qv, _ = normalise(np.einsum("cij,cpi->cpj", P[v], t))
                assert slot < pre_slots and slot not in owner
                stack[slot] = qv
                owner[slot] = ("q", v)
            elif slot != pre_slots:  # else the discard slot
                assert slot == d["s_q"] and not d["root"]  # q_u's slot, consumed by this operation
    assert visited == set(range(N, n_nodes))
    assert not owner
    return logL, G, post_slots, pre_slots, stored


def _check(prob, recompute_tips):
    logL, G, ps, qs, stored = run_programs(prob, recompute_tips)
    want = O.log_likelihood(prob)
    assert abs(logL - want) <= 1e-12 * abs(want)
    G_ref = O.branch_adjoints(prob)
    assert np.linalg.norm(G - G_ref) <= 1e-10 * np.linalg.norm(G_ref)
    return ps, qs, stored


@pytest.mark.parametrize("N", [2, 3, 5, 9, 33])
@pytest.mark.parametrize("recompute", [2, 3, 5])
def test_walk_programs_match_oracle(N, recompute):
    rng = np.random.default_rng(4000 + 10 * N + recompute)
    prob = W.random_problem(rng, N, 4, 12, n_categories=3, n_intervals=3, reversible=False,
                            missing_frac=0.1)
    _check(prob, recompute)


def _tree_problem(parent, rng, npat=7):
    n = len(parent)
    N = (n + 1) // 2
    prob = W.random_problem(rng, N, 4, npat, n_categories=2, n_intervals=2)
    # heights: one more than the deepest child
    height = np.zeros(n)
    for u in range(N, n):
        ch = [v for v in range(n) if parent[v] == u]
        height[u] = 1.0 + max(height[v] for v in ch)
    import dataclasses
    return dataclasses.replace(prob, parent=np.asarray(parent, np.int32), height=height / height[-1])


def caterpillar(N):
    parent = [-1] * (2 * N - 1)
    parent[0] = parent[1] = N
    for k in range(2, N):
        parent[k] = N + k - 1
        parent[N + k - 2] = N + k - 1
    return parent


def balanced(N):
    parent = [-1] * (2 * N - 1)
    level = list(range(N))
    nxt = N
    while len(level) > 1:
        new = []
        for i in range(0, len(level), 2):
            parent[level[i]] = nxt
            parent[level[i + 1]] = nxt
            new.append(nxt)
            nxt += 1
        level = new
    return parent


def test_caterpillar_needs_two_slots():
    rng = np.random.default_rng(4100)
    prob = _tree_problem(caterpillar(12), rng)
    ps, qs, stored = _check(prob, 2)
    assert ps <= 2 and qs <= 3


def test_balanced_tree_slots_grow_like_log2():
    rng = np.random.default_rng(4101)
    prob = _tree_problem(balanced(32), rng)
    ps, qs, stored = _check(prob, 2)
    assert ps <= 6 and qs <= 7
    # recompute everything below the root's children: only they and the root are stored
    ps, qs, stored = _check(prob, 15)
    assert sorted(stored) == sorted([62, 60, 61])


def test_stored_set_is_the_non_cherries():
    rng = np.random.default_rng(4102)
    prob = W.random_problem(rng, 40, 4, 3)
    post, pre, _, _ = _abi.plan_walk(prob.parent, prob.height, 2)
    N = prob.n_tips
    kids = {}
    for v, u in enumerate(prob.parent):
        kids.setdefault(int(u), []).append(v)
    cherries = {u for u, ch in kids.items() if u >= 0 and all(v < N for v in ch)}
    stored = {int(u) for info, a, b, u in post if int(info) & STORE}
    assert stored == set(range(N, 2 * N - 1)) - cherries | {2 * N - 2}


def test_plan_walk_rejects_bad_arguments():
    rng = np.random.default_rng(4103)
    prob = W.random_problem(rng, 6, 4, 3)
    with pytest.raises(Exception):
        _abi.plan_walk(prob.parent, prob.height, 1)
