"""Pins of the oracle's incremental insertion of a query batch into a merged
graph (Section 4.3, index maintenance): a hand-derived example, the 1-D case
where the RNG prune has a closed form, and the invariants of the result."""
import numpy as np
import pytest

import oracle


def _line(vals):
    return np.asarray(vals, np.float32).reshape(-1, 1)


def test_hand_example_on_a_line():
    # data {0, 10}, one old query at 20, merged rows 0:[1] 1:[0, 2] 2:[1];
    # insert queries at 5 (node 3) and 15 (node 4), R = 2.
    #  node 3: kNN 0 (5), 1 (5), 4 (10), 2 (15); the RNG prune keeps 0 and 1
    #          (d(0, 1) = 10 is not below 5), drops 4 (d(1, 4) = 5 < 10), 2
    #  node 4: keeps 1 and 2 alike
    #  offers: 0 <- 3; 1 <- 3, 4; 2 <- 4
    #  node 0: {1 (10), 3 (5)} fits R -> [3, 1]
    #  node 1: {0 (10), 2 (10), 3 (5), 4 (5)} > R -> prune: 3, 4 kept (d = 10
    #          not below 5), 0 dropped by 3 (5 < 10), 2 dropped by 4
    #  node 2: {1 (10), 4 (5)} -> [4, 1]
    X = _line([0, 10])
    Q_old = _line([20])
    adj = np.array([[1, -1], [0, 2], [1, -1]], np.int32)
    g = oracle.insert_batch(Q_old, X, adj, 0, _line([5, 15]))
    assert g.adj.tolist() == [[3, 1], [3, 4], [4, 1], [0, 1], [1, 2]]
    assert g.repairs == 0 and g.entry == 0
    assert g.elen.tolist() == [[5, 10], [5, 5], [5, 10], [5, 5], [5, 5]]


def test_one_dimensional_closed_form():
    # in 1-D with distinct gaps the RNG prune of the full candidate list keeps
    # exactly the nearest node on each side; with R large every re-pruned row
    # keeps its whole candidate set, so each final row is (old row or the two
    # side neighbours) plus the new nodes that chose it, sorted by distance
    rng = np.random.default_rng(5)
    for trial in range(20):
        n_x, n_q, n_new = rng.integers(2, 9), rng.integers(0, 6), rng.integers(1, 7)
        vals = rng.permutation(np.arange(200, dtype=np.float64))[: n_x + n_q + n_new]
        vals = np.sort(vals)
        vals = vals + np.cumsum(rng.random(vals.size) * 1e-3)   # distinct gaps
        vals = rng.permutation(vals).astype(np.float32)
        n_old = n_x + n_q
        n = n_old + n_new
        R = n - 1
        # old graph: every old row holds every other old node, nearest first
        adj = np.full((n_old, R), -1, np.int32)
        v64 = vals.astype(np.float64)
        for u in range(n_old):
            others = sorted((abs(v64[u] - v64[w]), w) for w in range(n_old) if w != u)
            adj[u, : len(others)] = [w for _, w in others]
        g = oracle.insert_batch(_line(vals[n_x:n_old]), _line(vals[:n_x]), adj, 0,
                                _line(vals[n_old:]), R=R)
        fwd = {}
        for u in range(n_old, n):
            left = [w for w in range(n) if v64[w] < v64[u]]
            right = [w for w in range(n) if v64[w] > v64[u]]
            s = set()
            if left:
                s.add(max(left, key=lambda w: v64[w]))
            if right:
                s.add(min(right, key=lambda w: v64[w]))
            fwd[u] = s
        for v in range(n):
            base = set(adj[v][adj[v] >= 0].tolist()) if v < n_old else set(fwd[v])
            cand = base | {u for u in fwd if v in fwd[u]}
            want = sorted(cand, key=lambda w: (abs(v64[v] - v64[w]), w))
            got = g.adj[v][g.adj[v] >= 0].tolist()
            assert got == want, (trial, v)
        assert g.repairs == 0


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_invariants(seed):
    rng = np.random.default_rng(seed)
    d, R = 6, 6
    X = rng.integers(-8, 9, (120, d)).astype(np.float32)
    Q = rng.integers(-8, 9, (60, d)).astype(np.float32)
    Qn = rng.integers(-8, 9, (40, d)).astype(np.float32)
    base = oracle.build_merged(Q, X, R)
    g = oracle.insert_batch(Q, X, base.adj.copy(), base.entry, Qn)
    V = np.concatenate([X, Q, Qn]).astype(np.float64)
    n_old, n = 180, 220
    assert g.adj.shape == (n, R) and g.entry == base.entry
    # every node is reached from the entry (the repair's guarantee)
    seen = np.zeros(n, bool)
    stack = [g.entry]
    seen[g.entry] = True
    while stack:
        u = stack.pop()
        for v in g.adj[u]:
            if v >= 0 and not seen[v]:
                seen[v] = True
                stack.append(v)
    assert seen.all()
    offered = set()
    for u in range(n):
        row = g.adj[u]
        k = int((row >= 0).sum())
        assert (row[:k] >= 0).all() and (row[k:] == -1).all()
        assert u not in row[:k] and len(set(row[:k].tolist())) == k
        dd = np.linalg.norm(V[row[:k]] - V[u], axis=1)
        np.testing.assert_allclose(g.elen[u, :k], dd, rtol=1e-15)
        if u >= n_old:
            offered.update(row[:k].tolist())
    # an old row that was offered nothing, and was given no repair edge,
    # is unchanged
    if g.repairs == 0:
        for u in range(n_old):
            if u not in offered:
                assert (g.adj[u] == base.adj[u]).all()


def test_empty_batch_keeps_the_graph():
    rng = np.random.default_rng(3)
    X = rng.integers(-5, 6, (50, 4)).astype(np.float32)
    Q = rng.integers(-5, 6, (20, 4)).astype(np.float32)
    base = oracle.build_merged(Q, X, 5)
    g = oracle.insert_batch(Q, X, base.adj.copy(), base.entry, np.zeros((0, 4), np.float32))
    assert (g.adj == base.adj).all() and g.repairs == 0
