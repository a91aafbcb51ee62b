"""Pins of the oracle's HNSW-style upper layers (the paper's index-type
experiment, Section 5): SplitMix64 levels, the greedy descent and the join
seeded by it.  CPU only."""
from collections import deque

import numpy as np
import pytest

import oracle
import workloads


def test_splitmix64_published_vectors():
    # the first outputs of SplitMix64 seeded with 1234567, as published with
    # the generator's reference code
    want = [6457827717110365317, 3203168211198807973, 9817491932198370423,
            4593380528125082431, 16408922859458223821]
    assert [oracle.splitmix64(1234567, k) for k in range(1, 6)] == want


def test_levels_digit_rule():
    # level = trailing zero 4-bit digits of the output, capped
    n = 1 << 20
    lvl = oracle.levels(n, 7, max_levels=8)
    for v in range(0, n, 9973):
        z, l = oracle.splitmix64(7, v + 1), 0
        while l < 8 and z % 16 == 0:
            z //= 16
            l += 1
        assert lvl[v] == l
    # P(level >= l) = 16^-l: within 5 standard deviations for l = 1, 2
    for l in (1, 2):
        p = 16.0 ** -l
        c = int((lvl >= l).sum())
        assert abs(c - n * p) < 5 * np.sqrt(n * p * (1 - p)), (l, c)
    assert lvl.max() <= 8
    assert np.array_equal(oracle.levels(n, 7, max_levels=1), np.minimum(lvl, 1))


def _line_layers():
    """Data on a line at 0, 1, ..., 15 (d = 2, second coordinate 0).  Layer 2
    = {0, 8} (one edge), layer 1 = {0, 4, 8, 12} as a chain 0-4-8-12."""
    X = np.zeros((16, 2), np.float32)
    X[:, 0] = np.arange(16)
    L = oracle.Layers(lvl=np.zeros(16, np.int8),
                      ids=[np.array([0, 4, 8, 12], np.int32), np.array([0, 8], np.int32)],
                      adj=[np.array([[4, -1], [0, 8], [4, 12], [8, -1]], np.int32),
                           np.array([[8, -1], [0, -1]], np.int32)],
                      entry=[0, 0])
    return X, L


def test_descent_hand_example():
    X, L = _line_layers()
    Q = np.array([[9.6, 0], [13.0, 0], [1.0, 0], [6.0, 0]], np.float32)
    seed, moves = oracle.descend(Q, X, L)
    # 9.6: layer 2: 0 -> 8 (1.6 < 9.6); layer 1: 4 (5.6), 12 (2.4) no better -> 8
    # 13:  layer 2: 0 -> 8; layer 1: 12 (1.0 < 5.0) -> 12, then 8 is worse -> 12
    # 1:   layer 2: 8 is worse than 0; layer 1: 4 (3.0) worse than 0 (1.0) -> 0
    # 6:   layer 2: 0 -> 8 (2 < 6); layer 1: 4 (2.0) ties 8 (2.0), smaller id -> 4;
    #      from 4: 0 (6) and 8 (2) are not smaller than (2, 4) -> 4
    assert seed.tolist() == [8, 12, 0, 4]
    assert moves.tolist() == [1, 2, 0, 2]


@pytest.fixture(scope="module")
def tiny_layers():
    w = workloads.config_tiny(scale=0.3)  # 3,000 data, 300 queries, d = 32
    L = oracle.build_layers(w.X, 8, seed=3)
    return w, L


def test_layers_are_nested_builds(tiny_layers):
    w, L = tiny_layers
    assert len(L.ids) >= 2
    for j, sel in enumerate(L.ids):
        assert np.array_equal(sel, np.nonzero(L.lvl >= j + 1)[0])
        if j:
            assert set(sel.tolist()) <= set(L.ids[j - 1].tolist())
        # each layer's graph is the merged-graph recipe over its nodes alone
        g = oracle.build_merged(np.zeros((0, w.d), np.float32), w.X[sel], 8)
        assert np.array_equal(L.adj[j], np.where(g.adj >= 0, sel[np.maximum(g.adj, 0)], -1))
        assert L.entry[j] == sel[g.entry]
        assert set(L.adj[j][L.adj[j] >= 0].tolist()) <= set(sel.tolist())


def test_descent_ends_in_a_local_minimum(tiny_layers):
    w, L = tiny_layers
    seed, moves = oracle.descend(w.Q, w.X, L)
    X = w.X.astype(np.float64)
    pos1 = {v: i for i, v in enumerate(L.ids[0].tolist())}
    top = L.entry[-1]
    for qi in range(w.Q.shape[0]):
        q = w.Q[qi].astype(np.float64)
        s = int(seed[qi])
        assert s in pos1
        ds = np.linalg.norm(X[s] - q)
        # no layer-1 neighbour of the seed is smaller by (distance, id)
        for v in L.adj[0][pos1[s]].tolist():
            if v >= 0:
                dv = np.linalg.norm(X[v] - q)
                assert (dv, v) >= (ds, s)
        # every move decreased (distance, id): the seed is not worse than the top entry
        assert (ds, s) <= (np.linalg.norm(X[top] - q), top)


def test_complete_layers_find_the_nearest_node():
    # when every layer graph is complete, the descent reaches the exact
    # nearest node of layer 1 by (distance, id) (brute force)
    w = workloads.config_tiny(scale=0.1)
    lvl = oracle.levels(w.X.shape[0], 5)
    ids = [np.nonzero(lvl >= 1)[0].astype(np.int32), np.nonzero(lvl >= 2)[0].astype(np.int32)]
    if ids[1].size < 2:
        ids[1] = ids[0][:3]
    adj = []
    for sel in ids:
        m = sel.size
        a = np.full((m, m - 1), -1, np.int32)
        for i in range(m):
            a[i] = np.delete(sel, i)
        adj.append(np.pad(a, ((0, 0), (0, max(0, ids[0].size - m))), constant_values=-1))
    L = oracle.Layers(lvl=lvl, ids=ids, adj=adj, entry=[int(ids[0][0]), int(ids[1][0])])
    seed, _ = oracle.descend(w.Q, w.X, L)
    sel = ids[0]
    D = np.linalg.norm(w.X[sel].astype(np.float64)[None, :, :] - w.Q.astype(np.float64)[:, None, :], axis=2)
    best = np.array([sel[min(range(sel.size), key=lambda k: (D[qi, k], sel[k]))] for qi in range(D.shape[0])])
    assert np.array_equal(seed, best)


def _closure(adj, nx, start, inr):
    seen = {v for v in start if inr[v]}
    dq = deque(seen)
    while dq:
        a = dq.popleft()
        for v in adj[a].tolist():
            if 0 <= v < nx and inr[v] and v not in seen:
                seen.add(v)
                dq.append(v)
    return seen


def test_seeded_join_reductions():
    w = workloads.config_tiny(scale=0.3)
    eps = oracle.calibrate_eps(w.Q, w.X, w.target_matches)
    adj, entry, gx, gq = oracle.build_separate(w.Q, w.X, 16)
    nq, nx = w.Q.shape[0], w.X.shape[0]
    # every seed = the entry: the unseeded join
    a = oracle.join(w.Q, w.X, adj, entry, eps, merged=False, work_sharing="none")
    b = oracle.join(w.Q, w.X, adj, entry, eps, merged=False, work_sharing="none",
                    qseed=np.full(nq, entry, np.int32))
    assert a.pairs() == b.pairs() and np.array_equal(a.stats, b.stats)
    # seed = the exact nearest data node: when it is in range the greedy phase
    # stops at once (rule 1) and BFS returns its in-range closure
    D = np.linalg.norm(w.X.astype(np.float64)[None, :, :] - w.Q.astype(np.float64)[:, None, :], axis=2)
    nn = D.argmin(1).astype(np.int32)
    r = oracle.join(w.Q, w.X, adj, entry, eps, merged=False, work_sharing="none", qseed=nn)
    got = {}
    for q, x in r.pairs():
        got.setdefault(q, set()).add(x)
    for qi in range(nq):
        inr = D[qi] < eps
        want = _closure(adj, nx, [int(nn[qi])], inr) if inr[nn[qi]] else None
        if want is not None:
            assert got.get(qi, set()) == want, qi
            assert r.stats[qi, 4] == 0  # no greedy pop
