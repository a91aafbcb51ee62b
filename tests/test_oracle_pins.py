"""Pins of the CPU oracle against things other than itself.

Each test checks one oracle function against a library routine, exact
integer arithmetic, a closed form, an invariant of the problem or a result
derived by hand.  None of them re-types the oracle's own formula.
"""
import json
import os
from collections import deque

import numpy as np
import pytest
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import minimum_spanning_tree
from scipy.spatial.distance import cdist

import oracle
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _pairs(qi, xj):
    return set(zip(np.asarray(qi).tolist(), np.asarray(xj).tolist()))


def _rand(n, d, seed, grid=None):
    r = np.random.default_rng(seed)
    v = r.standard_normal((n, d))
    if grid:
        v = np.round(v * grid) / grid
    return v.astype(np.float32)


# ---------------------------------------------------------------- O1 -------

@pytest.mark.parametrize("metric", ["l2", "ip"])
def test_nlj_matches_scipy_cdist(metric):
    Q, X = _rand(37, 9, 1), _rand(53, 9, 2)
    D = cdist(Q.astype(np.float64), X.astype(np.float64),
              "euclidean" if metric == "l2" else lambda a, b: 1.0 - a @ b)
    eps = float(np.quantile(D, 0.2))
    qi, xj, dd = oracle.nlj(Q, X, eps, metric)
    ref = np.argwhere(D < eps)
    assert _pairs(qi, xj) == _pairs(ref[:, 0], ref[:, 1])
    np.testing.assert_allclose(dd, D[qi, xj], rtol=1e-12, atol=1e-12)
    # emitted in (i, j) order
    key = qi.astype(np.int64) * 1000 + xj
    assert np.all(np.diff(key) > 0)


def test_nlj_exact_on_integer_data():
    r = np.random.default_rng(5)
    Q = r.integers(0, 219, size=(40, 128)).astype(np.float32)
    X = r.integers(0, 219, size=(300, 128)).astype(np.float32)
    Qi, Xi = Q.astype(np.int64), X.astype(np.int64)
    D2 = ((Qi[:, None, :] - Xi[None, :, :]) ** 2).sum(-1)  # exact in int64
    dk = int(np.sort(D2.ravel())[500])
    eps = float(np.sqrt(dk + 0.5))
    qi, xj, dd = oracle.nlj(Q, X, eps)
    ref = np.argwhere(D2 <= dk)
    assert _pairs(qi, xj) == _pairs(ref[:, 0], ref[:, 1])
    assert np.array_equal(np.rint(dd * dd).astype(np.int64), D2[qi, xj])


def test_nlj_invariants():
    A = _rand(60, 6, 7, grid=4)
    eps = 2.2
    # self-join symmetry and the diagonal
    qi, xj, _ = oracle.nlj(A, A, eps)
    S = _pairs(qi, xj)
    assert all((j, i) in S for i, j in S)
    assert all((i, i) in S for i in range(A.shape[0]))
    # query-data symmetry J(Q,X)^T = J(X,Q)
    Q, X = A[:20], A[20:]
    a = _pairs(*oracle.nlj(Q, X, eps)[:2])
    b = _pairs(*oracle.nlj(X, Q, eps)[:2])
    assert a == {(j, i) for i, j in b}
    # monotonicity in eps
    small = _pairs(*oracle.nlj(Q, X, 1.5)[:2])
    assert small <= a and len(small) < len(a)
    # eps <= 0 gives nothing; eps above every distance gives everything
    assert oracle.nlj(Q, X, 0.0)[0].size == 0
    assert oracle.nlj(Q, X, 1e9)[0].size == Q.shape[0] * X.shape[0]
    # translation invariance (grid data + integer shift: exact in fp32)
    t = np.float32(3.0)
    assert _pairs(*oracle.nlj(Q + t, X + t, eps)[:2]) == a
    # permutation equivariance
    pq, px = np.random.default_rng(0).permutation(20), np.random.default_rng(1).permutation(40)
    c = _pairs(*oracle.nlj(Q[pq], X[px], eps)[:2])
    assert {(int(pq[i]), int(px[j])) for i, j in c} == a


def test_ip_equals_l2_on_unit_vectors():
    # for unit vectors 1 - <q,x> = |q-x|^2 / 2, so IP-join(e) = L2-join(sqrt(2e))
    A = _rand(80, 16, 9).astype(np.float64)
    A /= np.linalg.norm(A, axis=1, keepdims=True)
    A = A.astype(np.float32)
    Q, X = A[:30], A[30:]
    D = cdist(Q.astype(np.float64), X.astype(np.float64))
    vals = np.sort(D.ravel())
    mid = 0.5 * (vals[200] + vals[201])  # well away from any pair
    e_ip = mid * mid / 2.0
    assert _pairs(*oracle.nlj(Q, X, e_ip, "ip")[:2]) == _pairs(*oracle.nlj(Q, X, mid, "l2")[:2])


def test_pooled_kth_and_calibration():
    Q, X = _rand(25, 5, 11), _rand(400, 5, 12)
    D = np.sort(cdist(Q.astype(np.float64), X.astype(np.float64)).ravel())
    for k in (1, 37, 250, 999):
        vk, vk1 = oracle.pooled_kth(Q, X, k, M=64)
        assert vk == pytest.approx(D[k - 1], rel=1e-12) and vk1 == pytest.approx(D[k], rel=1e-12)
    eps = oracle.calibrate_eps(Q, X, 10.0)
    assert oracle.nlj_counts(Q, X, eps).sum() == 250


# ---------------------------------------------------------------- O2 -------

def test_knn_matches_brute_force():
    V = _rand(150, 7, 13, grid=2)  # grid data: plenty of exact distance ties
    ids, dd = oracle.knn(V, 12)
    D = cdist(V.astype(np.float64), V.astype(np.float64))
    for u in range(V.shape[0]):
        order = [v for v in np.lexsort((np.arange(150), D[u])) if v != u][:12]
        assert ids[u].tolist() == order
        np.testing.assert_allclose(dd[u], D[u, order], rtol=1e-12)


def _check_prune_rule(D, u, cand, kept, R):
    """Definition of the RNG edge rule, checked directly: a kept v has no
    earlier kept w with D[w,v] < D[u,v]; a skipped v (before R are kept) has
    one."""
    kept_so_far = []
    for v in cand:
        if len(kept_so_far) == R:
            break
        blocked = any(D[w, v] < D[u, v] for w in kept_so_far)
        if v in kept:
            assert not blocked
            kept_so_far.append(v)
        else:
            assert blocked
    assert kept_so_far == list(kept)


def test_rng_prune_rule_and_theorem():
    V = _rand(120, 4, 17)
    n = V.shape[0]
    D = cdist(V.astype(np.float64), V.astype(np.float64))
    ids, dd = oracle.knn(V, n - 1)
    for u in range(n):
        kept = oracle.rng_prune(V, u, ids[u], dd[u], n - 1).tolist()
        _check_prune_rule(D, u, ids[u].tolist(), kept, n - 1)
        # Appendix C: the closest node of u is a neighbour of u
        assert ids[u, 0] in kept
        # every exact RNG edge (no w closer to both ends) survives the prune
        for v in range(n):
            if v == u:
                continue
            lune = (D[u] < D[u, v]) & (D[v] < D[u, v])
            lune[[u, v]] = False
            if not lune.any():
                assert v in kept
    # the cap R keeps a prefix of the uncapped scan
    kept5 = oracle.rng_prune(V, 3, ids[3], dd[3], 5).tolist()
    full = oracle.rng_prune(V, 3, ids[3], dd[3], n - 1).tolist()
    assert kept5 == full[:5]


def _reach(adj, s):
    seen = {s}
    dq = deque([s])
    while dq:
        u = dq.popleft()
        for v in adj[u]:
            if v >= 0 and v not in seen:
                seen.add(v)
                dq.append(v)
    return seen


def test_build_merged_properties():
    w = workloads.config_tiny(scale=0.08)  # 800 data, 80 queries
    R, Kc = 16, 32
    g = oracle.build_merged(w.Q, w.X, R, Kc)
    V = np.concatenate([w.X, w.Q]).astype(np.float64)
    n = V.shape[0]
    D = cdist(V, V)
    adj = g.adj
    # out-degree <= R, -1 padding at the end, no self loops, no duplicates
    for u in range(n):
        row = adj[u]
        k = int((row >= 0).sum())
        assert np.all(row[:k] >= 0) and np.all(row[k:] == -1)
        assert u not in row[:k].tolist() and len(set(row[:k].tolist())) == k
        # rows sorted by (dist, id)
        key = list(zip(D[u, row[:k]].tolist(), row[:k].tolist()))
        assert key == sorted(key)
        np.testing.assert_allclose(g.elen[u, :k], D[u, row[:k]], rtol=1e-12)
    # entry = node nearest to the centroid
    c = V.mean(axis=0)
    assert g.entry == int(np.argmin(((V - c) ** 2).sum(1)))
    # every node reachable from the entry
    assert len(_reach(adj, g.entry)) == n
    # nearest neighbour of every node is one of its out-neighbours
    Dn = D + np.diag(np.full(n, np.inf))
    nn = np.argmin(Dn, axis=1)
    assert all(nn[u] in adj[u].tolist() for u in range(n))
    # reverse-edge step: with fwd(v) the pruned kNN list of v and rev(v) the
    # nodes whose list holds v, the final row of v is fwd+rev when that fits
    # in R, and otherwise an RNG prune of fwd+rev (plus repair edges)
    ids, dd = oracle.knn(V.astype(np.float32), Kc)
    fwd = [oracle.rng_prune(V.astype(np.float32), u, ids[u], dd[u], R).tolist() for u in range(n)]
    rev = [[] for _ in range(n)]
    for u in range(n):
        for v in fwd[u]:
            rev[v].append(u)
    repairs = 0
    for v in range(n):
        cand = sorted(set(fwd[v]) | set(rev[v]), key=lambda x: (D[v, x], x))
        row = [x for x in adj[v].tolist() if x >= 0]
        extra = [x for x in row if x not in cand]
        repairs += len(extra)
        if len(cand) <= R:
            assert set(cand) <= set(row)
        else:
            kept = [x for x in row if x in cand]
            _check_prune_rule(D, v, cand, kept, R) if not extra else None
    assert repairs == g.repairs


def test_mst_matches_scipy():
    w = workloads.config_tiny(scale=0.08)
    g = oracle.build_merged(w.Q, w.X, 16)
    parent, order, wt = oracle.mst_parents(w.Q, w.X, g.adj, g.entry)
    nx, nq = w.X.shape[0], w.Q.shape[0]
    V = np.concatenate([w.X, w.Q]).astype(np.float64)
    # vertex set {s} + queries; edges: G edges between queries + (s, q)
    nodes = [g.entry] + [nx + i for i in range(nq) if nx + i != g.entry]
    loc = {u: i for i, u in enumerate(nodes)}
    rows, cols, vals = [], [], []
    for i in range(nq):
        u = nx + i
        for v in g.adj[u]:
            if v >= nx and v != u:
                rows.append(loc[u]); cols.append(loc[int(v)])
                vals.append(np.linalg.norm(V[u] - V[v]))
        if u != g.entry:
            rows.append(0); cols.append(loc[u]); vals.append(np.linalg.norm(V[u] - V[g.entry]))
    M = coo_matrix((vals, (rows, cols)), shape=(len(nodes), len(nodes))).tocsr()
    M = M.maximum(M.T)
    assert wt == pytest.approx(minimum_spanning_tree(M).sum(), rel=1e-12)
    # parent pointers form a tree rooted at s, listed parents-first
    pos = {int(q): k for k, q in enumerate(order)}
    assert sorted(pos) == list(range(nq))
    for i in range(nq):
        p = int(parent[i])
        if p >= 0:
            assert p >= nx and pos[p - nx] < pos[i]
    tot = 0.0
    # tree weight from the parent pointers equals the MST weight
    for i in range(nq):
        p = int(parent[i])
        tot += np.linalg.norm(V[nx + i] - V[p if p >= 0 else g.entry])
    assert tot == pytest.approx(wt, rel=1e-12)


# ---------------------------------------------------------------- O3 -------

def _load_examples():
    with open(os.path.join(GOLDEN, "worked_examples.json")) as f:
        return json.load(f)["examples"]


@pytest.mark.parametrize("ex", _load_examples(), ids=lambda e: e["name"])
def test_worked_examples(ex):
    Q = np.array(ex["Q"], np.float32)
    X = np.array(ex["X"], np.float32)
    adj = np.array(ex["adj"], np.int32)
    parent = np.array(ex.get("parent", [-1] * Q.shape[0]), np.int32)
    for key, want in ex.get("expect", {}).items():
        parts = key.split("_")
        ws, hy = parts[0], parts[1]
        beam = 0 if key.endswith("beam0") else 256
        r = oracle.join(Q, X, adj, ex["entry"], ex["eps"], work_sharing=ws,
                        hybrid=hy, hybrid_beam=beam, parent=parent)
        assert r.pairs() == {tuple(p) for p in want}, key
    if "ood" in ex:
        r = oracle.join(Q, X, adj, ex["entry"], ex["eps"], hybrid="adapt")
        assert r.stats[:, 4].tolist() == ex["ood"]
    ex_pairs = _pairs(*oracle.nlj(Q, X, ex["eps"])[:2])
    assert ex_pairs == {tuple(p) for p in ex["exact"]}
    if "parent" in ex:
        par, order, _ = oracle.mst_parents(Q, X, adj, ex["entry"])
        assert par.tolist() == ex["parent"]
    if "features" in ex:
        f = oracle.features(Q, X, adj, ex["entry"], ex["eps"])
        assert np.allclose(f[0, :Q.shape[1]], Q[0])
        np.testing.assert_allclose(f[0, Q.shape[1]:], ex["features"]["expect"], rtol=1e-6, atol=1e-12)


def test_features_ip_single_neighbour_closed_form():
    # unit vectors, one data neighbour y: for IP the feature distances are
    # 1 - <q, y>, while d1 is the L2 length |q - y| = sqrt(2 (1 - <q, y>))
    ang = np.array([0.0, 0.3, 1.2, 2.0])
    X = np.stack([np.cos(ang), np.sin(ang)], 1).astype(np.float32)  # data 0..3
    Q = np.array([[1.0, 0.0]], np.float32)                          # node 4
    adj = np.array([[1, -1], [0, -1], [1, -1], [2, -1], [1, -1]], np.int32)
    f = oracle.features(Q, X, adj, 3, 0.5, metric="ip")[0, 2:]
    ip = float(np.cos(0.3))
    assert f[1] == pytest.approx(1 - np.cos(2.0), rel=1e-6)        # dist(q, s), s = 3
    assert f[2] == pytest.approx(1 - ip, rel=1e-5)                  # min over A = {1}
    assert f[3] == pytest.approx(np.sqrt(2 * (1 - ip)), rel=1e-5)   # d1 in L2 units
    assert f[4] == pytest.approx(np.sqrt(2 * (1 - ip)), rel=1e-5)   # d2: N(1) = {0}, |x1 - x0|
    assert f[6] == 0.5 and f[7] == 0.5                              # |A| / R, in range / R


@pytest.fixture(scope="module")
def small_graph():
    w = workloads.config_tiny(scale=0.15)  # 1500 data, 150 queries
    g = oracle.build_merged(w.Q, w.X, 16)
    eps = oracle.calibrate_eps(w.Q, w.X, 10.0)
    return w, g, eps


def _closure_reference(w, g, eps, qi):
    """BFS join result of one query, as a plain graph search: the in-range
    data nodes reachable from the in-range data nodes among {s} + N(q)
    through in-range data nodes (independent of the oracle's loop)."""
    nx = w.X.shape[0]
    q = w.Q[qi].astype(np.float64)
    dist = np.linalg.norm(w.X.astype(np.float64) - q, axis=1)
    inr = dist < eps
    start = [u for u in [g.entry] + g.adj[nx + qi].tolist() if 0 <= u < nx and inr[u]]
    seen = set(start)
    dq = deque(start)
    while dq:
        u = dq.popleft()
        for v in g.adj[u]:
            if 0 <= v < nx and inr[v] and v not in seen:
                seen.add(int(v))
                dq.append(int(v))
    visited = set(u for u in [g.entry] + g.adj[nx + qi].tolist() if 0 <= u < nx)
    for u in seen:
        visited |= set(int(v) for v in g.adj[u] if 0 <= v < nx)
    return seen, visited


def test_bfs_join_is_in_range_closure(small_graph):
    w, g, eps = small_graph
    r = oracle.join(w.Q, w.X, g.adj, g.entry, eps)
    got = {}
    for a, b in zip(r.qi.tolist(), r.xj.tolist()):
        got.setdefault(a, set()).add(b)
    for qi in range(w.Q.shape[0]):
        ref, visited = _closure_reference(w, g, eps, qi)
        assert got.get(qi, set()) == ref
        assert r.stats[qi, 6] == len(visited)  # visited data nodes
        assert r.stats[qi, 0] == len(ref)


def test_join_precision_is_one(small_graph):
    w, g, eps = small_graph
    for kw in ({}, {"hybrid": "force"}, {"hybrid": "adapt"}):
        r = oracle.join(w.Q, w.X, g.adj, g.entry, eps, **kw)
        d = np.linalg.norm(w.Q[r.qi].astype(np.float64) - w.X[r.xj].astype(np.float64), axis=1)
        assert np.all(d < eps)
        np.testing.assert_allclose(r.dist, d, rtol=1e-12)
        assert len(r.pairs()) == r.qi.size  # no duplicates


def test_join_order_independent(small_graph):
    w, g, eps = small_graph
    for hy in ("off", "force"):
        base = oracle.join(w.Q, w.X, g.adj, g.entry, eps, hybrid=hy)
        for seed in (1, 99, 12345):
            r = oracle.join(w.Q, w.X, g.adj, g.entry, eps, hybrid=hy, shuffle_seed=seed)
            assert r.pairs() == base.pairs()
            assert np.array_equal(r.stats[:, :7], base.stats[:, :7])


def test_join_eps_monotone_in_self_bfs(small_graph):
    w, g, eps = small_graph
    prev = set()
    for e in (0.6 * eps, 0.8 * eps, eps, 1.2 * eps):
        cur = oracle.join(w.Q, w.X, g.adj, g.entry, e).pairs()
        assert prev <= cur
        prev = cur


def test_join_reductions(small_graph):
    w, g, eps = small_graph
    bfs = oracle.join(w.Q, w.X, g.adj, g.entry, eps)
    # hybrid with an empty heap bound is BFS
    b0 = oracle.join(w.Q, w.X, g.adj, g.entry, eps, hybrid="force", hybrid_beam=0)
    assert b0.pairs() == bfs.pairs()
    # per-query budget 0 everywhere is BFS
    z = oracle.join(w.Q, w.X, g.adj, g.entry, eps, hybrid="budget",
                    budget=np.zeros(w.Q.shape[0], np.int32))
    assert z.pairs() == bfs.pairs()
    # hybrid only adds pairs to BFS, and a larger budget never loses any
    f = oracle.join(w.Q, w.X, g.adj, g.entry, eps, hybrid="force")
    assert bfs.pairs() <= f.pairs()
    b4 = oracle.join(w.Q, w.X, g.adj, g.entry, eps, hybrid="budget",
                     budget=np.full(w.Q.shape[0], 4, np.int32))
    b16 = oracle.join(w.Q, w.X, g.adj, g.entry, eps, hybrid="budget",
                      budget=np.full(w.Q.shape[0], 16, np.int32))
    assert bfs.pairs() <= b4.pairs() <= b16.pairs()
    assert np.all(b4.stats[:, 3] <= 4) and np.all(b16.stats[:, 3] <= 16)


def test_complete_graph_gives_exact_join():
    Q, X = _rand(12, 5, 21), _rand(60, 5, 22)
    n = 72
    adj = np.array([[v for v in range(n) if v != u] for u in range(n)], np.int32)
    eps = 2.0
    exact = _pairs(*oracle.nlj(Q, X, eps)[:2])
    assert oracle.join(Q, X, adj, 0, eps).pairs() == exact


def test_connected_data_hybrid_unbounded_is_exact():
    # X-induced subgraph strongly connected (a ring both ways), queries link
    # to one data node each; hybrid with an unbounded heap and no stop rule
    # reaches every in-range node of queries whose probe found one.
    r = np.random.default_rng(4)
    X = r.standard_normal((50, 3)).astype(np.float32)
    Q = r.standard_normal((10, 3)).astype(np.float32)
    nx = 50
    adj = np.full((60, 2), -1, np.int32)
    for u in range(nx):
        adj[u] = [(u + 1) % nx, (u - 1) % nx]
    D = cdist(Q.astype(np.float64), X.astype(np.float64))
    for i in range(10):
        adj[nx + i, 0] = int(np.argmin(D[i]))
    eps = float(np.quantile(D, 0.3))
    res = oracle.join(Q, X, adj, 0, eps, hybrid="force", hybrid_beam=10 ** 6,
                      conv_threshold=0)
    exact = _pairs(*oracle.nlj(Q, X, eps)[:2])
    got = res.pairs()
    for i in range(10):
        first = int(np.argmin(D[i]))
        has_seed = D[i, first] < eps or D[i, 0] < eps
        want = {p for p in exact if p[0] == i}
        mine = {p for p in got if p[0] == i}
        assert mine == (want if has_seed else set())


def test_soft_cache_is_nearest_visited(small_graph):
    # with soft work sharing the child's extra seed is its parent's closest
    # visited data point, so a child's result contains every in-range node of
    # the self-mode result (closure is monotone in the seed set)
    w, g, eps = small_graph
    par, order, _ = oracle.mst_parents(w.Q, w.X, g.adj, g.entry)
    soft = oracle.join(w.Q, w.X, g.adj, g.entry, eps, work_sharing="soft", parent=par)
    selfm = oracle.join(w.Q, w.X, g.adj, g.entry, eps)
    assert selfm.pairs() <= soft.pairs()
    hard = oracle.join(w.Q, w.X, g.adj, g.entry, eps, work_sharing="hard", parent=par)
    assert selfm.pairs() <= hard.pairs()


def test_uncertain_band_sandwich(small_graph):
    w, g, eps = small_graph
    lo = oracle.join(w.Q, w.X, g.adj, g.entry, eps, uncertain="out", uncertain_rel=1e-2)
    mid = oracle.join(w.Q, w.X, g.adj, g.entry, eps)
    hi = oracle.join(w.Q, w.X, g.adj, g.entry, eps, uncertain="in", uncertain_rel=1e-2)
    assert lo.pairs() <= mid.pairs() <= hi.pairs()


def test_self_counts_agree_with_join(small_graph):
    w, g, eps = small_graph
    c = oracle.join_self_counts(w.Q, w.X, g.adj, g.entry, eps)
    r = oracle.join(w.Q, w.X, g.adj, g.entry, eps)
    assert np.array_equal(c, r.stats[:, 0].astype(np.int64))


# ---------------------------------------------------------------- O5 -------

def _mlp_params(din, h1, h2, k, seed):
    r = np.random.default_rng(seed)
    return [r.standard_normal((h1, din)) * 0.5, r.standard_normal(h1) * 0.1,
            r.standard_normal((h2, h1)) * 0.5, r.standard_normal(h2) * 0.1,
            r.standard_normal((k, h2)) * 0.5, r.standard_normal(k) * 0.1]


def test_mlp_forward_hand_example():
    # din=2, h1=h2=2, k=1: W1 = I, b1 = (0,-1); W2 = [[1,1],[1,-1]], b2 = 0;
    # W3 = [[2, -1]], b3 = 0.5.  x = (3, 0.5): a1 = relu(3, -0.5) = (3, 0);
    # a2 = relu(3, 3) = (3, 3); z = 2*3 - 3 + 0.5 = 3.5.  x = (-1, 2):
    # a1 = (0, 1); a2 = relu(1, -1) = (1, 0); z = 2 + 0.5 = 2.5.
    p = [np.eye(2), np.array([0.0, -1.0]), np.array([[1.0, 1.0], [1.0, -1.0]]),
         np.zeros(2), np.array([[2.0, -1.0]]), np.array([0.5])]
    z = oracle.mlp_forward(p, np.array([[3.0, 0.5], [-1.0, 2.0]]))
    assert z[:, 0].tolist() == [3.5, 2.5]
    # BCE with logit 0 and target 1 is log 2
    p0 = [np.zeros((2, 2)), np.zeros(2), np.zeros((2, 2)), np.zeros(2), np.zeros((1, 2)), np.zeros(1)]
    loss, _ = oracle.mlp_bce_backward(p0, np.ones((3, 2)), np.ones((3, 1)))
    assert loss == pytest.approx(np.log(2.0), rel=1e-15)


def test_mlp_gradients_finite_differences():
    din, h1, h2, k, n = 7, 6, 5, 4, 9
    p = _mlp_params(din, h1, h2, k, 3)
    r = np.random.default_rng(8)
    Xin = r.standard_normal((n, din))
    Y = r.random((n, k))
    mask = (r.random((n, k)) < 0.7).astype(np.float64)
    loss, grads = oracle.mlp_bce_backward(p, Xin, Y, mask)
    h = 1e-6
    for pi in range(6):
        flat = p[pi].reshape(-1)
        for idx in r.choice(flat.size, size=min(flat.size, 12), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp, _ = oracle.mlp_bce_backward(p, Xin, Y, mask)
            flat[idx] = old - h
            lm, _ = oracle.mlp_bce_backward(p, Xin, Y, mask)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            assert grads[pi].reshape(-1)[idx] == pytest.approx(fd, rel=1e-5, abs=1e-9)


def test_mlp_training_reduces_loss():
    r = np.random.default_rng(2)
    Xin = r.standard_normal((200, 4))
    Y = (Xin[:, :1] + Xin[:, 1:2] > 0).astype(np.float64)  # separable
    p = _mlp_params(4, 8, 8, 1, 5)
    l0, _ = oracle.mlp_bce_backward(p, Xin, Y)
    for _ in range(300):
        loss, g = oracle.mlp_bce_backward(p, Xin, Y)
        p = [a - 0.2 * b for a, b in zip(p, g)]
    assert loss < 0.2 * l0
    acc = ((oracle.mlp_forward(p, Xin) > 0) == (Y > 0.5)).mean()
    assert acc > 0.95


def test_adam_step_hand_examples():
    """or_adam_step against hand-derived values (Kingma and Ba 2015, Algorithm
    1): two steps of a scalar, and the constant-gradient closed form, which a
    wrong bias correction or an eps inside the square root would break."""
    ex = json.load(open(os.path.join(GOLDEN, "adam_worked_example.json")))
    e = ex["two_steps"]
    h = e["hyper"]
    p, m, v = (np.array([x], np.float64) for x in (e["p0"], 0.0, 0.0))
    for t, (g, want) in enumerate(zip(e["grads"], e["after"]), start=1):
        oracle.adam_step(p, np.array([g]), m, v, t, h["lr"], h["beta1"], h["beta2"], h["eps"])
        assert m[0] == pytest.approx(want["m"], rel=1e-14)
        assert v[0] == pytest.approx(want["v"], rel=1e-13)
        assert p[0] == pytest.approx(want["p"], rel=1e-14)
    c = ex["constant_gradient"]
    h = c["hyper"]
    p = np.array(c["p0"], np.float64)
    m, v = np.zeros_like(p), np.zeros_like(p)
    for t in range(1, c["steps"] + 1):
        oracle.adam_step(p, np.array(c["g"]), m, v, t, h["lr"], h["beta1"], h["beta2"], h["eps"])
    np.testing.assert_allclose(p, c["p_after"], rtol=1e-12, atol=1e-15)


def test_nlj_counts_per_query_against_scipy():
    """Per-query counts of the exact join on integer data, at an eps equal to
    an actual pair distance: the pairs at exactly eps must not be counted
    (strict predicate of Definition 1), and each query's count is its own."""
    r = np.random.default_rng(77)
    Q = r.integers(0, 6, size=(45, 5)).astype(np.float32)
    X = r.integers(0, 6, size=(260, 5)).astype(np.float32)
    D = cdist(Q.astype(np.float64), X.astype(np.float64))
    # squared distances are small integers: sqrt of one is the same double on
    # both sides, and many pairs tie with it
    eps = float(np.sqrt(np.median(np.rint(D * D))))
    ties = int((np.rint(D * D) == np.rint(eps * eps)).sum())
    assert ties > 100
    want = (D < eps).sum(axis=1)
    got = oracle.nlj_counts(Q, X, eps)
    assert np.array_equal(got, want)
    assert len(set(want.tolist())) > 10  # the split differs from query to query
    assert np.array_equal(oracle.nlj_counts(Q, X, eps, "l2"),
                          np.bincount(oracle.nlj(Q, X, eps)[0], minlength=Q.shape[0]))


def test_build_hub_worked_example():
    """or_build_merged on the hub workload, against rows derived by hand from
    the RNG rule of Appendix C (keep v unless a kept w has dist(w, v) <
    dist(u, v); ties by id).  Chain vector a_t (node 1 + t) is at squared
    distance 2k from a_(t+-k) (k < 60) and 60 from the hub (node 0): its kNN
    list puts a_(t-1), a_(t+1) first, both kept, every other chain vector is
    blocked by one of them, and the hub (at 60, not strictly farther from
    a_(t-1) than from a_t) is kept.  So the hub has 1,024 reverse-edge
    candidates, all at squared distance 60, scanned by id: a_s is blocked by
    a kept a_t iff the cyclic offset |s - t| < 30, so the kept ones are a_0,
    a_30, ..., up to R = 32 of them.  A prune limited to the 768 nearest
    candidates would stop at a_750 with 26 edges."""
    w = workloads.hub_chain()
    g = oracle.build_merged(w.Q, w.X, 32)
    assert g.adj[0].tolist() == [1 + 30 * j for j in range(32)]
    for t in (5, 500, 1000):
        assert g.adj[1 + t, :3].tolist() == [t, t + 2, 0] and (g.adj[1 + t, 3:] == -1).all()
    # the same prune over the first 768 candidates only keeps 26
    V = np.concatenate([w.X, w.Q])
    cand = np.arange(1, 769, dtype=np.int32)
    kept = oracle.rng_prune(V, 0, cand, np.full(768, np.sqrt(60.0)), 32)
    assert kept.tolist() == [1 + 30 * j for j in range(26)]


# ------------------------------------------- O3, separate indexes ---------

def _line_sep(Qv, eps, entry, **kw):
    """Data 0..9 on a line (node i at coordinate i), the data graph a chain
    (i - 1, i + 1), queries at Qv; separate-index join of Algorithm 1."""
    X = np.arange(10, dtype=np.float32)[:, None]
    Q = np.asarray(Qv, np.float32)[:, None]
    nx, nq = 10, Q.shape[0]
    adj = np.full((nx + nq, 2), -1, np.int32)
    for i in range(nx):
        adj[i] = [i - 1 if i > 0 else -1, i + 1 if i < 9 else -1]
    adj[:nx] = np.sort(np.where(adj[:nx] < 0, 99, adj[:nx]), 1)
    adj[adj == 99] = -1
    return oracle.join(Q, X, adj, entry, eps, merged=False, work_sharing="none", **kw)


def test_separate_greedy_rule1_worked_example():
    """Query at 7.2, entry 0.  eps = 0.5: best-first walks 0, 1, ..., 6 (7
    pops) until the front is 7 (distance 0.2 < eps, rule 1); the expansion
    from 7 finds 6 (1.2) and 8 (0.8) out of range: I = {7}.  eps = 1.3: the
    pop of 5 visits 6 (1.2, in range) which is then the front: 6 pops; the
    expansion adds 7 (0.2) and 8 (0.8), 9 (1.8) is out: I = {6, 7, 8}."""
    r = _line_sep([7.2], 0.5, 0)
    assert sorted(r.xj.tolist()) == [7] and r.stats[0, 4] == 7
    r = _line_sep([7.2], 1.3, 0)
    assert sorted(r.xj.tolist()) == [6, 7, 8] and r.stats[0, 4] == 6


def _star(conv, beam):
    """Entry 0 at the origin, 10 leaves at coordinates 2, 3, ..., 11 (ids
    1..10), edges 0 <-> leaf; the query at -1 (distance 1 to the entry, 3..12
    to the leaves), eps = 0.5: nothing in range."""
    X = np.array([[0.0]] + [[2.0 + k] for k in range(10)], np.float32)
    Q = np.array([[-1.0]], np.float32)
    adj = np.full((12, 10), -1, np.int32)
    adj[0, :10] = np.arange(1, 11)
    adj[1:11, 0] = 0
    return oracle.join(Q, X, adj, 0, 0.5, merged=False, work_sharing="none",
                       conv_threshold=conv, greedy_beam=beam)


def test_separate_greedy_rule2_and_trim_worked_example():
    """Rule 2 with conv_threshold 3: check 1 (front = entry, distance 1)
    sets the best and pops; checks 2 and 3 see leaves at 3 and 4 (no
    decrease: stall 1, 2) and pop them; check 4 sees the leaf at 5, stall 3
    -> stop: 3 pops, every node visited by the first pop.  Without rule 2
    all 11 nodes are popped.  With greedy_beam 2 the first pop's queue is
    trimmed to the two nearest leaves: 3 pops, all 11 nodes still visited."""
    r = _star(3, 256)
    assert r.qi.size == 0 and r.stats[0, 4] == 3 and r.stats[0, 6] == 11
    r = _star(0, 256)
    assert r.stats[0, 4] == 11 and r.stats[0, 6] == 11
    r = _star(0, 2)
    assert r.stats[0, 4] == 3 and r.stats[0, 6] == 11


def test_separate_complete_graph_gives_exact_join():
    # a complete data graph: the first pop visits every data node, so INLJ
    # (and HWS / SWS) return the exact join for every query
    Q, X = _rand(12, 4, 31), _rand(40, 4, 32)
    nx = X.shape[0]
    adj = np.full((nx + 12, nx - 1), -1, np.int32)
    for i in range(nx):
        adj[i] = [j for j in range(nx) if j != i]
    for i in range(12):  # query graph: a chain
        adj[nx + i, 0] = nx + (i + 1) % 12
    eps = 1.6
    want = _pairs(*oracle.nlj(Q, X, eps)[:2])
    par, _, _ = oracle.mst_parents(Q, X, adj, 0)
    for ws in ("none", "soft", "hard"):
        r = oracle.join(Q, X, adj, 0, eps, merged=False, work_sharing=ws, parent=par)
        assert r.pairs() == want, ws


# ---------------------------------------------------------- NN-Map --------

def test_nnmap_witness_matches_brute_force_and_property():
    """Witnesses against a brute-force argmin on integer data (exact, the
    first of equal minima = the smaller id), and the witness property of
    Section 6 for many thresholds: dist[q] >= eps gives no match for q,
    otherwise the witness itself is a match."""
    r = np.random.default_rng(41)
    Q = r.integers(0, 5, size=(60, 6)).astype(np.float32)
    X = r.integers(0, 5, size=(300, 6)).astype(np.float32)
    adj, entry, _, _ = oracle.build_separate(Q, X, 8)
    m = oracle.nnmap(Q, X, adj)
    D = cdist(Q.astype(np.float64), X.astype(np.float64))
    assert np.array_equal(m.w, np.argmin(D, axis=1))
    assert np.array_equal(m.dist, D.min(axis=1))
    for eps in np.unique(np.round(D.ravel(), 6))[:40]:
        counts = (D < eps).sum(axis=1)
        assert np.all(counts[m.dist >= eps] == 0)
        has = m.dist < eps
        assert np.all(D[np.nonzero(has)[0], m.w[has]] < eps)


def test_nnmap_ood_bit_worked_example():
    """Data: a tight line 0, 1, 2, 3 (chain edges, length 1) on the x axis.
    Query A at (1, 0.5): witness 1 (distance 0.5), d2 = mean edge length of
    node 1 = 1 -> ratio 0.5, not OOD.  Query B at (2, 3): witness 2 (distance
    3), ratio 3 > 1.5 -> OOD."""
    X = np.array([[0, 0], [1, 0], [2, 0], [3, 0]], np.float32)
    Q = np.array([[1, 0.5], [2, 3]], np.float32)
    adj = np.full((6, 2), -1, np.int32)
    adj[0, 0] = 1
    adj[1] = [0, 2]
    adj[2] = [1, 3]
    adj[3, 0] = 2
    m = oracle.nnmap(Q, X, adj)
    assert m.w.tolist() == [1, 2]
    np.testing.assert_allclose(m.dist, [0.5, 3.0])
    assert m.ood.tolist() == [0, 1]


def test_nnmap_join_worked_example():
    """Line 0..9 with chain edges, query at 7.2.  eps = 1.3: the witness 7
    (0.2) is in range, BFS adds 6 (1.2) and 8 (0.8), not 5 (2.2) or 9 (1.8):
    {6, 7, 8}.  eps = 0.1 <= dist = 0.2: certified empty, nothing visited."""
    X = np.arange(10, dtype=np.float32)[:, None]
    Q = np.array([[7.2]], np.float32)
    adj = np.full((11, 2), -1, np.int32)
    for i in range(10):
        row = [j for j in (i - 1, i + 1) if 0 <= j < 10]
        adj[i, :len(row)] = row
    m = oracle.nnmap(Q, X, adj)
    assert m.w.tolist() == [7]
    r = oracle.join(Q, X, adj, 0, 1.3, merged=False, work_sharing="nnmap", nnmap=m)
    assert sorted(r.xj.tolist()) == [6, 7, 8]
    r = oracle.join(Q, X, adj, 0, 0.1, merged=False, work_sharing="nnmap", nnmap=m)
    assert r.qi.size == 0 and r.stats[0, 1] == 0 and r.stats[0, 6] == 0


def test_nnmap_complete_graph_gives_exact_join():
    Q, X = _rand(15, 4, 51), _rand(50, 4, 52)
    nx = X.shape[0]
    adj = np.full((nx + 15, nx - 1), -1, np.int32)
    for i in range(nx):
        adj[i] = [j for j in range(nx) if j != i]
    m = oracle.nnmap(Q, X, adj)
    for eps in (0.8, 1.5, 2.5):
        want = _pairs(*oracle.nlj(Q, X, eps)[:2])
        r = oracle.join(Q, X, adj, 0, eps, merged=False, work_sharing="nnmap", nnmap=m)
        assert r.pairs() == want
