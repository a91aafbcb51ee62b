"""GPU parity of the merged-graph build (vj_build_merged_index) with the
oracle's deterministic build (exact kNN, RNG prune, reverse edges, entry,
connectivity repair; ties on smaller id).

On integer data every distance the build compares is exact on both sides,
so the adjacency must be identical.  On float data rows may differ only
where fp32 and fp64 order two near-equal distances differently; at least
99.5% of rows must be identical and every structural invariant must hold.
"""
from collections import deque

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2603_16360_amd import vj  # noqa: E402


def _build(w, R):
    print(f"[gpu-step] build nq={w.Q.shape[0]} nx={w.X.shape[0]} d={w.d} R={R}", flush=True)
    idx = vj.vj_build_merged_index(torch.from_numpy(w.Q).cuda(), torch.from_numpy(w.X).cuda(),
                                   metric=w.metric, R=R)
    adj, elen, parent = idx.export_graph()
    return idx, adj.cpu().numpy(), elen.cpu().numpy(), parent.cpu().numpy()


def _invariants(w, adj, elen, entry, R):
    V = np.concatenate([w.X, w.Q]).astype(np.float64)
    n = V.shape[0]
    deg = (adj >= 0).sum(1)
    assert deg.max() <= R
    for u in range(0, n, max(1, n // 500)):
        row = adj[u, :deg[u]]
        assert np.all(adj[u, deg[u]:] == -1) and u not in row.tolist()
        d = np.linalg.norm(V[row] - V[u], axis=1)
        assert np.all(np.diff(d) >= -1e-5 * (1 + d[1:]))
        np.testing.assert_allclose(elen[u, :deg[u]], d, rtol=1e-5, atol=1e-4)
    seen = np.zeros(n, bool)
    seen[entry] = True
    dq = deque([entry])
    while dq:
        u = dq.popleft()
        for v in adj[u]:
            if v >= 0 and not seen[v]:
                seen[v] = True
                dq.append(v)
    assert seen.all()


def test_build_integer_data_identical():
    w = workloads.config_mid(scale=0.01)  # 10,000 + 1,000 nodes, d=128
    idx, adj, elen, parent = _build(w, 32)
    g = oracle.build_merged(w.Q, w.X, 32)
    info = idx.info()
    assert info["entry"] == g.entry
    same = (adj == g.adj).all(axis=1)
    print(f"[build] integer rows identical {same.mean():.5f}; {idx.build_stats()}", flush=True)
    assert same.all()
    _invariants(w, adj, elen, info["entry"], 32)


def test_build_pruned_sweep_identical():
    # well-separated integer clusters: the kNN sweep's second pass skips most
    # groups of nodes (the triangle bound rules them out for every row of a
    # block), and the graph must still be the oracle's, row for row
    w = workloads.separated_integer_case()
    idx, adj, elen, parent = _build(w, w.R)
    st = idx.build_stats()
    print(f"[build] separated clusters: {st}", flush=True)
    assert st["tiles_all"] > 0 and st["tiles_first"] > 0
    assert st["tiles_first"] + st["tiles_second"] < 0.5 * st["tiles_all"]
    assert 0 <= st["repairs_listed"] <= st["repairs"]
    g = oracle.build_merged(w.Q, w.X, w.R)
    assert idx.info()["entry"] == g.entry
    same = (adj == g.adj).all(axis=1)
    print(f"[build] separated rows identical {same.mean():.5f}", flush=True)
    assert same.all()
    _invariants(w, adj, elen, g.entry, w.R)


def test_build_pruned_sweep_float():
    # the same well-separated geometry in float32: the pruning bound then
    # carries the three-term tile key's error bound; rows may differ from
    # the fp64 oracle's only where fp32 and fp64 order near-equal distances
    w = workloads.separated_float_case()
    idx, adj, elen, parent = _build(w, w.R)
    st = idx.build_stats()
    print(f"[build] separated float clusters: {st}", flush=True)
    assert st["tiles_first"] + st["tiles_second"] < 0.5 * st["tiles_all"]
    g = oracle.build_merged(w.Q, w.X, w.R)
    same = (adj == g.adj).all(axis=1)
    print(f"[build] separated float rows identical {same.mean():.5f}", flush=True)
    assert same.mean() >= 0.995
    _invariants(w, adj, elen, idx.info()["entry"], w.R)


def test_build_hub_identical():
    # one node with 1,024 reverse-edge candidates whose 768 nearest prune to
    # fewer than R edges: the build must prune the whole list, as the oracle
    # does (its rows are pinned by a hand derivation on the CPU)
    w = workloads.hub_chain()
    idx, adj, elen, parent = _build(w, 32)
    g = oracle.build_merged(w.Q, w.X, 32)
    assert idx.info()["entry"] == g.entry
    print(f"[build] hub row {adj[0].tolist()}", flush=True)
    assert adj[0].tolist() == g.adj[0].tolist()
    same = (adj == g.adj).all(axis=1)
    assert same.all(), np.nonzero(~same)[0][:10]
    _invariants(w, adj, elen, g.entry, 32)


def test_build_float_data():
    w = workloads.config_tiny()  # 10,000 + 1,000 nodes, d=32
    idx, adj, elen, parent = _build(w, 16)
    g = oracle.build_merged(w.Q, w.X, 16)
    info = idx.info()
    assert info["entry"] == g.entry
    same = (adj == g.adj).all(axis=1)
    print(f"[build] float rows identical {same.mean():.5f}", flush=True)
    assert same.mean() >= 0.995
    _invariants(w, adj, elen, info["entry"], 16)
    # the library's query MST (parent pointers) is a spanning tree of the
    # query-query edges plus (s, q) edges with scipy's minimum total weight
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import minimum_spanning_tree
    V = np.concatenate([w.X, w.Q]).astype(np.float64)
    nx, nq, s = w.X.shape[0], w.Q.shape[0], info["entry"]
    loc = lambda u: u - nx if u >= nx else nq  # vertex nq stands for s
    rows, cols, vals = [], [], []
    for i in range(nq):
        u = nx + i
        for v in adj[u]:
            if v >= nx and v != u:
                rows.append(loc(u)); cols.append(loc(int(v))); vals.append(np.linalg.norm(V[u] - V[v]))
        if u != s:
            rows.append(loc(s)); cols.append(loc(u)); vals.append(np.linalg.norm(V[u] - V[s]))
    M = coo_matrix((vals, (rows, cols)), shape=(nq + 1, nq + 1)).tocsr()
    want = minimum_spanning_tree(M.maximum(M.T)).sum()
    tot = sum(np.linalg.norm(V[nx + i] - V[p if p >= 0 else s]) for i, p in enumerate(parent.tolist()))
    assert tot == pytest.approx(want, rel=1e-5)


# row widths of the kNN sweep's register-row kernel: (d, integer, vmax);
# integer cases keep 2 Kp vmax^2 < 2^24 so the one-term tiles are exact
WIDTHS = [(40, True, 218), (96, True, 218), (160, True, 150), (200, True, 100),
          (64, False, 0), (96, False, 0), (128, False, 0)]


@pytest.mark.parametrize("d,integer,vmax", WIDTHS,
                         ids=[f"d{d}-{'int' if i else 'float'}" for d, i, _ in WIDTHS])
def test_build_widths(d, integer, vmax):
    # ragged node counts (not multiples of any tile) and small enough for
    # the column-split path of the kNN sweep
    w = workloads.width_case(d, 5_003, 697, integer, 900 + d, vmax=vmax or 218)
    idx, adj, elen, parent = _build(w, 16)
    g = oracle.build_merged(w.Q, w.X, 16)
    assert idx.info()["entry"] == g.entry
    same = (adj == g.adj).all(axis=1)
    print(f"[build] width {d} {'integer' if integer else 'float'} rows identical "
          f"{same.mean():.5f}", flush=True)
    if integer:
        assert same.all(), np.nonzero(~same)[0][:10]
    else:
        assert same.mean() >= 0.995
    _invariants(w, adj, elen, g.entry, 16)


def test_build_then_join_recall():
    # end to end: GPU graph + GPU join vs the GPU brute-force ground truth
    w = workloads.config_tiny()
    eps = oracle.calibrate_eps(w.Q, w.X, w.target_matches)
    idx, adj, _, _ = _build(w, 16)
    res = vj.vj_join(idx, eps)
    qx, _ = res.export()
    gt, _ = vj.vj_bruteforce_join(torch.from_numpy(w.Q).cuda(), torch.from_numpy(w.X).cuda(),
                                  eps).export()
    G = set(map(tuple, qx.cpu().numpy().tolist()))
    T = set(map(tuple, gt.cpu().numpy().tolist()))
    assert G <= T
    print(f"[build] recall {len(G) / len(T):.4f}", flush=True)
    assert len(G) / len(T) > 0.9
