"""The query-data role switch of a merged index (Appendix E): the relabelled
index holds the same graph, and a join on it equals the oracle's join with
the roles exchanged (Q' = X, X' = Q on the relabelled adjacency, relabelled
here independently of the library); on a complete graph both directions
give the exact join, transposed."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2603_16360_amd import vj  # noqa: E402


def _relabel(adj, nx, nq):
    """Role switch of a merged adjacency in numpy: rows of the old queries
    first, data id v -> nq + v, query node id v -> v - nx."""
    rows = np.concatenate([adj[nx:], adj[:nx]])
    out = np.where(rows < 0, -1, np.where(rows < nx, rows + nq, rows - nx))
    return np.ascontiguousarray(out.astype(np.int32))


def test_swapped_graph_and_join_match_oracle():
    w = workloads.config_mid(scale=0.01)  # integer data: exact on both sides
    eps = oracle.calibrate_eps(w.Q, w.X, w.target_matches, integer=True)
    nq, nx = w.Q.shape[0], w.X.shape[0]
    g = oracle.build_merged(w.Q, w.X, 32)
    print(f"[gpu-step] roles nq={nq} nx={nx}", flush=True)
    a = vj.vj_index_from_graph(torch.from_numpy(w.Q).cuda(), torch.from_numpy(w.X).cuda(),
                               torch.from_numpy(g.adj).cuda(), g.entry)
    b = a.swap_roles()
    info = b.info()
    assert info["nq"] == nx and info["nx"] == nq
    adj2 = _relabel(g.adj, nx, nq)
    entry2 = g.entry + nq if g.entry < nx else g.entry - nx
    assert info["entry"] == entry2
    assert np.array_equal(b.export_graph(with_parent=False)[0].cpu().numpy(), adj2)
    r = vj.vj_join(b, eps)
    qx, _ = r.export(sorted=True)
    got = set(map(tuple, qx.cpu().numpy().tolist()))
    want = oracle.join(w.X, w.Q, adj2, entry2, eps).pairs()
    assert got == want
    # transposed, every pair is a pair of the original join (precision 1)
    exact = set(zip(*oracle.nlj(w.Q, w.X, eps)[:2]))
    assert {(i, j) for j, i in got} <= exact
    fwd = set(map(tuple, vj.vj_join(a, eps).export()[0].cpu().numpy().tolist()))
    print(f"[roles] recall forward {len(fwd) / len(exact):.4f}, switched "
          f"{len(got) / len(exact):.4f}", flush=True)


def test_complete_graph_both_directions_exact():
    r = np.random.default_rng(3)
    Q = r.standard_normal((10, 4)).astype(np.float32)
    X = r.standard_normal((40, 4)).astype(np.float32)
    n = 50
    adj = np.array([[j for j in range(n) if j != i] for i in range(n)], np.int32)  # R = 49
    a = vj.vj_index_from_graph(torch.from_numpy(Q).cuda(), torch.from_numpy(X).cuda(),
                               torch.from_numpy(adj).cuda(), 0)
    eps = 1.6
    exact = set(zip(*oracle.nlj(Q, X, eps)[:2]))
    fwd = set(map(tuple, vj.vj_join(a, eps).export()[0].cpu().numpy().tolist()))
    b = a.swap_roles(build_mst=True)
    got = set(map(tuple, vj.vj_join(b, eps).export()[0].cpu().numpy().tolist()))
    assert fwd == exact
    assert {(i, j) for j, i in got} == exact
    with pytest.raises(vj.VJError):
        vj.vj_build_separate_index(torch.from_numpy(Q).cuda(), torch.from_numpy(X).cuda(),
                                   R=8).swap_roles()
