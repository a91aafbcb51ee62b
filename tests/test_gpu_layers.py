"""GPU parity of the HNSW-style upper layers (vj_index_build_layers,
vj_index_descend) and of separate-index joins seeded by the descent
(layer_seeds = 1) with the oracle's build_layers, descend and
join(qseed=...).

On integer data every distance is exact in fp32, so the layers' node sets,
adjacency and entries, each query's seed and number of moves, and the
seeded joins' pair sets and counters must be identical.  Float data: the
seeds must be local minima of layer 1 within fp32 rounding.
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2603_16360_amd import vj  # noqa: E402

MODES = [{"work_sharing": "none"}, {"work_sharing": "soft"}, {"work_sharing": "hard"},
         {"work_sharing": "none", "hybrid": "force"},
         {"work_sharing": "none", "greedy_beam": 4, "conv_threshold": 3}]


def _say(msg):
    print(f"[gpu-step] {msg}", flush=True)


@pytest.fixture(scope="module")
def integer_case():
    w = workloads.config_mid(scale=0.01)  # 10,000 x 128 integer data, 1,000 queries
    eps = oracle.calibrate_eps(w.Q, w.X, w.target_matches, integer=True)
    adj, entry, _, _ = oracle.build_separate(w.Q, w.X, 32)
    parent, _, _ = oracle.mst_parents(w.Q, w.X, adj, entry)
    _say(f"separate index nq={w.Q.shape[0]} nx={w.X.shape[0]} d={w.d}, layers R=16 seed=11")
    idx = vj.vj_index_from_separate_graphs(torch.from_numpy(w.Q).cuda(), torch.from_numpy(w.X).cuda(),
                                           torch.from_numpy(adj).cuda(), entry,
                                           parent=torch.from_numpy(parent).cuda())
    vj.vj_index_build_layers(idx, R=16, seed=11)
    L = oracle.build_layers(w.X, 16, seed=11)
    return w, eps, adj, entry, parent, idx, L


def test_layers_match_oracle(integer_case):
    w, eps, adj, entry, parent, idx, L = integer_case
    got = vj.vj_index_layers(idx)
    assert len(got) == len(L.ids) >= 2
    for j, (ids, ladj, ent) in enumerate(got):
        assert np.array_equal(ids.cpu().numpy(), L.ids[j]), j
        assert np.array_equal(ladj.cpu().numpy(), L.adj[j]), j
        assert ent == L.entry[j], j
    print(f"[layers] sizes {[int(g[0].numel()) for g in got]}", flush=True)


def test_descent_matches_oracle(integer_case):
    w, eps, adj, entry, parent, idx, L = integer_case
    seed, moves = vj.vj_index_descend(idx)
    ws, wm = oracle.descend(w.Q, w.X, L)
    assert np.array_equal(seed.cpu().numpy(), ws)
    assert np.array_equal(moves.cpu().numpy(), wm)
    # a listed subset in another order
    sub = torch.tensor([7, 3, 900, 0, 512], dtype=torch.int32, device="cuda")
    s2, m2 = vj.vj_index_descend(idx, sub)
    assert np.array_equal(s2.cpu().numpy(), ws[[7, 3, 900, 0, 512]])


@pytest.mark.parametrize("kw", MODES, ids=lambda k: "-".join(f"{a}={b}" for a, b in k.items()))
def test_seeded_joins_match_oracle(integer_case, kw):
    w, eps, adj, entry, parent, idx, L = integer_case
    seeds, _ = oracle.descend(w.Q, w.X, L)
    kw = dict(kw)
    _say(f"vj_join separate layer_seeds {kw}")
    r = vj.vj_join(idx, eps, layer_seeds=1, **kw)
    qx, _ = r.export(sorted=True)
    st = r.stats().cpu().numpy()
    got = {}
    for q, x in qx.cpu().numpy().tolist():
        got.setdefault(q, set()).add(x)
    beam = kw.pop("greedy_beam", 256)
    ref = oracle.join(w.Q, w.X, adj, entry, eps, merged=False, greedy_beam=beam, parent=parent,
                      qseed=seeds, **kw)
    want = {}
    for q, x in zip(ref.qi.tolist(), ref.xj.tolist()):
        want.setdefault(q, set()).add(x)
    bad = [q for q in range(w.Q.shape[0]) if got.get(q, set()) != want.get(q, set())]
    assert not bad, f"{len(bad)} queries differ, e.g. {bad[:5]}"
    for col in (0, 2, 3, 4, 6):
        diff = np.nonzero(st[:, col] != ref.stats[:, col])[0]
        assert diff.size == 0, (col, diff[:5], st[diff[:5], col], ref.stats[diff[:5], col])
    exact = int(oracle.nlj_counts(w.Q, w.X, eps).sum())
    print(f"[layers] {kw}: recall {ref.qi.size / exact:.4f}, greedy pops mean {st[:, 4].mean():.2f}",
          flush=True)


def test_float_seeds_are_local_minima():
    w = workloads.config_tiny()
    _say("separate index tiny with layers")
    idx = vj.vj_build_separate_index(torch.from_numpy(w.Q).cuda(), torch.from_numpy(w.X).cuda(), R=16)
    vj.vj_index_build_layers(idx, R=8, seed=3)
    layers = vj.vj_index_layers(idx)
    seed, _ = vj.vj_index_descend(idx)
    seed = seed.cpu().numpy()
    ids1 = layers[0][0].cpu().numpy()
    adj1 = layers[0][1].cpu().numpy()
    pos = {v: i for i, v in enumerate(ids1.tolist())}
    X = w.X.astype(np.float64)
    for qi in range(w.Q.shape[0]):
        s = int(seed[qi])
        assert s in pos
        q = w.Q[qi].astype(np.float64)
        ds = np.linalg.norm(X[s] - q)
        for v in adj1[pos[s]].tolist():
            if v >= 0:
                assert np.linalg.norm(X[v] - q) >= ds * (1 - 1e-5), (qi, s, v)


def test_layer_seeds_errors():
    w = workloads.config_tiny(scale=0.1)
    idx = vj.vj_build_merged_index(torch.from_numpy(w.Q).cuda(), torch.from_numpy(w.X).cuda(), R=8)
    with pytest.raises(vj.VJError):
        vj.vj_join(idx, 1.0, layer_seeds=1)   # merged index
    sep = vj.vj_build_separate_index(torch.from_numpy(w.Q).cuda(), torch.from_numpy(w.X).cuda(), R=8)
    with pytest.raises(vj.VJError):
        vj.vj_join(sep, 1.0, work_sharing="none", layer_seeds=1)   # no layers yet
    with pytest.raises(vj.VJError):
        vj.vj_index_descend(sep)
    with pytest.raises(vj.VJError):
        vj.vj_index_build_layers(sep, R=0)
