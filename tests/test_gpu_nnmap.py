"""GPU parity of the NN-Map (Section 6): the exact nearest data node of each
query (vj_build_nnmap: MFMA tile minima, fp64 re-check within the tiles'
proven error bound) against the oracle's fp64 brute force, the OOD bit, and
the NN-Map join (certified empty when the witness is not in range, else
expansion from the witness) against the oracle's join with the same map.

Integer data: witnesses, distances and bits must be identical, and so must
every join result.  Float and inner-product data: a witness may differ only
where two data nodes tie in fp64 up to summation order (relative 1e-12)."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2603_16360_amd import vj  # noqa: E402


def _say(msg):
    print(f"[gpu-step] {msg}", flush=True)


def _case(w, R):
    adj, entry, _, _ = oracle.build_separate(w.Q, w.X, R)
    _say(f"nnmap index nq={w.Q.shape[0]} nx={w.X.shape[0]} d={w.d}")
    idx = vj.vj_index_from_separate_graphs(torch.from_numpy(w.Q).cuda(), torch.from_numpy(w.X).cuda(),
                                           torch.from_numpy(adj).cuda(), entry, metric=w.metric)
    idx.build_nnmap()
    gw, gd, go = (t.cpu().numpy() for t in idx.export_nnmap())
    m = oracle.nnmap(w.Q, w.X, adj, metric=w.metric)
    return idx, adj, entry, m, gw, gd, go


def _check_map(w, m, gw, gd, go, exact):
    if exact:
        assert np.array_equal(gw, m.w)
        assert np.array_equal(gd, m.dist)
        assert np.array_equal(go, m.ood)
        return
    diff = np.nonzero(gw != m.w)[0]
    if diff.size:
        # only exact ties (up to the order of the fp64 sums) may differ
        mine = oracle.pair_dists(w.Q, w.X, diff, gw[diff], w.metric)
        assert np.allclose(mine, m.dist[diff], rtol=1e-12, atol=1e-12)
    print(f"[nnmap] witnesses differing on ties: {diff.size}", flush=True)
    np.testing.assert_allclose(gd, m.dist, rtol=1e-12, atol=1e-12)
    assert (go != m.ood).mean() <= 0.001


def test_integer_data_map_and_join_exact():
    w = workloads.config_mid(scale=0.01)
    eps = oracle.calibrate_eps(w.Q, w.X, w.target_matches, integer=True)
    idx, adj, entry, m, gw, gd, go = _case(w, 32)
    _check_map(w, m, gw, gd, go, exact=True)
    for hyb in ("off", "adapt", "force"):
        _say(f"vj_join nnmap {hyb}")
        r = vj.vj_join(idx, eps, work_sharing="nnmap", hybrid=hyb)
        qx, _ = r.export(sorted=True)
        got = set(map(tuple, qx.cpu().numpy().tolist()))
        ref = oracle.join(w.Q, w.X, adj, entry, eps, merged=False, work_sharing="nnmap",
                          nnmap=m, hybrid=hyb)
        assert got == ref.pairs(), hyb
        st = r.stats().cpu().numpy()
        for col in (0, 2, 3, 4, 5, 6):
            assert np.array_equal(st[:, col], ref.stats[:, col]), (hyb, col)
    # the certificate: queries whose witness is out of range evaluate nothing
    empty = gd >= eps
    assert empty.any() and (st[empty, 1] == 0).all() and (st[empty, 0] == 0).all()
    exact = oracle.nlj(w.Q, w.X, eps)[0]
    print(f"[nnmap] integer: {empty.mean():.3f} certified empty, recall "
          f"{len(got) / max(1, exact.size):.4f}", flush=True)


@pytest.mark.parametrize("name", ["tiny", "ood"])
def test_float_data_map(name):
    w = workloads.config_tiny() if name == "tiny" else workloads.config_ood(scale=0.004)
    idx, adj, entry, m, gw, gd, go = _case(w, 16 if name == "tiny" else 32)
    _check_map(w, m, gw, gd, go, exact=False)
    eps = oracle.calibrate_eps(w.Q, w.X, w.target_matches, w.metric)
    # BFS join from the GPU's witnesses, compared where they agree with the
    # oracle's, by the sandwich rule of the uncertain band
    r = vj.vj_join(idx, eps, metric=w.metric, work_sharing="nnmap")
    qx, _ = r.export(sorted=True)
    got = {}
    for q, x in qx.cpu().numpy().tolist():
        got.setdefault(q, set()).add(x)
    lo = oracle.join(w.Q, w.X, adj, entry, eps, metric=w.metric, merged=False,
                     work_sharing="nnmap", nnmap=m, uncertain="out")
    hi = oracle.join(w.Q, w.X, adj, entry, eps, metric=w.metric, merged=False,
                     work_sharing="nnmap", nnmap=m, uncertain="in")
    L, U = {}, {}
    for q, x in zip(lo.qi.tolist(), lo.xj.tolist()):
        L.setdefault(q, set()).add(x)
    for q, x in zip(hi.qi.tolist(), hi.xj.tolist()):
        U.setdefault(q, set()).add(x)
    same = np.nonzero(gw == m.w)[0]
    bad = [q for q in same.tolist()
           if not (L.get(q, set()) <= got.get(q, set()) <= U.get(q, set()))]
    assert not bad, bad[:5]
    # witness property on the GPU result
    assert all(gd[q] < eps for q in got)


def test_nnmap_refused_on_merged_index():
    w = workloads.config_tiny(scale=0.1)
    idx = vj.vj_build_merged_index(torch.from_numpy(w.Q).cuda(), torch.from_numpy(w.X).cuda(), R=16)
    with pytest.raises(vj.VJError):
        idx.build_nnmap()
    with pytest.raises(vj.VJError):
        vj.vj_join(idx, 1.0, work_sharing="nnmap")
