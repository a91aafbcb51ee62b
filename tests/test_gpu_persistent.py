"""The persistent workgroup tier (one launch; resident workgroups claim
queries in processing order; soft / hard work sharing waits on the device
for each query's MST parent) against one workgroup per query with one
launch per MST level: identical pair sets and counters in every mode, also
when queries outgrow the LDS tables, run out of in-launch global regions and
are deferred (with their MST descendants) to later launches.  Both are also
checked against the oracle on integer data."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = [pytest.mark.gpu, pytest.mark.skip(
    reason="persistent launches are switched off: one run of this module faulted the GPU in "
           "soft work-sharing mode and the cause is not established (see the design notes)")]

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2603_16360_amd import vj  # noqa: E402

MODES = [{}, {"work_sharing": "soft"}, {"work_sharing": "hard"}, {"hybrid": "force"},
         {"work_sharing": "soft", "hybrid": "adapt"}]


def _say(msg):
    print(f"[gpu-step] {msg}", flush=True)


def _res(idx, eps, **kw):
    r = vj.vj_join(idx, eps, **kw)
    qx, _ = r.export(sorted=True)
    return qx.cpu().numpy(), r.stats().cpu().numpy(), r


@pytest.fixture(scope="module")
def integer_case():
    w = workloads.config_mid(scale=0.01)
    eps = oracle.calibrate_eps(w.Q, w.X, w.target_matches, integer=True)
    g = oracle.build_merged(w.Q, w.X, 32)
    parent, _, _ = oracle.mst_parents(w.Q, w.X, g.adj, g.entry)
    _say("persistent integer index")
    idx = vj.vj_index_from_graph(torch.from_numpy(w.Q).cuda(), torch.from_numpy(w.X).cuda(),
                                 torch.from_numpy(g.adj).cuda(), g.entry,
                                 parent=torch.from_numpy(parent).cuda())
    return w, eps, g, parent, idx


@pytest.mark.parametrize("kw", MODES, ids=lambda k: "-".join(f"{a}={b}" for a, b in k.items()) or "self")
def test_persistent_equals_level_launches_and_oracle(integer_case, kw):
    w, eps, g, parent, idx = integer_case
    _say(f"persistent {kw}")
    qa, sa, ra = _res(idx, eps, persistent=1, **kw)
    qb, sb, rb = _res(idx, eps, persistent=0, **kw)
    assert np.array_equal(qa, qb)
    assert np.array_equal(sa[:, :7], sb[:, :7])
    ref = oracle.join(w.Q, w.X, g.adj, g.entry, eps, parent=parent, **kw)
    assert set(map(tuple, qa.tolist())) == ref.pairs()
    # one launch on the workgroup tier, against one per MST level
    print(f"[persistent] {kw}: launches persistent {ra.tiers()[1]['launches']}, per level "
          f"{rb.tiers()[1]['launches']}", flush=True)
    assert ra.tiers()[1]["launches"] == 1


@pytest.mark.parametrize("ws", ["soft", "hard"])
def test_persistent_deferral_chain(ws):
    # a wide eps with the small LDS tables: many queries outgrow them and
    # exhaust the in-launch global regions, so they and their MST
    # descendants are deferred to the re-run launches
    w = workloads.config_tiny()
    eps = oracle.calibrate_eps(w.Q, w.X, w.target_matches) * 2.6
    g = oracle.build_merged(w.Q, w.X, w.R)
    parent, _, _ = oracle.mst_parents(w.Q, w.X, g.adj, g.entry)
    idx = vj.vj_index_from_graph(torch.from_numpy(w.Q).cuda(), torch.from_numpy(w.X).cuda(),
                                 torch.from_numpy(g.adj).cuda(), g.entry,
                                 parent=torch.from_numpy(parent).cuda())
    _say(f"persistent deferral {ws}")
    qa, sa, ra = _res(idx, eps, persistent=1, work_sharing=ws, coop_tables=1)
    qb, sb, rb = _res(idx, eps, persistent=0, work_sharing=ws, coop_tables=1)
    deferred = ra.timing()["n_spilled"]
    print(f"[persistent] {ws} wide eps: {deferred} queries re-run after the persistent launch "
          f"({int(((sa[:, 7] & 16) > 0).sum())} in re-run launches)", flush=True)
    assert deferred > 0  # tables and in-launch regions ran out: queries were deferred
    assert np.array_equal(qa, qb)
    assert np.array_equal(sa[:, :7], sb[:, :7])
    # and the oracle agrees on every query it does not flag as fragile
    ref = oracle.join(w.Q, w.X, g.adj, g.entry, eps, parent=parent, work_sharing=ws)
    ok = ~ref.stats[:, 7].astype(bool)
    got = {}
    for q, x in qa.tolist():
        got.setdefault(q, set()).add(x)
    want = {}
    for q, x in zip(ref.qi.tolist(), ref.xj.tolist()):
        want.setdefault(q, set()).add(x)
    bad = [q for q in np.nonzero(ok)[0].tolist() if got.get(q, set()) != want.get(q, set())]
    assert not bad, bad[:5]
