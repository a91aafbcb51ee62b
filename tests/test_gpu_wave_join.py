"""GPU parity of the merged-index join (vj_join: by default one workgroup
per query with its tables in LDS; also the one-wave and global-table
tiers) against the CPU oracle.

Both sides run on the same graph (built by the oracle), the same queries,
parents and eps.  BFS mode is compared with the sandwich rule: with L and U
the oracle's results when every node within 1e-5*eps of eps is taken as out
(L) or in (U), the GPU result G must satisfy L <= G <= U per query.  Modes
whose orderings can flip under fp32 rounding (hybrid, adapt, soft, hard)
must match exactly on every query the oracle does not flag as fragile, and
overall recall must agree within 0.5 points.
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

REL = 1e-5


def _by_query(qx):
    out = {}
    for q, x in qx:
        out.setdefault(int(q), set()).add(int(x))
    return out


def _gpu_pairs(res):
    qx, dist = res.export(sorted=True)
    qx = qx.cpu().numpy()
    return qx, dist.cpu().numpy()


class Case:
    def __init__(self, w, eps, R=None, scale_name=""):
        self.w = w
        self.eps = eps
        self.g = oracle.build_merged(w.Q, w.X, R or w.R)
        self.Q = torch.from_numpy(w.Q).cuda()
        self.X = torch.from_numpy(w.X).cuda()
        self.parent, self.order, _ = oracle.mst_parents(w.Q, w.X, self.g.adj, self.g.entry)
        self.idx = vj.vj_index_from_graph(self.Q, self.X, torch.from_numpy(self.g.adj).cuda(),
                                          self.g.entry, metric=w.metric,
                                          parent=torch.from_numpy(self.parent).cuda())


def _say(msg):
    print(f"[gpu-step] {msg}", flush=True)


def test_a_hundred_queries():
    # smallest case first: 1,000 data, 100 queries, d=32, R=16
    w = workloads.config_tiny(scale=0.1)
    eps = oracle.calibrate_eps(w.Q, w.X, w.target_matches)
    g = oracle.build_merged(w.Q, w.X, w.R)
    _say("index_from_graph 100q")
    idx = vj.vj_index_from_graph(torch.from_numpy(w.Q).cuda(), torch.from_numpy(w.X).cuda(),
                                 torch.from_numpy(g.adj).cuda(), g.entry)
    _say("vj_join 100q")
    res = vj.vj_join(idx, eps)
    _say("export 100q")
    qx, _ = res.export(sorted=True)
    got = set(map(tuple, qx.cpu().numpy().tolist()))
    lo = oracle.join(w.Q, w.X, g.adj, g.entry, eps, uncertain="out").pairs()
    hi = oracle.join(w.Q, w.X, g.adj, g.entry, eps, uncertain="in").pairs()
    assert lo <= got <= hi


@pytest.fixture(scope="module")
def tiny():
    w = workloads.config_tiny()
    eps = oracle.calibrate_eps(w.Q, w.X, w.target_matches)
    print(f"[case] tiny nq={w.Q.shape[0]} nx={w.X.shape[0]} d={w.d} eps={eps:.6f}", flush=True)
    return Case(w, eps)


def _check_sandwich(case, res, qids=None, **kw):
    w = case.w
    lo = oracle.join(w.Q, w.X, case.g.adj, case.g.entry, case.eps, metric=w.metric,
                     query_ids=qids, uncertain="out", uncertain_rel=REL, **kw)
    hi = oracle.join(w.Q, w.X, case.g.adj, case.g.entry, case.eps, metric=w.metric,
                     query_ids=qids, uncertain="in", uncertain_rel=REL, **kw)
    qx, dist = _gpu_pairs(res)
    G, L, U = qx_set(qx), lo.pairs(), hi.pairs()
    assert L <= G, f"missing {len(L - G)} pairs"
    assert G <= U, f"extra {len(G - U)} pairs"
    # reported distances are the fp32 evaluation of the exact ones
    if len(qx):
        d64 = oracle.pair_dists(w.Q, w.X, qx[:, 0], qx[:, 1], w.metric)
        np.testing.assert_allclose(dist, d64, rtol=2e-5, atol=2e-5 * max(1.0, case.eps))
    return lo, hi, G


def qx_set(qx):
    return set(map(tuple, np.asarray(qx).tolist()))


def test_self_bfs_all_queries(tiny):
    _say("vj_join tiny 1000q")
    res = vj.vj_join(tiny.idx, tiny.eps)
    lo, hi, G = _check_sandwich(tiny, res)
    st = res.stats().cpu().numpy()
    # per-query counters: pairs, distinct visited data nodes, expansions
    exact = lo.stats[:, 0] == hi.stats[:, 0]
    assert np.array_equal(st[exact, 0], lo.stats[exact, 0])
    assert np.array_equal(st[exact, 6], lo.stats[exact, 6])
    assert np.array_equal(st[exact, 2], lo.stats[exact, 2])
    assert (st[:, 7] & 4).sum() == 0


def test_self_bfs_subset_and_duplicates(tiny):
    r = np.random.default_rng(3)
    ids = r.choice(tiny.w.Q.shape[0], size=257, replace=False).astype(np.int32)
    ids = np.concatenate([ids, ids[:5]])  # a query may appear twice
    res = vj.vj_join(tiny.idx, tiny.eps, query_ids=torch.from_numpy(ids).cuda())
    qx, _ = _gpu_pairs(res)
    st = res.stats().cpu().numpy()
    lo = oracle.join(tiny.w.Q, tiny.w.X, tiny.g.adj, tiny.g.entry, tiny.eps, query_ids=ids,
                     uncertain="out")
    hi = oracle.join(tiny.w.Q, tiny.w.X, tiny.g.adj, tiny.g.entry, tiny.eps, query_ids=ids,
                     uncertain="in")
    assert lo.pairs() <= qx_set(qx) <= hi.pairs()
    assert st.shape == (ids.size, 8)
    assert np.array_equal(st[:5, 0], st[-5:, 0])
    assert int(st[:, 0].sum()) == len(qx)


def _overflow_case(tiny, mult, start_tier):
    eps = tiny.eps * mult
    res = vj.vj_join(tiny.idx, eps, start_tier=start_tier)
    st = res.stats().cpu().numpy()
    ref = oracle.join(tiny.w.Q, tiny.w.X, tiny.g.adj, tiny.g.entry, eps, uncertain="out")
    refu = oracle.join(tiny.w.Q, tiny.w.X, tiny.g.adj, tiny.g.entry, eps, uncertain="in")
    assert ref.pairs() <= qx_set(_gpu_pairs(res)[0]) <= refu.pairs()
    exact = ref.stats[:, 0] == refu.stats[:, 0]
    assert np.array_equal(st[exact, 0], ref.stats[exact, 0])
    assert np.array_equal(st[exact, 6], ref.stats[exact, 6])
    return st


def test_tier_overflow_one_wave_tier(tiny):
    # at 1.4x eps (oracle: 178 of 1,000 queries hold > 512 pairs) queries
    # started on the one-wave tier outgrow its pair list and re-run on the
    # workgroup tier
    st = _overflow_case(tiny, 1.4, 0)
    assert 0 < (st[:, 7] & 1).sum() < len(st)


def test_tier_overflow_to_global_tables(tiny):
    # at 2.6x eps (oracle: up to 4,449 pairs and 5,135 visited nodes; 301
    # queries hold > 1,536 pairs) queries outgrow the workgroup tier's LDS
    # tables and re-run on global tables: 64 of them within the launch (the
    # regions a 1,000-query call may take), the rest in a re-run launch
    st = _overflow_case(tiny, 2.6, 1)
    on_global = (st[:, 7] & 8) > 0
    rerun = (st[:, 7] & 16) > 0
    assert 0 < on_global.sum() < len(st)
    assert (on_global & ~rerun).sum() == 64 and rerun.sum() > 0


def test_tier_overflow_small_tables(tiny):
    # the small workgroup tables (4,096 slots, 1,024 pairs) overflow earlier
    eps = tiny.eps * 2.2
    res = vj.vj_join(tiny.idx, eps, coop_tables=1)
    st = res.stats().cpu().numpy()
    ref = oracle.join(tiny.w.Q, tiny.w.X, tiny.g.adj, tiny.g.entry, eps, uncertain="out")
    refu = oracle.join(tiny.w.Q, tiny.w.X, tiny.g.adj, tiny.g.entry, eps, uncertain="in")
    assert ref.pairs() <= qx_set(_gpu_pairs(res)[0]) <= refu.pairs()
    assert ((st[:, 7] & 8) > 0).sum() > 0


def test_tier_overflow_chain(tiny):
    # the same from the one-wave tier: every query re-runs, some twice
    st = _overflow_case(tiny, 2.6, 0)
    assert np.all(st[:, 7] & 1) and 0 < ((st[:, 7] & 8) > 0).sum() < len(st)


def test_launch_order_keeps_results(tiny):
    # dense-first launch order (default) and the given order: same pairs and
    # the same per-query counters, by caller position, incl. a subset
    ids = torch.from_numpy(np.random.default_rng(8).permutation(1000)[:600].astype(np.int32)).cuda()
    for q in (None, ids):
        a = vj.vj_join(tiny.idx, tiny.eps * 1.5, query_ids=q, dense_first=1)
        b = vj.vj_join(tiny.idx, tiny.eps * 1.5, query_ids=q, dense_first=0)
        assert qx_set(_gpu_pairs(a)[0]) == qx_set(_gpu_pairs(b)[0])
        sa, sb = a.stats().cpu().numpy(), b.stats().cpu().numpy()
        assert np.array_equal(sa[:, :7], sb[:, :7])


def test_small_result_capacity_regrows(tiny):
    base = qx_set(_gpu_pairs(vj.vj_join(tiny.idx, tiny.eps))[0])
    res = vj.vj_join(tiny.idx, tiny.eps, pair_capacity=7)
    assert qx_set(_gpu_pairs(res)[0]) == base


def test_empty_and_nonpositive_eps(tiny):
    res = vj.vj_join(tiny.idx, 0.0)
    assert res.count() == 0
    res = vj.vj_join(tiny.idx, -1.0)
    assert res.count() == 0
    res = vj.vj_join(tiny.idx, tiny.eps, query_ids=torch.empty(0, dtype=torch.int32, device="cuda"))
    assert res.count() == 0


def test_invalid_arguments(tiny):
    with pytest.raises(vj.VJError) as e:
        vj.vj_join(tiny.idx, float("nan"))
    assert e.value.status == 1
    with pytest.raises(vj.VJError) as e:
        vj.vj_join(tiny.idx, tiny.eps, metric="ip")
    assert e.value.status == 2
    bad = torch.tensor([0, 5, tiny.w.Q.shape[0]], dtype=torch.int32, device="cuda")
    with pytest.raises(vj.VJError) as e:
        vj.vj_join(tiny.idx, tiny.eps, query_ids=bad)
    assert e.value.status == 1
    with pytest.raises(vj.VJError) as e:
        vj.vj_join(tiny.idx, tiny.eps, start_tier=3)
    assert e.value.status == 1


def _mode_parity(case, start_tier=1, coop_tables=0, **kw):
    w = case.w
    par = case.parent if kw.get("work_sharing", "self") != "self" else None
    ref = oracle.join(w.Q, w.X, case.g.adj, case.g.entry, case.eps, metric=w.metric,
                      parent=par, **kw)
    res = vj.vj_join(case.idx, case.eps, metric=w.metric, start_tier=start_tier,
                     coop_tables=coop_tables, **kw)
    qx, _ = _gpu_pairs(res)
    got, want = _by_query(qx), _by_query(zip(ref.qi, ref.xj))
    fragile = ref.stats[:, 7].astype(bool)
    mism = [q for q in range(w.Q.shape[0]) if not fragile[q] and got.get(q, set()) != want.get(q, set())]
    exact = oracle.nlj_counts(w.Q, w.X, case.eps, w.metric).sum()
    rec_gpu, rec_ref = len(qx) / exact, len(ref.qi) / exact
    print(f"[mode] {kw} fragile={fragile.mean():.4f} mism={len(mism)} "
          f"recall gpu={rec_gpu:.4f} oracle={rec_ref:.4f}", flush=True)
    assert not mism, f"{len(mism)} non-fragile queries differ, e.g. {mism[:5]}"
    assert abs(rec_gpu - rec_ref) <= 0.005
    return res, ref


@pytest.mark.parametrize("kw", [
    {"hybrid": "force"},
    {"hybrid": "adapt"},
    {"hybrid": "force", "hybrid_beam": 16, "conv_threshold": 3},
    {"work_sharing": "soft"},
    {"work_sharing": "hard"},
    {"work_sharing": "soft", "hybrid": "force"},
], ids=lambda k: "-".join(f"{a}={b}" for a, b in k.items()))
def test_modes_match_oracle(tiny, kw):
    res, ref = _mode_parity(tiny, **kw)
    st = res.stats().cpu().numpy()
    ok = ~ref.stats[:, 7].astype(bool)
    for col in (0, 2, 3, 6):
        assert np.array_equal(st[ok, col], ref.stats[ok, col]), col
    if kw.get("hybrid") == "adapt":
        ok = ~ref.stats[:, 7].astype(bool)
        assert np.array_equal(st[ok, 4], ref.stats[ok, 4])


@pytest.mark.parametrize("start_tier,coop_tables", [(0, 0), (2, 0), (1, 1)],
                         ids=["one-wave", "global", "small-lds"])
@pytest.mark.parametrize("kw", [
    {},
    {"hybrid": "force"},
    {"hybrid": "adapt"},
    {"hybrid": "force", "hybrid_beam": 16, "conv_threshold": 3},
    {"work_sharing": "soft", "hybrid": "force"},
    {"work_sharing": "hard"},
], ids=lambda k: "-".join(f"{a}={b}" for a, b in k.items()) or "bfs")
def test_other_tiers_match_oracle(tiny, kw, start_tier, coop_tables):
    # every query starts on the one-wave tier (0), on the global-table tier
    # (2), or on the workgroup tier with its small LDS tables, instead of the
    # default; per-query results and counters as with the default
    _say(f"vj_join tiny start_tier={start_tier} coop_tables={coop_tables} {kw}")
    res, ref = _mode_parity(tiny, start_tier=start_tier, coop_tables=coop_tables, **kw)
    st = res.stats().cpu().numpy()
    if start_tier == 2:
        assert np.all(st[:, 7] & 8)
    ok = ~ref.stats[:, 7].astype(bool)
    for col in (0, 2, 3, 6):  # pairs, expanded, out-range pops, visited data nodes
        assert np.array_equal(st[ok, col], ref.stats[ok, col]), col


def test_budget_mode(tiny):
    _budget_mode(tiny, 1)


@pytest.mark.parametrize("start_tier", [0, 2])
def test_budget_mode_other_tiers(tiny, start_tier):
    _budget_mode(tiny, start_tier)


def _budget_mode(tiny, start_tier):
    r = np.random.default_rng(11)
    b = r.integers(0, 8, size=tiny.w.Q.shape[0]).astype(np.int32)
    b[::7] = -1  # routed elsewhere: no traversal
    res = vj.vj_join(tiny.idx, tiny.eps, hybrid="budget", budget=torch.from_numpy(b).cuda(),
                     start_tier=start_tier)
    ref = oracle.join(tiny.w.Q, tiny.w.X, tiny.g.adj, tiny.g.entry, tiny.eps, hybrid="budget",
                      budget=np.maximum(b, 0))
    qx, _ = _gpu_pairs(res)
    got, want = _by_query(qx), _by_query(zip(ref.qi, ref.xj))
    st = res.stats().cpu().numpy()
    fragile = ref.stats[:, 7].astype(bool)
    for q in range(b.size):
        if b[q] < 0:
            assert q not in got and st[q, 7] & 2
        elif not fragile[q]:
            assert got.get(q, set()) == want.get(q, set())
            assert st[q, 3] <= b[q]


@pytest.fixture(scope="module")
def integer_case():
    w = workloads.config_mid(scale=0.01)  # 10,000 x 128 integer data, 1,000 queries
    eps = oracle.calibrate_eps(w.Q, w.X, w.target_matches, integer=True)
    print(f"[case] mid/100 nq={w.Q.shape[0]} nx={w.X.shape[0]} eps^2={eps * eps:.1f}", flush=True)
    return Case(w, eps)


@pytest.mark.parametrize("precision,start_tier", [("fp32", 1), ("u8", 1), ("auto", 1),
                                                  ("u8", 0), ("fp32", 0), ("u8", 2)])
def test_integer_data_exact(integer_case, precision, start_tier):
    c = integer_case
    res = vj.vj_join(c.idx, c.eps, precision=precision, start_tier=start_tier)
    ref = oracle.join(c.w.Q, c.w.X, c.g.adj, c.g.entry, c.eps)
    qx, dist = _gpu_pairs(res)
    assert qx_set(qx) == ref.pairs()  # squared distances are exact integers
    st = res.stats().cpu().numpy()
    assert np.array_equal(st[:, 6], ref.stats[:, 6])
    assert np.array_equal(st[:, 2], ref.stats[:, 2])


@pytest.mark.parametrize("kw", [{"hybrid": "adapt"}, {"work_sharing": "soft"},
                                {"work_sharing": "hard", "hybrid": "force"}])
def test_integer_data_modes_exact(integer_case, kw):
    c = integer_case
    par = c.parent if kw.get("work_sharing", "self") != "self" else None
    ref = oracle.join(c.w.Q, c.w.X, c.g.adj, c.g.entry, c.eps, parent=par, **kw)
    res = vj.vj_join(c.idx, c.eps, precision="u8", **kw)
    qx, _ = _gpu_pairs(res)
    got, want = _by_query(qx), _by_query(zip(ref.qi, ref.xj))
    fragile = ref.stats[:, 7].astype(bool)
    bad = [q for q in range(c.w.Q.shape[0]) if not fragile[q] and got.get(q, set()) != want.get(q, set())]
    assert not bad


@pytest.fixture(scope="module")
def ip_case():
    w = workloads.config_ood(scale=0.004)  # 8,000 x 768 unit vectors, 800 queries, IP
    eps = oracle.calibrate_eps(w.Q, w.X, w.target_matches, metric="ip")
    print(f"[case] ood/250 nq={w.Q.shape[0]} nx={w.X.shape[0]} eps={eps:.6f}", flush=True)
    return Case(w, eps)


def test_inner_product_bfs(ip_case):
    res = vj.vj_join(ip_case.idx, ip_case.eps, metric="ip")
    _check_sandwich(ip_case, res)


def test_inner_product_adapt(ip_case):
    _mode_parity(ip_case, hybrid="adapt")
