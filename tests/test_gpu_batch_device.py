"""GPU tests of the device batch runner (vj_join_batches_device): batch steps
that read their parameters from device memory, with no host synchronisation
between batches, submitted by direct launches or as replayed HIP graphs.

Every batch must give the pair set of a separate vj_join of the same
queries at its eps (the traversal of a query does not depend on the batch
it runs in), satisfy the oracle's sandwich (BFS) or match the oracle on
every non-fragile query (ADAPT), and be bit-exact on integer data; queries
that outgrow the workgroup tier's tables must be re-run inside the replay
on global tables and, beyond those, on tables as large as the data set.
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


def _say(msg):
    print(f"[gpu-step] {msg}", flush=True)


def _set(res):
    qx, _ = res.export(sorted=True)
    return set(map(tuple, qx.cpu().numpy().tolist()))


def _by_query(pairs):
    out = {}
    for q, x in pairs:
        out.setdefault(int(q), set()).add(int(x))
    return out


class Case:
    def __init__(self, w, eps):
        self.w, self.eps = w, eps
        self.g = oracle.build_merged(w.Q, w.X, w.R)
        self.idx = vj.vj_index_from_graph(torch.from_numpy(w.Q).cuda(), torch.from_numpy(w.X).cuda(),
                                          torch.from_numpy(self.g.adj).cuda(), self.g.entry,
                                          metric=w.metric)


@pytest.fixture(scope="module")
def tiny():
    w = workloads.config_tiny()
    eps = oracle.calibrate_eps(w.Q, w.X, w.target_matches)
    _say(f"tiny nq={w.Q.shape[0]} nx={w.X.shape[0]} eps={eps:.6g}")
    return Case(w, eps)


RUNNERS = ["device", "graph"]


def _check_against_joins(case, starts, counts, eps_list, runner, query_ids=None, **kw):
    res, ms = vj.vj_join_batches(case.idx, starts, counts, eps_list, metric=case.w.metric,
                                 query_ids=query_ids, runner=runner, **kw)
    assert len(res) == len(starts)
    for b, (st, ct, e) in enumerate(zip(starts, counts, eps_list)):
        if query_ids is None:
            ids = torch.arange(st, st + ct, dtype=torch.int32, device="cuda")
        else:
            ids = query_ids[st:st + ct].contiguous()
        one = vj.vj_join(case.idx, e, metric=case.w.metric, query_ids=ids, **kw)
        assert res[b].count() == one.count(), b
        assert _set(res[b]) == _set(one), b
        sg, so = res[b].stats().cpu().numpy(), one.stats().cpu().numpy()
        assert sg.shape == (ct, 8)
        assert np.array_equal(sg[:, 0], so[:, 0]), b  # pairs per caller position
        if ct > 0 and (e > 0 or case.w.metric != "l2"):
            assert ms[b] > 0
    return res, ms


@pytest.mark.parametrize("runner", RUNNERS)
@pytest.mark.parametrize("dense_first", [1, 0])
def test_batches_equal_separate_joins(tiny, dense_first, runner):
    starts = [0, 7, 300, 301, 301, 650, 0]
    counts = [7, 293, 1, 0, 349, 350, 1000]
    f = (1.3, 1.0, 0.7, 1.0, 1.6, 2.6, -1.0)  # an empty batch, one that outgrows LDS, eps < 0
    eps_list = [tiny.eps * v for v in f]
    res, ms = _check_against_joins(tiny, starts, counts, eps_list, runner, dense_first=dense_first)
    assert res[3].count() == 0 and res[6].count() == 0
    assert not res[6].stats().any()
    tiers = res[5].tiers()
    _say(f"{runner} batches: device ms {[round(m, 3) for m in ms]}; "
         f"batch 5 re-runs {tiers[2]['queries']}")
    for b in (0, 1, 4):  # the oracle's sandwich (pairs carry Q indices)
        qids = np.arange(starts[b], starts[b] + counts[b], dtype=np.int32)
        lo = oracle.join(tiny.w.Q, tiny.w.X, tiny.g.adj, tiny.g.entry, eps_list[b], query_ids=qids,
                         uncertain="out")
        hi = oracle.join(tiny.w.Q, tiny.w.X, tiny.g.adj, tiny.g.entry, eps_list[b], query_ids=qids,
                         uncertain="in")
        assert lo.pairs() <= _set(res[b]) <= hi.pairs()


@pytest.mark.parametrize("runner", RUNNERS)
def test_batches_rerun_on_global_tables(tiny, runner):
    # large eps: many queries outgrow the LDS tables and the promotion regions
    # (64 for these batch sizes), so the replay's re-run launch takes them
    n = tiny.w.Q.shape[0]
    res, _ = _check_against_joins(tiny, [0, 500], [500, n - 500], [tiny.eps * 3.5, tiny.eps * 3.0],
                                  runner)
    t = [r.tiers() for r in res]
    _say(f"re-runs on global tables: {[x[2]['queries'] for x in t]}")
    assert sum(x[2]["queries"] for x in t) > 0


@pytest.mark.parametrize("runner", RUNNERS)
def test_batches_query_list_and_small_capacity(tiny, runner):
    perm = np.random.default_rng(4).permutation(tiny.w.Q.shape[0]).astype(np.int32)
    ids = torch.from_numpy(perm).cuda()
    _check_against_joins(tiny, [0, 500, 100], [500, 500, 37], [tiny.eps, tiny.eps * 1.2, tiny.eps],
                         runner, query_ids=ids)
    # a pair capacity far too small regrows and runs again
    _check_against_joins(tiny, [0, 10], [10, 990], [tiny.eps, tiny.eps * 1.5], runner,
                         pair_capacity=16)


def test_many_batches_and_kept_graphs(tiny):
    # 37 batches: graphs of 16 steps, the last padded with steps that run
    # nothing; shapes alternate so kept graphs are replaced and re-made
    rng = np.random.default_rng(9)
    n = tiny.w.Q.shape[0]
    counts = rng.integers(0, 60, size=37).tolist()
    starts = [int(rng.integers(0, n - c + 1)) for c in counts]
    eps_list = (tiny.eps * rng.uniform(0.5, 2.0, size=37)).tolist()
    direct, _ = vj.vj_join_batches(tiny.idx, starts, counts, eps_list, runner="device")
    for shape in range(3):
        if shape == 1:
            _check_against_joins(tiny, [0, 100], [100, 400], [tiny.eps, tiny.eps], "graph")
            continue
        res, ms = vj.vj_join_batches(tiny.idx, starts, counts, eps_list, runner="graph")
        assert len(res) == 37
        for b in range(37):
            assert _set(res[b]) == _set(direct[b]), b
    for b in (0, 5, 36):
        ids = torch.arange(starts[b], starts[b] + counts[b], dtype=torch.int32, device="cuda")
        assert _set(direct[b]) == _set(vj.vj_join(tiny.idx, eps_list[b], query_ids=ids))


@pytest.mark.parametrize("runner", RUNNERS)
@pytest.mark.parametrize("hybrid", ["adapt", "force"])
def test_batches_hybrid_matches_oracle(tiny, runner, hybrid):
    w = tiny.w
    n = w.Q.shape[0]
    res, _ = vj.vj_join_batches(tiny.idx, [0, 123, 600], [123, 477, n - 600], [tiny.eps] * 3,
                                runner=runner, hybrid=hybrid)
    got = {}
    for r in res:
        for q, xs in _by_query(r.export(sorted=True)[0].cpu().numpy().tolist()).items():
            got[q] = xs
    ref = oracle.join(w.Q, w.X, tiny.g.adj, tiny.g.entry, tiny.eps, hybrid=hybrid)
    want = _by_query(zip(ref.qi.tolist(), ref.xj.tolist()))
    fragile = ref.stats[:, 7].astype(bool)
    mism = [q for q in range(n) if not fragile[q] and got.get(q, set()) != want.get(q, set())]
    _say(f"{runner} {hybrid}: fragile {fragile.mean():.4f}, mismatches {len(mism)}")
    assert not mism, f"{len(mism)} non-fragile queries differ, e.g. {mism[:5]}"


@pytest.mark.parametrize("runner", RUNNERS)
def test_batches_errors(tiny, runner):
    with pytest.raises(vj.VJError):
        vj.vj_join_batches(tiny.idx, [0], [10], [tiny.eps], runner=runner, work_sharing="soft")
    with pytest.raises(vj.VJError):
        vj.vj_join_batches(tiny.idx, [0, 990], [10, 20], [tiny.eps] * 2, runner=runner)
    bad = torch.tensor([0, 1, 10 ** 6], dtype=torch.int32, device="cuda")
    with pytest.raises(vj.VJError):
        vj.vj_join_batches(tiny.idx, [0], [3], [tiny.eps], query_ids=bad, runner=runner)
    res, ms = vj.vj_join_batches(tiny.idx, [], [], [], runner=runner)
    assert res == [] and ms == []
    # the index still joins after the errors
    one, _ = vj.vj_join_batches(tiny.idx, [0], [50], [tiny.eps], runner=runner)
    assert _set(one[0]) == _set(vj.vj_join(tiny.idx, tiny.eps,
                                           query_ids=torch.arange(50, dtype=torch.int32,
                                                                  device="cuda")))


@pytest.fixture(scope="module")
def integer_case():
    w = workloads.config_mid(scale=0.01)  # 10,000 x 128 integer data, 1,000 queries
    eps = oracle.calibrate_eps(w.Q, w.X, w.target_matches, integer=True)
    _say(f"mid/100 nq={w.Q.shape[0]} nx={w.X.shape[0]} eps^2={eps * eps:.1f}")
    return Case(w, eps)


@pytest.mark.parametrize("runner", RUNNERS)
@pytest.mark.parametrize("precision", ["u8", "fp32", "bf16"])
def test_batches_integer_exact(integer_case, precision, runner):
    c = integer_case
    n = c.w.Q.shape[0]
    starts, counts = [0, 1, 300], [1, 299, n - 300]
    res, _ = vj.vj_join_batches(c.idx, starts, counts, [c.eps] * 3, runner=runner,
                                precision=precision)
    got = set()
    for r in res:
        got |= _set(r)
    ref = oracle.join(c.w.Q, c.w.X, c.g.adj, c.g.entry, c.eps)
    assert got == ref.pairs()  # squared distances are exact integers


@pytest.mark.parametrize("runner", RUNNERS)
def test_batches_full_size_tables(runner):
    # every data node in range: a query's closure outgrows the global tables
    # (2^16 slots, 32,768 pairs) and goes to tables as large as the data set
    w = workloads.config_mid(scale=0.05)  # 50,000 x 128
    Q, X = torch.from_numpy(w.Q).cuda(), torch.from_numpy(w.X).cuda()
    _say(f"mid/20 nq={w.Q.shape[0]} nx={w.X.shape[0]}: build")
    idx = vj.vj_build_merged_index(Q, X, R=w.R)
    eps = 1e9
    res, _ = vj.vj_join_batches(idx, [0, 4], [4, 4], [eps, eps], runner=runner)
    for b, st in enumerate((0, 4)):
        ids = torch.arange(st, st + 4, dtype=torch.int32, device="cuda")
        one = vj.vj_join(idx, eps, query_ids=ids)
        assert _set(res[b]) == _set(one)
        t = res[b].tiers()
        _say(f"batch {b}: tier queries {[x['queries'] for x in t]}, pairs {res[b].count()}")
        assert t[3]["queries"] > 0
