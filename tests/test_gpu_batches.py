"""GPU tests of the batch runner (vj_join_batches), the autotuner
(vj_autotune_join) and the reuse of the join's buffers between calls.

Batches of uneven sizes, each with its own eps, must give exactly the
result of a separate vj_join of the same queries, and each must satisfy the
oracle's sandwich; a tuned configuration must give the default result.
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


@pytest.fixture(scope="module")
def tiny():
    w = workloads.config_tiny()
    eps = oracle.calibrate_eps(w.Q, w.X, w.target_matches)
    g = oracle.build_merged(w.Q, w.X, w.R)
    idx = vj.vj_index_from_graph(torch.from_numpy(w.Q).cuda(), torch.from_numpy(w.X).cuda(),
                                 torch.from_numpy(g.adj).cuda(), g.entry)
    return w, eps, g, idx


def _set(res):
    qx, _ = res.export(sorted=True)
    return set(map(tuple, qx.cpu().numpy().tolist()))


def test_batches_equal_separate_joins(tiny):
    w, eps, g, idx = tiny
    starts = [0, 7, 300, 301, 650]
    counts = [7, 293, 1, 349, 350]
    eps_list = [eps * f for f in (1.3, 1.0, 0.7, 1.6, 2.6)]  # the last outgrows LDS tables
    res, ms = vj.vj_join_batches(idx, starts, counts, eps_list)
    assert len(res) == 5 and all(m > 0 for m in ms)
    for b, (st, ct, e) in enumerate(zip(starts, counts, eps_list)):
        ids = torch.arange(st, st + ct, dtype=torch.int32, device="cuda")
        one = vj.vj_join(idx, e, query_ids=ids)
        assert _set(res[b]) == _set(one)
        qids = np.arange(st, st + ct, dtype=np.int32)
        lo = oracle.join(w.Q, w.X, g.adj, g.entry, e, query_ids=qids, uncertain="out")
        hi = oracle.join(w.Q, w.X, g.adj, g.entry, e, query_ids=qids, uncertain="in")
        assert lo.pairs() <= _set(res[b]) <= hi.pairs()  # pairs carry Q indices


def test_batches_with_query_list(tiny):
    w, eps, g, idx = tiny
    perm = np.random.default_rng(4).permutation(w.Q.shape[0]).astype(np.int32)
    res, _ = vj.vj_join_batches(idx, [0, 500], [500, 500], [eps, eps * 1.2],
                                query_ids=torch.from_numpy(perm).cuda())
    for b, (st, e) in enumerate(((0, eps), (500, eps * 1.2))):
        one = vj.vj_join(idx, e, query_ids=torch.from_numpy(perm[st:st + 500]).cuda())
        assert _set(res[b]) == _set(one)


def test_batch_errors_keep_nothing(tiny):
    w, eps, g, idx = tiny
    with pytest.raises(vj.VJError):
        vj.vj_join_batches(idx, [0, 990], [10, 20], [eps, eps])  # beyond nq
    with pytest.raises(vj.VJError):
        vj.vj_join_batches(idx, [0], [10], [float("nan")])


def test_autotune_keeps_results(tiny):
    w, eps, g, idx = tiny
    params, ms = vj.vj_autotune_join(idx, eps)
    assert params.start_tier in (0, 1) and ms > 0
    assert _set(vj.vj_join(idx, eps, params=params)) == _set(vj.vj_join(idx, eps))


def test_buffers_reused_across_sizes(tiny):
    # a large call grows the index's buffers, a small one reuses them; each
    # result must stay valid after later calls
    w, eps, g, idx = tiny
    big = vj.vj_join(idx, eps * 2.0)
    small = vj.vj_join(idx, eps, query_ids=torch.arange(0, 50, dtype=torch.int32, device="cuda"))
    big_again = vj.vj_join(idx, eps * 2.0)
    assert _set(big) == _set(big_again)
    lo = oracle.join(w.Q, w.X, g.adj, g.entry, eps, query_ids=np.arange(50, dtype=np.int32),
                     uncertain="out")
    hi = oracle.join(w.Q, w.X, g.adj, g.entry, eps, query_ids=np.arange(50, dtype=np.int32),
                     uncertain="in")
    assert lo.pairs() <= _set(small) <= hi.pairs()
