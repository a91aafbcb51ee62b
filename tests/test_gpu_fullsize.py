"""Parity at the benchmark's full size: X = 1,000,000 and Q = 100,000 integer
vectors (d = 128, R = 32), the configuration bench.py times (GPU-built
merged index, default join parameters, fp32 and u8 rows).

The oracle cannot build the graph or join every query at this size, so the
check uses sampled outputs and properties that hold at any size:
* for 2,000 sampled queries, fp64 distances to all of X (numpy) give the exact
  in-range sets: every GPU pair is in them (precision 1) and the GPU's
  reported distances are exact (integer data: fp32 squared distances are
  exact);
* BFS mode returns, per query, the in-range data nodes reachable from the
  in-range data nodes among {s} + N(q) through in-range data nodes of the
  index's own graph; the sampled queries' GPU sets must equal that closure
  computed here in fp64;
* the exact MFMA brute-force join agrees with the fp64 sets of the samples.
"""
import json
import os
from collections import deque

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2603_16360_amd import vj  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def mid():
    w = workloads.config_mid()
    eps = json.load(open(os.path.join(HERE, "golden", "eps.json")))["mid"]["eps"]
    print(f"[case] mid full size nq={w.Q.shape[0]} nx={w.X.shape[0]} eps={eps}", flush=True)
    Q = torch.from_numpy(w.Q).cuda()
    X = torch.from_numpy(w.X).cuda()
    idx = vj.vj_build_merged_index(Q, X, R=w.R)
    adj, _, _ = idx.export_graph()
    return w, eps, Q, X, idx, adj.cpu().numpy()


def _exact_dists(w, sample):
    """fp64 distances from every data row to the sampled queries: on this
    integer data |x|^2 + |q|^2 - 2 x.q is exact in fp64 (all terms are
    integers below 2^53)."""
    Xd = w.X.astype(np.float64)
    Qs = w.Q[sample].astype(np.float64)
    D2 = (Xd * Xd).sum(1)[:, None] + (Qs * Qs).sum(1)[None, :] - 2.0 * (Xd @ Qs.T)
    return np.sqrt(np.maximum(D2, 0.0))


def _closure(w, adj, entry, eps, qi, d64):
    nx = w.X.shape[0]
    inr = d64 < eps
    u = nx + qi
    start = [v for v in [entry] + adj[u].tolist() if 0 <= v < nx and inr[v]]
    seen = set(start)
    dq = deque(start)
    while dq:
        a = dq.popleft()
        for v in adj[a].tolist():
            if 0 <= v < nx and inr[v] and v not in seen:
                seen.add(v)
                dq.append(v)
    return seen


def test_fullsize_sampled_queries(mid):
    w, eps, Q, X, idx, adj = mid
    entry = idx.info()["entry"]
    rng = np.random.default_rng(17)
    sample = np.sort(rng.choice(w.Q.shape[0], size=2000, replace=False))
    results = {}
    for precision in ("fp32", "u8"):
        qx, dist = vj.vj_join(idx, eps, precision=precision).export(sorted=True)
        qx, dist = qx.cpu().numpy(), dist.cpu().numpy()
        results[precision] = (qx, dist, np.searchsorted(qx[:, 0], sample, side="left"),
                              np.searchsorted(qx[:, 0], sample, side="right"))
    n_exact = 0
    n_got = {p: 0 for p in results}
    for c0 in range(0, sample.size, 250):  # 250 queries' distances at a time (2 GB)
        chunk = sample[c0:c0 + 250]
        D = _exact_dists(w, chunk)
        for j, qi in enumerate(chunk.tolist()):
            d64 = D[:, j]
            exact = set(np.nonzero(d64 < eps)[0].tolist())
            closure = _closure(w, adj, entry, eps, qi, d64)
            n_exact += len(exact)
            for precision, (qx, dist, starts, ends) in results.items():
                a, b = int(starts[c0 + j]), int(ends[c0 + j])
                got = set(qx[a:b, 1].tolist())
                assert got <= exact, (precision, qi)              # precision 1
                assert got == closure, (precision, qi)            # BFS closure
                np.testing.assert_allclose(dist[a:b], d64[qx[a:b, 1]], rtol=1e-6)
                n_got[precision] += len(got)
    for precision in results:
        print(f"[fullsize] {precision}: sampled recall {n_got[precision] / max(1, n_exact):.4f} "
              f"({n_got[precision]} of {n_exact} pairs, {sample.size} queries)", flush=True)


def test_fullsize_bruteforce_sampled(mid):
    w, eps, Q, X, idx, adj = mid
    rng = np.random.default_rng(18)
    sample = np.sort(rng.choice(w.Q.shape[0], size=32, replace=False))
    gt = vj.vj_bruteforce_join(Q[torch.from_numpy(sample).cuda().long()].contiguous(), X, eps,
                               precision="bf16")
    qx, _ = gt.export(sorted=True)
    qx = qx.cpu().numpy()
    D = _exact_dists(w, sample)
    for j, qi in enumerate(sample.tolist()):
        want = set(np.nonzero(D[:, j] < eps)[0].tolist())
        assert set(qx[qx[:, 0] == j, 1].tolist()) == want
