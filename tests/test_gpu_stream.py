"""Parity on the stream workload (d = 96, 1,024-cluster Gaussian mixture,
uneven batches, each with its own eps) at a small scale: X = 40,000 rows and
12 batches, on the GPU-built merged index.

Per batch, eps comes from the oracle's calibration on that batch's queries.
For 16 sampled queries of every batch, fp64 distances to all of X (numpy)
bound the result.  The data are floats, so a pair whose distance lies within
1e-5 eps of eps may go either way, i.e. within a relative 2e-5 of eps^2:
* every GPU pair lies within eps^2 (1 + 2e-5) (precision 1);
* the GPU set lies between the BFS closures (in-range data nodes reachable
  from the in-range nodes among {s} + N(q) through in-range data nodes of the
  index's graph) taken at eps^2 (1 - 2e-5) and eps^2 (1 + 2e-5).
All three batch runners (one vj_join per batch, device-driven with direct
launches, HIP graph replay) must give these bounds and the same pair sets.
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

REL = 2e-5  # (1 +- 1e-5)^2 - 1 on eps^2, to first order


@pytest.fixture(scope="module")
def stream():
    w = workloads.config_stream(scale=0.004, n_batches=12)
    batches = workloads.stream_batches(w)
    eps = [oracle.calibrate_eps(w.Q[st:st + ct], w.X, tgt) for st, ct, tgt in batches]
    print(f"[case] stream/250 nq={w.Q.shape[0]} nx={w.X.shape[0]} batches={[b[1] for b in batches]}",
          flush=True)
    Q = torch.from_numpy(w.Q).cuda()
    X = torch.from_numpy(w.X).cuda()
    idx = vj.vj_build_merged_index(Q, X, R=w.R)
    adj, _, _ = idx.export_graph()
    return w, batches, eps, idx, adj.cpu().numpy(), idx.info()["entry"]


def _closure(nx, adj, entry, u, inr):
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


def _by_query(res):
    qx, _ = res.export(sorted=True)
    out = {}
    for q, x in qx.cpu().numpy().tolist():
        out.setdefault(q, set()).add(x)
    return out


@pytest.mark.parametrize("runner", ["host", "device", "graph"])
def test_stream_batches_sampled(stream, runner):
    w, batches, eps, idx, adj, entry = stream
    starts = [b[0] for b in batches]
    counts = [b[1] for b in batches]
    res, ms = vj.vj_join_batches(idx, starts, counts, eps, runner=runner)
    nx = w.X.shape[0]
    Xd = w.X.astype(np.float64)
    xn = (Xd * Xd).sum(1)
    rng = np.random.default_rng(31)
    checked = 0
    for b, (st, ct, _) in enumerate(batches):
        got = _by_query(res[b])
        e2 = float(eps[b]) ** 2
        sample = np.sort(rng.choice(ct, size=min(16, ct), replace=False))
        qs = w.Q[st + sample].astype(np.float64)
        D2 = xn[:, None] + (qs * qs).sum(1)[None, :] - 2.0 * (Xd @ qs.T)
        for j, qi in enumerate((st + sample).tolist()):
            g = got.get(qi, set())
            d2 = D2[:, j]
            assert all(d2[x] < e2 * (1 + REL) for x in g), (b, qi)
            u = nx + qi
            lo = _closure(nx, adj, entry, u, d2 < e2 * (1 - REL))
            hi = _closure(nx, adj, entry, u, d2 < e2 * (1 + REL))
            assert lo <= g <= hi, (b, qi, len(lo), len(g), len(hi))
            checked += 1
    print(f"[stream] {runner}: {checked} sampled queries in {len(batches)} batches, "
          f"{sum(r.count() for r in res)} pairs", flush=True)


def test_stream_runners_agree(stream):
    w, batches, eps, idx, adj, entry = stream
    starts = [b[0] for b in batches]
    counts = [b[1] for b in batches]
    sets = {}
    for runner in ("host", "device", "graph"):
        res, _ = vj.vj_join_batches(idx, starts, counts, eps, runner=runner)
        sets[runner] = [_by_query(r) for r in res]
    assert sets["device"] == sets["host"]
    assert sets["graph"] == sets["host"]
