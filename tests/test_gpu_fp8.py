"""GPU parity of the fp8 (OCP e4m3) precision form of the join.

Data rows are read as e4m3 codes with a power-of-two scale per row; the
query row stays fp32.  The library stores, per row, a bound on |x - x~|
computed in fp64 at quantisation; by the triangle inequality |q - x~| and
|q - x| differ by at most that bound, so a candidate whose fp8 value lies
inside it (plus the fp32 summation bound) of eps is re-decided from the
fp32 rows in the fp32 kernels' arithmetic.  Threshold-only modes (BFS, hard
work sharing) must therefore give the fp32 pair set exactly, on every
workload shape; ordered modes are compared by recall (within 0.5 points).
Each case reports max |d_reported - d64| / eps and the share re-checked.
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
_cache = {}


def case(name):
    if name in _cache:
        return _cache[name]
    if name == "tiny":
        w = workloads.config_tiny()
    elif name == "highdim":
        w = workloads.config_highdim(scale=0.01)
    elif name == "ood_ip":
        w = workloads.config_ood(scale=0.004)
    elif name == "stream":  # d = 96 Gaussian mixture, the stream workload's shape
        w = workloads.config_stream(scale=0.001, n_batches=4)
    else:
        w = workloads.config_mid(scale=0.01)
    eps = oracle.calibrate_eps(w.Q, w.X, 10.0 if name == "stream" else w.target_matches,
                               w.metric, integer=bool(w.meta.get("integer")))
    g = oracle.build_merged(w.Q, w.X, w.R)
    print(f"[case] {name} nq={w.Q.shape[0]} nx={w.X.shape[0]} d={w.d} eps={eps:.6g}", flush=True)
    idx = vj.vj_index_from_graph(torch.from_numpy(w.Q).cuda(), torch.from_numpy(w.X).cuda(),
                                 torch.from_numpy(g.adj).cuda(), g.entry, metric=w.metric)
    _cache[name] = (w, eps, g, idx)
    return _cache[name]


def _pairs(res):
    qx, d = res.export(sorted=True)
    return qx.cpu().numpy(), d.cpu().numpy()


def _set(qx):
    return set(map(tuple, np.asarray(qx).tolist()))


@pytest.mark.parametrize("name", ["tiny", "highdim", "ood_ip", "stream", "integer"])
def test_fp8_bfs_equals_fp32(name):
    w, eps, g, idx = case(name)
    r32 = vj.vj_join(idx, eps, metric=w.metric, precision="fp32")
    r8 = vj.vj_join(idx, eps, metric=w.metric, precision="fp8")
    qx32, _ = _pairs(r32)
    qx8, d8 = _pairs(r8)
    assert _set(qx8) == _set(qx32)
    lo = oracle.join(w.Q, w.X, g.adj, g.entry, eps, metric=w.metric, uncertain="out",
                     uncertain_rel=REL).pairs()
    hi = oracle.join(w.Q, w.X, g.adj, g.entry, eps, metric=w.metric, uncertain="in",
                     uncertain_rel=REL).pairs()
    assert lo <= _set(qx8) <= hi
    st32, st8 = r32.stats().cpu().numpy(), r8.stats().cpu().numpy()
    assert np.array_equal(st32[:, [0, 2, 6]], st8[:, [0, 2, 6]])
    if len(qx8):
        d64 = oracle.pair_dists(w.Q, w.X, qx8[:, 0], qx8[:, 1], w.metric)
        err = np.abs(d8.astype(np.float64) - d64) / eps
        # e4m3 keeps 3 mantissa bits: |x - x~| <= 2^-4 |x| in the normal
        # range, plus the subnormal step of the row's scale
        xn = np.linalg.norm(w.X[qx8[:, 1]].astype(np.float64), axis=1)
        scale = 2.0 * np.abs(w.X[qx8[:, 1]]).max(axis=1) / 448.0
        bound = 2.0 ** -4 * xn + scale * 2.0 ** -10 * np.sqrt(w.d)
        if w.metric == "ip":
            bound = bound * np.linalg.norm(w.Q[qx8[:, 0]].astype(np.float64), axis=1)
        print(f"[fp8] {name}: pairs={len(qx8)} rechecked={r8.rechecked()} "
              f"(of {int(st8[:, 1].sum())} evaluations) max|d-d64|/eps={err.max():.3e} "
              f"mean={err.mean():.3e}", flush=True)
        assert np.all(err <= bound / eps * 1.01 + 1e-5)


def test_fp8_hard_mode_and_wide_eps_equal_fp32():
    w, eps, g, idx = case("tiny")
    for kw, e in (({"work_sharing": "hard"}, eps), ({}, eps * 2.6)):
        r32 = vj.vj_join(idx, e, precision="fp32", **kw)
        r8 = vj.vj_join(idx, e, precision="fp8", **kw)
        assert _set(_pairs(r8)[0]) == _set(_pairs(r32)[0]), kw


@pytest.mark.parametrize("kw", [{"hybrid": "force"}, {"hybrid": "adapt"}, {"work_sharing": "soft"}],
                         ids=lambda k: "-".join(f"{a}={b}" for a, b in k.items()))
def test_fp8_ordered_modes_recall(kw):
    w, eps, g, idx = case("tiny")
    exact = oracle.nlj_counts(w.Q, w.X, eps, w.metric).sum()
    r32 = vj.vj_join(idx, eps, precision="fp32", **kw)
    r8 = vj.vj_join(idx, eps, precision="fp8", **kw)
    rec32, rec8 = r32.count() / exact, r8.count() / exact
    qx8, _ = _pairs(r8)
    d64 = oracle.pair_dists(w.Q, w.X, qx8[:, 0], qx8[:, 1], w.metric)
    assert np.all(d64 < eps * (1 + REL))
    print(f"[fp8] tiny {kw}: recall fp32={rec32:.4f} fp8={rec8:.4f}", flush=True)
    assert abs(rec8 - rec32) <= 0.005


def test_fp8_separate_and_build_copy():
    # the precision form applies to separate indexes too (copies & 2 makes
    # the fp8 rows at build time); the best-first greedy queue orders and
    # stops by its keys, so every node the greedy phase visits is re-decided
    # from the fp32 rows: the greedy path is the fp32 one, and the pair sets
    # equal the fp32 sets
    w = workloads.config_tiny(scale=0.3)
    eps = oracle.calibrate_eps(w.Q, w.X, w.target_matches)
    idx = vj.vj_build_separate_index(torch.from_numpy(w.Q).cuda(), torch.from_numpy(w.X).cuda(),
                                     R=16, copies=2)
    for ws in ("none", "hard"):
        a = _set(_pairs(vj.vj_join(idx, eps, precision="fp32", work_sharing=ws))[0])
        b = _set(_pairs(vj.vj_join(idx, eps, precision="fp8", work_sharing=ws))[0])
        c = _set(_pairs(vj.vj_join(idx, eps, precision="bf16", work_sharing=ws))[0])
        assert a == b == c, ws
    # soft work sharing caches an arg-min over the visited keys: an ordered
    # decision, compared by recall as in the merged index
    exact = oracle.nlj_counts(w.Q, w.X, eps).sum()
    r32 = vj.vj_join(idx, eps, precision="fp32", work_sharing="soft").count() / exact
    r8 = vj.vj_join(idx, eps, precision="fp8", work_sharing="soft").count() / exact
    print(f"[fp8] separate soft: recall fp32={r32:.4f} fp8={r8:.4f}", flush=True)
    assert abs(r32 - r8) <= 0.005
