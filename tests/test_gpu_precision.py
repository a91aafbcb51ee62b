"""GPU parity of the precision form of the join (vj_join with bf16 rows).

The query row stays fp32; data rows are read as bf16.  By the triangle
inequality |q - x~| differs from |q - x| by at most |x - x~| <= 2^-8 |x|,
and the fp32 sums add a bounded relative error; a candidate whose bf16
value lies inside that margin of eps is re-decided from the fp32 rows in
the fp32 kernels' own arithmetic.  Hence in threshold-only modes (BFS, hard
work sharing) the bf16 pair set must EQUAL the fp32 pair set, and both must
satisfy the oracle's sandwich.  Modes that order candidates by distance
(hybrid queue, soft cache, d1/d2) use the bf16 values for the order, so
there only recall is compared (within 0.5 points of fp32).

Each case also reports the FP64 error of the reported distances: max and
mean |d_reported - d64| / eps, and the share of candidates re-checked.
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
U_BF16 = 2.0 ** -8


class Case:
    def __init__(self, name, w, eps):
        self.name = name
        self.w = w
        self.eps = eps
        self.g = oracle.build_merged(w.Q, w.X, w.R)
        self.parent, _, _ = oracle.mst_parents(w.Q, w.X, self.g.adj, self.g.entry)
        self.idx = vj.vj_index_from_graph(torch.from_numpy(w.Q).cuda(), torch.from_numpy(w.X).cuda(),
                                          torch.from_numpy(self.g.adj).cuda(), self.g.entry,
                                          metric=w.metric,
                                          parent=torch.from_numpy(self.parent).cuda())


def _make(name):
    if name == "tiny":  # d = 32 Gaussian mixture: values not exact in bf16
        w = workloads.config_tiny()
    elif name == "highdim":  # 10,000 x 960 Beta mixture in [0, 1]
        w = workloads.config_highdim(scale=0.01)
    elif name == "ood_ip":  # 8,000 x 768 unit vectors, inner product
        w = workloads.config_ood(scale=0.004)
    else:  # 10,000 x 128 integers in [0, 218]: exact in bf16
        w = workloads.config_mid(scale=0.01)
    eps = oracle.calibrate_eps(w.Q, w.X, w.target_matches, w.metric,
                               integer=bool(w.meta.get("integer")))
    print(f"[case] {name} nq={w.Q.shape[0]} nx={w.X.shape[0]} d={w.d} {w.metric} eps={eps:.6g}",
          flush=True)
    return Case(name, w, eps)


_cache = {}


def case(name):
    if name not in _cache:
        _cache[name] = _make(name)
    return _cache[name]


def _pairs(res):
    qx, dist = res.export(sorted=True)
    return qx.cpu().numpy(), dist.cpu().numpy()


def _set(qx):
    return set(map(tuple, np.asarray(qx).tolist()))


def _error_report(c, qx, dist, res, label):
    if len(qx) == 0:
        return 0.0
    d64 = oracle.pair_dists(c.w.Q, c.w.X, qx[:, 0], qx[:, 1], c.w.metric)
    err = np.abs(dist.astype(np.float64) - d64) / c.eps
    xn = np.linalg.norm(c.w.X[qx[:, 1]].astype(np.float64), axis=1)
    bound = U_BF16 * xn / (1 - U_BF16) / c.eps if c.w.metric == "l2" else \
        U_BF16 * xn * np.linalg.norm(c.w.Q[qx[:, 0]].astype(np.float64), axis=1) / c.eps
    print(f"[precision] {c.name} {label}: pairs={len(qx)} rechecked={res.rechecked()} "
          f"max|d-d64|/eps={err.max():.3e} mean={err.mean():.3e} "
          f"max bound u|x|/eps={bound.max():.3e}", flush=True)
    assert np.all(err <= bound * 1.01 + 1e-5)
    return err.max()


@pytest.mark.parametrize("name", ["tiny", "highdim", "ood_ip", "integer"])
def test_bf16_bfs_equals_fp32(name):
    c = case(name)
    r32 = vj.vj_join(c.idx, c.eps, metric=c.w.metric, precision="fp32")
    r16 = vj.vj_join(c.idx, c.eps, metric=c.w.metric, precision="bf16")
    qx32, _ = _pairs(r32)
    qx16, d16 = _pairs(r16)
    assert _set(qx16) == _set(qx32)
    lo = oracle.join(c.w.Q, c.w.X, c.g.adj, c.g.entry, c.eps, metric=c.w.metric,
                     uncertain="out", uncertain_rel=REL).pairs()
    hi = oracle.join(c.w.Q, c.w.X, c.g.adj, c.g.entry, c.eps, metric=c.w.metric,
                     uncertain="in", uncertain_rel=REL).pairs()
    assert lo <= _set(qx16) <= hi
    st32, st16 = r32.stats().cpu().numpy(), r16.stats().cpu().numpy()
    assert np.array_equal(st32[:, [0, 2, 6]], st16[:, [0, 2, 6]])
    err = _error_report(c, qx16, d16, r16, "bfs")
    if name == "integer":
        # integers in [0, 218] are exact in bf16: the only margin left is the
        # fp32 summation bound, and the reported distances are exact in fp32
        assert err < 1e-6


def test_bf16_hard_mode_equals_fp32():
    c = case("tiny")
    r32 = vj.vj_join(c.idx, c.eps, precision="fp32", work_sharing="hard")
    r16 = vj.vj_join(c.idx, c.eps, precision="bf16", work_sharing="hard")
    assert _set(_pairs(r16)[0]) == _set(_pairs(r32)[0])


def test_bf16_wide_eps_equals_fp32():
    # 2.6x eps: large in-range sets, tier overflow and in-launch promotion
    c = case("tiny")
    r32 = vj.vj_join(c.idx, c.eps * 2.6, precision="fp32")
    r16 = vj.vj_join(c.idx, c.eps * 2.6, precision="bf16")
    assert _set(_pairs(r16)[0]) == _set(_pairs(r32)[0])
    st = r16.stats().cpu().numpy()
    assert ((st[:, 7] & 8) > 0).sum() > 0


@pytest.mark.parametrize("kw", [{"hybrid": "force"}, {"hybrid": "adapt"},
                                {"work_sharing": "soft"}],
                         ids=lambda k: "-".join(f"{a}={b}" for a, b in k.items()))
def test_bf16_ordered_modes_recall(kw):
    c = case("tiny")
    exact = oracle.nlj_counts(c.w.Q, c.w.X, c.eps, c.w.metric).sum()
    r32 = vj.vj_join(c.idx, c.eps, precision="fp32", **kw)
    r16 = vj.vj_join(c.idx, c.eps, precision="bf16", **kw)
    rec32, rec16 = r32.count() / exact, r16.count() / exact
    qx16, _ = _pairs(r16)
    print(f"[precision] tiny {kw}: recall fp32={rec32:.4f} bf16={rec16:.4f}", flush=True)
    # precision stays 1: every pair is within eps (up to the fp32 band)
    d64 = oracle.pair_dists(c.w.Q, c.w.X, qx16[:, 0], qx16[:, 1], c.w.metric)
    assert np.all(d64 < c.eps * (1 + REL))
    assert abs(rec16 - rec32) <= 0.005


def test_bf16_one_wave_tier_request_runs_on_workgroup_tier():
    c = case("tiny")
    r = vj.vj_join(c.idx, c.eps, precision="bf16", start_tier=0)
    st = r.stats().cpu().numpy()
    assert np.all(st[:, 7] & 1)
    assert _set(_pairs(r)[0]) == _set(_pairs(vj.vj_join(c.idx, c.eps, precision="fp32"))[0])
