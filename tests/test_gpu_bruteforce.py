"""GPU parity of the MFMA brute-force join (vj_bruteforce_join) with the
oracle's exact nested-loop join (Definition 1).

Rule: the GPU pair set equals the oracle's, except pairs whose fp64
distance lies within 1e-5*eps of eps (the eps handed to the library is
rounded to fp32).  Integer data in [0, 218] is exact in bf16 and the sets
must then be identical.  Reported distances are the fp64 re-check rounded to
fp32.
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


def _gpu(Q, X, eps, metric="l2", precision="fp32"):
    print(f"[gpu-step] bruteforce nq={Q.shape[0]} nx={X.shape[0]} d={Q.shape[1]} "
          f"{metric} {precision}", flush=True)
    r = vj.vj_bruteforce_join(torch.from_numpy(Q).cuda(), torch.from_numpy(X).cuda(), eps,
                              metric=metric, precision=precision)
    qx, d = r.export(sorted=True)
    return qx.cpu().numpy(), d.cpu().numpy()


def _check(Q, X, eps, metric, precision, exact=False):
    qx, d = _gpu(Q, X, eps, metric, precision)
    G = set(map(tuple, qx.tolist()))
    oq, ox, od = oracle.nlj(Q, X, eps, metric)
    O = set(zip(oq.tolist(), ox.tolist()))
    if exact:
        assert G == O
    else:
        diff = G ^ O
        if diff:
            a = np.array(sorted(diff), dtype=np.int32)
            dd = oracle.pair_dists(Q, X, a[:, 0], a[:, 1], metric)
            assert np.all(np.abs(dd - eps) <= 1e-5 * abs(eps)), (len(diff), dd[:5], eps)
    # sorted by (query, data), distances = fp64 values rounded to fp32
    key = qx[:, 0].astype(np.int64) * (X.shape[0] + 1) + qx[:, 1]
    assert np.all(np.diff(key) > 0)
    if len(qx):
        ref = oracle.pair_dists(Q, X, qx[:, 0], qx[:, 1], metric)
        np.testing.assert_allclose(d, ref.astype(np.float32), rtol=1e-6, atol=1e-6)
    return G, O


@pytest.mark.parametrize("metric", ["l2", "ip"])
@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_ragged_small(metric, precision):
    r = np.random.default_rng(7)
    Q = r.standard_normal((37, 50)).astype(np.float32)
    X = r.standard_normal((203, 50)).astype(np.float32)
    if metric == "ip":
        Q /= np.linalg.norm(Q, axis=1, keepdims=True)
        X /= np.linalg.norm(X, axis=1, keepdims=True)
    D = oracle.dist_matrix(Q, X, metric)
    eps = float(np.quantile(D, 0.1))
    G, O = _check(Q, X, eps, metric, precision)
    assert len(O) > 100


def test_single_rows():
    Q = np.array([[1.0, 2.0, 3.0]], np.float32)
    X = np.array([[1.0, 2.0, 3.5]], np.float32)
    G, O = _check(Q, X, 0.6, "l2", "fp32", exact=True)
    assert G == {(0, 0)}
    G, O = _check(Q, X, 0.4, "l2", "fp32", exact=True)
    assert G == set()


def test_tiny_config_all_pairs():
    w = workloads.config_tiny()
    eps = oracle.calibrate_eps(w.Q, w.X, w.target_matches)
    G, O = _check(w.Q, w.X, eps, "l2", "fp32")
    assert abs(len(G) - 10_000) <= 2


def test_integer_data_exact():
    w = workloads.config_mid(scale=0.01)
    eps = oracle.calibrate_eps(w.Q, w.X, w.target_matches, integer=True)
    for precision in ("bf16", "fp32"):
        _check(w.Q, w.X, eps, "l2", precision, exact=True)


def test_unit_vectors_inner_product():
    w = workloads.config_ood(scale=0.002)
    eps = oracle.calibrate_eps(w.Q, w.X, w.target_matches, metric="ip")
    _check(w.Q, w.X, eps, "ip", "fp32")
    _check(w.Q, w.X, eps, "ip", "bf16")


def test_nonpositive_eps_and_errors():
    Q = np.ones((3, 4), np.float32)
    X = np.ones((5, 4), np.float32)
    assert _gpu(Q, X, 0.0)[0].shape[0] == 0
    assert _gpu(Q, X, -1.0)[0].shape[0] == 0
    with pytest.raises(vj.VJError):
        vj.vj_bruteforce_join(torch.ones((3, 4), device="cuda"), torch.ones((5, 4), device="cuda"),
                              float("inf"))


@pytest.mark.parametrize("d", [96, 128, 250, 384, 500, 768, 960, 1000])
@pytest.mark.parametrize("metric", ["l2", "ip"])
@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_register_row_widths_and_splits(d, metric, precision):
    # 37 query rows (one row block) against 16,411 data rows: 513 tiles of
    # 32 over column splits with a ragged last tile; rows wider than 256
    # are staged in chunks of 128 (960: 192) dimensions
    r = np.random.default_rng(d)
    Q = r.standard_normal((37, d)).astype(np.float32)
    X = r.standard_normal((16_411, d)).astype(np.float32)
    if metric == "ip":
        Q /= np.linalg.norm(Q, axis=1, keepdims=True)
        X /= np.linalg.norm(X, axis=1, keepdims=True)
    D = oracle.dist_matrix(Q, X, metric)
    eps = float(np.quantile(D, 0.002))
    G, O = _check(Q, X, eps, metric, precision)
    assert len(O) > 500


def test_kept_blocks_are_returned_by_trim():
    # the all-pairs result (6M pairs, 72 MB) and the call's candidate arrays
    # are kept for reuse when freed; trimming returns them, a second trim
    # finds nothing
    r = np.random.default_rng(5)
    X = r.standard_normal((4000, 32)).astype(np.float32)
    res = vj.vj_bruteforce_join(torch.from_numpy(X[:1500]).cuda(), torch.from_numpy(X).cuda(), 1e6)
    assert res.count() == 1500 * 4000
    del res
    assert vj.vj_trim_memory() >= 72 << 20
    assert vj.vj_trim_memory() == 0
