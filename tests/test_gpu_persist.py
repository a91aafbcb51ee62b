"""Index and predictor files (vj_index_save / vj_index_load,
vj_predictor_save / vj_predictor_load): a reloaded index gives the same
join results, bit for bit, as the one it was saved from, in every mode; a
damaged file is refused with VJ_ERR_IO."""
import os

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2603_16360_amd import vj  # noqa: E402


def _sorted_result(r):
    qx, d = r.export(sorted=True)
    return qx.cpu().numpy(), d.cpu().numpy(), r.stats().cpu().numpy()


def test_index_round_trip(tmp_path):
    w = workloads.config_tiny(scale=0.3)
    eps = oracle.calibrate_eps(w.Q, w.X, w.target_matches)
    print(f"[gpu-step] persist build nq={w.Q.shape[0]} nx={w.X.shape[0]}", flush=True)
    a = vj.vj_build_merged_index(torch.from_numpy(w.Q).cuda(), torch.from_numpy(w.X).cuda(), R=16)
    path = str(tmp_path / "tiny.vjx")
    a.save(path)
    b = vj.vj_index_load(path)
    assert a.info() == b.info()
    for x, y in zip(a.export_graph(), b.export_graph()):
        assert torch.equal(x, y)
    for kw in ({}, {"work_sharing": "soft"}, {"work_sharing": "hard"},
               {"hybrid": "adapt"}, {"hybrid": "force", "precision": "bf16"}):
        ra, rb = _sorted_result(vj.vj_join(a, eps, **kw)), _sorted_result(vj.vj_join(b, eps, **kw))
        for x, y in zip(ra, rb):
            assert np.array_equal(x, y), kw
    # the join's oracle agrees with the reloaded graph as well
    adj = b.export_graph()[0].cpu().numpy()
    lo = oracle.join(w.Q, w.X, adj, b.info()["entry"], eps, uncertain="out").pairs()
    hi = oracle.join(w.Q, w.X, adj, b.info()["entry"], eps, uncertain="in").pairs()
    got = set(map(tuple, vj.vj_join(b, eps).export()[0].cpu().numpy().tolist()))
    assert lo <= got <= hi


def test_separate_index_with_nnmap_round_trip(tmp_path):
    w = workloads.config_tiny(scale=0.2)
    eps = oracle.calibrate_eps(w.Q, w.X, w.target_matches)
    a = vj.vj_build_separate_index(torch.from_numpy(w.Q).cuda(), torch.from_numpy(w.X).cuda(), R=16)
    a.build_nnmap()
    path = str(tmp_path / "sep.vjx")
    a.save(path)
    b = vj.vj_index_load(path)
    for x, y in zip(a.export_nnmap(), b.export_nnmap()):
        assert torch.equal(x, y)
    for kw in ({"work_sharing": "none"}, {"work_sharing": "soft"}, {"work_sharing": "nnmap"},
               {"work_sharing": "nnmap", "hybrid": "adapt"}):
        ra, rb = _sorted_result(vj.vj_join(a, eps, **kw)), _sorted_result(vj.vj_join(b, eps, **kw))
        for x, y in zip(ra, rb):
            assert np.array_equal(x, y), kw


def test_index_file_damage_is_refused(tmp_path):
    w = workloads.config_tiny(scale=0.05)
    a = vj.vj_build_merged_index(torch.from_numpy(w.Q).cuda(), torch.from_numpy(w.X).cuda(), R=16)
    path = str(tmp_path / "small.vjx")
    a.save(path)
    raw = bytearray(open(path, "rb").read())
    bad = str(tmp_path / "bad.vjx")
    raw[len(raw) // 2] ^= 0x40
    open(bad, "wb").write(bytes(raw))
    with pytest.raises(vj.VJError) as e:
        vj.vj_index_load(bad)
    assert e.value.status == 7 and "checksum" in str(e.value)
    open(bad, "wb").write(bytes(raw[: len(raw) // 3]))
    with pytest.raises(vj.VJError) as e:
        vj.vj_index_load(bad)
    assert e.value.status == 7
    with pytest.raises(vj.VJError) as e:
        vj.vj_index_load(str(tmp_path / "missing.vjx"))
    assert e.value.status == 7


def test_predictor_round_trip(tmp_path):
    rng = np.random.default_rng(4)
    X = torch.from_numpy(rng.standard_normal((512, 40)).astype(np.float32)).cuda()
    Y = torch.from_numpy(rng.random((512, 4)).astype(np.float32)).cuda()
    p = vj.Predictor(40, 32, 16, 4, seed=9)
    p.fit_normalization(X)
    p.train(X, Y, epochs=2, batch=128, lr=1e-3, seed=1)
    path = str(tmp_path / "p.vjm")
    p.save(path)
    q = vj.Predictor.load(path)
    assert q.shapes == p.shapes
    for k, v in p.get_params().items():
        assert torch.equal(v, q.get_params()[k]), k
    mp, vp, tp = p.adam_state()
    mq, vq, tq = q.adam_state()
    assert tp == tq and torch.equal(mp, mq) and torch.equal(vp, vq)
    assert torch.equal(p.forward(X), q.forward(X))
    # training resumes from the same state on both
    p.train(X, Y, epochs=1, batch=128, lr=1e-3, seed=2)
    q.train(X, Y, epochs=1, batch=128, lr=1e-3, seed=2)
    assert torch.equal(p.forward(X), q.forward(X))
