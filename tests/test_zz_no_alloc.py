"""The allocation-free brute-force join (vj_bruteforce_join_noalloc) against
the allocating one (vj_bruteforce_join) and the fp64 oracle, on two calls in
a row, the second with a smaller input (the fixed scratch region keeps the
first call's contents), plus its refusal of inputs that do not fit."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2603_16360_amd import vj  # noqa: E402


def _set(qx):
    return set(map(tuple, qx.cpu().numpy().tolist()))


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_noalloc_matches_allocating_entry_point(precision):
    big = workloads.config_tiny()
    small = workloads.config_tiny(scale=0.2)
    for w in (big, small):
        eps = oracle.calibrate_eps(w.Q, w.X, w.target_matches)
        Q, X = torch.from_numpy(w.Q).cuda(), torch.from_numpy(w.X).cuda()
        print(f"[gpu-step] noalloc {precision} nq={w.Q.shape[0]} nx={w.X.shape[0]}", flush=True)
        ref = vj.vj_bruteforce_join(Q, X, eps, precision=precision)
        rq, rd = ref.export(sorted=True)
        cap = ref.count() + 100
        qx = torch.full((cap, 2), -7, dtype=torch.int32, device="cuda")
        dist = torch.full((cap,), -1.0, dtype=torch.float32, device="cuda")
        n = vj.vj_bruteforce_join_noalloc(Q, X, eps, qx, dist, precision=precision)
        assert n == ref.count()
        got = qx[:n]
        assert _set(got) == _set(rq)
        assert torch.all(qx[n:] == -7) and torch.all(dist[n:] == -1.0)
        # same distance per pair as the allocating entry point
        order = torch.argsort(got[:, 0].long() * w.X.shape[0] + got[:, 1].long())
        assert torch.equal(dist[:n][order], rd)
        # and the oracle's exact set
        oq, ox, _ = oracle.nlj(w.Q, w.X, eps)
        assert _set(got) == set(zip(oq.tolist(), ox.tolist()))


def test_noalloc_capacity_and_limits():
    w = workloads.config_tiny(scale=0.2)
    eps = oracle.calibrate_eps(w.Q, w.X, w.target_matches)
    Q, X = torch.from_numpy(w.Q).cuda(), torch.from_numpy(w.X).cuda()
    full = vj.vj_bruteforce_join(Q, X, eps).count()
    qx = torch.full((10, 2), -7, dtype=torch.int32, device="cuda")
    n = vj.vj_bruteforce_join_noalloc(Q, X, eps, qx)
    assert n == full and n > 10
    allp = _set(vj.vj_bruteforce_join(Q, X, eps).export()[0])
    assert _set(qx) <= allp  # the 10 written are genuine pairs
    # inputs whose temporaries exceed the fixed region are refused
    bigX = torch.zeros((200_000, 128), dtype=torch.float32, device="cuda")
    with pytest.raises(vj.VJError) as e:
        vj.vj_bruteforce_join_noalloc(bigX[:1000], bigX, 1.0, qx)
    assert e.value.status == 6 and "scratch" in str(e.value)
    # still correct after the refusal
    qx2 = torch.empty((full, 2), dtype=torch.int32, device="cuda")
    assert vj.vj_bruteforce_join_noalloc(Q, X, eps, qx2) == full
    assert _set(qx2) == allp
