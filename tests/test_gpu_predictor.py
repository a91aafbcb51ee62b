"""GPU parity of the difficulty predictor and of learned routing.

* post-probe features (vj_join_features) against the oracle's fp64 features;
* MLP forward and the BCE gradients (vj_predictor_loss_grad) against the
  oracle's fp64 MLP: relative max-norm error <= 1e-4 on a fixed minibatch;
* the same at the product shape (768 + 8) -> 256 -> 256 -> 4 on a 1,024-row
  minibatch, which runs the multi-tile paths of the device GEMMs;
* the device Adam step against the oracle's fp64 Adam from the same
  parameters and the same gradients: parameters, moments and step count
  after steps 1, 2 and 10;
* training on the device reduces the loss;
* VJ_HYB_LEARNED: with the same weights on both sides, the oracle's fp64
  features -> fp64 MLP -> budget choice -> oracle budget-mode join (routed
  queries: the oracle's exact join) must match the GPU result on every query
  whose decision is not fragile (predicted recall within 1e-3 of the target,
  or a fragile join).
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

BUDGETS = (0, 16, 64, 256)


class Case:
    def __init__(self, w, eps):
        self.w, self.eps = w, eps
        self.g = oracle.build_merged(w.Q, w.X, w.R)
        self.idx = vj.vj_index_from_graph(torch.from_numpy(w.Q).cuda(), torch.from_numpy(w.X).cuda(),
                                          torch.from_numpy(self.g.adj).cuda(), self.g.entry,
                                          metric=w.metric)


_cases = {}


def case(name):
    if name not in _cases:
        w = workloads.config_tiny() if name == "tiny" else workloads.config_ood(scale=0.004)
        eps = oracle.calibrate_eps(w.Q, w.X, w.target_matches, w.metric)
        print(f"[case] {name} nq={w.Q.shape[0]} nx={w.X.shape[0]} d={w.d} eps={eps:.6g}", flush=True)
        _cases[name] = Case(w, eps)
    return _cases[name]


@pytest.mark.parametrize("name", ["tiny", "ood"])
def test_features_match_oracle(name):
    c = case(name)
    f = vj.vj_join_features(c.idx, c.eps, metric=c.w.metric).cpu().numpy().astype(np.float64)
    ref = oracle.features(c.w.Q, c.w.X, c.g.adj, c.g.entry, c.eps, metric=c.w.metric)
    d = c.w.d
    np.testing.assert_array_equal(f[:, :d], ref[:, :d])
    np.testing.assert_allclose(f[:, d:d + 7], ref[:, d:d + 7], rtol=2e-5, atol=1e-6)
    # the in-range count may differ where a distance lies within fp32 rounding of eps
    diff = np.abs(f[:, d + 7] - ref[:, d + 7])
    assert diff.max() <= 1.0 / c.w.R + 1e-9 and (diff > 0).mean() <= 0.005


def _rand_params(rng, din, h1, h2, k):
    def lay(o, i):
        return (rng.standard_normal((o, i)) * np.sqrt(2.0 / i)).astype(np.float32), \
               (rng.standard_normal(o) * 0.1).astype(np.float32)
    W1, b1 = lay(h1, din)
    W2, b2 = lay(h2, h1)
    W3, b3 = lay(k, h2)
    return [W1, b1, W2, b2, W3, b3]


def _to_dev(params, mu, inv_sigma):
    names = ("W1", "b1", "W2", "b2", "W3", "b3")
    kw = {n: torch.from_numpy(p).cuda() for n, p in zip(names, params)}
    kw["mu"] = torch.from_numpy(mu).cuda()
    kw["inv_sigma"] = torch.from_numpy(inv_sigma).cuda()
    return kw


def test_mlp_forward_and_gradients_match_oracle():
    rng = np.random.default_rng(7)
    n, din, h1, h2, k = 96, 40, 48, 32, 4
    params = _rand_params(rng, din, h1, h2, k)
    X = rng.standard_normal((n, din)).astype(np.float32) * 3 + 1
    mu = rng.standard_normal(din).astype(np.float32)
    inv_sigma = (0.5 + rng.random(din)).astype(np.float32)
    Y = rng.random((n, k)).astype(np.float32)
    mask = (rng.random((n, k)) < 0.8).astype(np.float32)
    p = vj.Predictor(din, h1, h2, k, seed=1)
    p.set_params(**_to_dev(params, mu, inv_sigma))
    Xn = (X.astype(np.float64) - mu) * inv_sigma.astype(np.float64)
    logits = p.forward(torch.from_numpy(X).cuda()).cpu().numpy()
    ref = oracle.mlp_forward(params, Xn)
    assert np.abs(logits - ref).max() <= 1e-4 * max(1.0, np.abs(ref).max())
    loss, g = p.loss_grad(torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda(),
                          torch.from_numpy(mask).cuda())
    rloss, rg = oracle.mlp_bce_backward(params, Xn, Y, mask)
    assert loss == pytest.approx(rloss, rel=1e-5)
    for name, ref_g in zip(("W1", "b1", "W2", "b2", "W3", "b3"), rg):
        got = g[name].cpu().numpy().astype(np.float64)
        err = np.abs(got - ref_g).max() / max(np.abs(ref_g).max(), 1e-12)
        print(f"[mlp] grad {name} rel max-norm error {err:.2e}", flush=True)
        assert err <= 1e-4, name


def test_mlp_gradients_match_oracle_at_product_shape():
    rng = np.random.default_rng(17)
    n, din, h1, h2, k = 1024, 768 + 8, 256, 256, 4
    params = _rand_params(rng, din, h1, h2, k)
    X = rng.standard_normal((n, din)).astype(np.float32)
    mu = (rng.standard_normal(din) * 0.1).astype(np.float32)
    inv_sigma = (0.8 + 0.4 * rng.random(din)).astype(np.float32)
    Y = rng.random((n, k)).astype(np.float32)
    p = vj.Predictor(din, h1, h2, k, seed=1)
    p.set_params(**_to_dev(params, mu, inv_sigma))
    Xn = (X.astype(np.float64) - mu) * inv_sigma.astype(np.float64)
    logits = p.forward(torch.from_numpy(X).cuda()).cpu().numpy()
    ref = oracle.mlp_forward(params, Xn)
    fwd_err = np.abs(logits - ref).max() / max(1.0, np.abs(ref).max())
    print(f"[mlp] product shape forward rel error {fwd_err:.2e}", flush=True)
    assert fwd_err <= 1e-4
    loss, g = p.loss_grad(torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda())
    rloss, rg = oracle.mlp_bce_backward(params, Xn, Y)
    assert loss == pytest.approx(rloss, rel=1e-5)
    for name, ref_g in zip(("W1", "b1", "W2", "b2", "W3", "b3"), rg):
        got = g[name].cpu().numpy().astype(np.float64)
        err = np.abs(got - ref_g).max() / max(np.abs(ref_g).max(), 1e-12)
        print(f"[mlp] product shape grad {name} rel max-norm error {err:.2e}", flush=True)
        assert err <= 1e-4, name


def test_adam_matches_oracle():
    rng = np.random.default_rng(29)
    din, h1, h2, k = 768 + 8, 256, 256, 4
    params = _rand_params(rng, din, h1, h2, k)
    p = vj.Predictor(din, h1, h2, k, seed=3)
    p.set_params(**_to_dev(params, np.zeros(din, np.float32), np.ones(din, np.float32)))
    flat0 = np.concatenate([x.ravel() for x in params]).astype(np.float64)
    n = flat0.size
    assert n == p.n_params
    P, M, V = flat0.copy(), np.zeros(n), np.zeros(n)
    lr = 3e-3
    path = np.zeros(n)  # sum over steps of |step|: successive steps may cancel
    for t in range(1, 11):
        # gradients of mixed scales, with exact zeros and values near eps
        g = rng.standard_normal(n) * np.exp(rng.uniform(-12, 2, n))
        g[rng.random(n) < 0.05] = 0.0
        g[rng.random(n) < 0.01] = 1e-8
        g = g.astype(np.float32)
        p.adam_step(torch.from_numpy(g).cuda(), lr)
        before = P.copy()
        oracle.adam_step(P, g.astype(np.float64), M, V, t, lr)
        path += np.abs(P - before)
        if t in (1, 2, 10):
            got = torch.cat([v.reshape(-1) for k2, v in p.get_params().items()
                             if k2 in vj.Predictor.PARAMS]).cpu().numpy().astype(np.float64)
            m, v, steps = p.adam_state()
            m, v = m.cpu().numpy().astype(np.float64), v.cpu().numpy().astype(np.float64)
            assert steps == t
            # the displacement from the start is what Adam computed: each step
            # within 1e-5 of its size, plus the fp32 rounding of the parameter
            # itself (an ulp per step)
            disp_err = np.abs((got - flat0) - (P - flat0))
            tol = 1e-5 * path + 2 * t * np.abs(P) * 2.0 ** -24 + 1e-12
            worst = float((disp_err / tol).max())
            m_err = np.abs(m - M).max() / np.abs(M).max()
            v_err = np.abs(v - V).max() / np.abs(V).max()
            print(f"[adam] t={t}: displacement err / tol {worst:.3f}, m rel {m_err:.2e}, "
                  f"v rel {v_err:.2e}", flush=True)
            assert worst <= 1.0
            np.testing.assert_allclose(m, M, rtol=1e-5, atol=1e-5 * np.abs(M).max())
            np.testing.assert_allclose(v, V, rtol=1e-5, atol=1e-5 * np.abs(V).max())


def test_training_reduces_loss():
    rng = np.random.default_rng(3)
    n, din = 4096, 16
    X = rng.standard_normal((n, din)).astype(np.float32)
    w = rng.standard_normal((din, 4))
    Y = (1 / (1 + np.exp(-3 * X.astype(np.float64) @ w))).astype(np.float32)  # soft, learnable
    p = vj.Predictor(din, 64, 64, 4, seed=5)
    Xd, Yd = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
    p.fit_normalization(Xd)
    l0, _ = p.loss_grad(Xd, Yd)
    losses = p.train(Xd, Yd, epochs=30, batch=256, lr=2e-3, seed=11)
    l1, _ = p.loss_grad(Xd, Yd)
    print(f"[mlp] loss {l0:.4f} -> {l1:.4f} (epochs: {losses[0]:.4f} .. {losses[-1]:.4f})", flush=True)
    # the entropy floor of soft targets is > 0: compare against it
    ent = float(np.mean(-(Y * np.log(Y + 1e-12) + (1 - Y) * np.log(1 - Y + 1e-12))))
    assert l1 - ent < 0.3 * (l0 - ent)


def _oracle_learned(c, params, mu, inv_sigma, target):
    """The learned join of the oracle: fp64 features -> fp64 MLP -> budgets;
    routed queries joined exactly.  Returns (pairs by query, budgets,
    decision margin per query)."""
    F = oracle.features(c.w.Q, c.w.X, c.g.adj, c.g.entry, c.eps, metric=c.w.metric)
    Xn = (F - mu.astype(np.float64)) * inv_sigma.astype(np.float64)
    rec = 1 / (1 + np.exp(-oracle.mlp_forward(params, Xn)))
    budgets = np.full(len(F), -1, np.int32)
    for i in range(len(F)):
        ok = np.nonzero(rec[i] >= target)[0]
        if ok.size:
            budgets[i] = BUDGETS[ok[0]]
    margin = np.abs(rec - target).min(axis=1)
    r = oracle.join(c.w.Q, c.w.X, c.g.adj, c.g.entry, c.eps, metric=c.w.metric, hybrid="budget",
                    budget=np.maximum(budgets, 0))
    by = {}
    for q, x in zip(r.qi.tolist(), r.xj.tolist()):
        if budgets[q] >= 0:
            by.setdefault(q, set()).add(x)
    oq, ox, _ = oracle.nlj(c.w.Q, c.w.X, c.eps, c.w.metric)
    for q, x in zip(oq.tolist(), ox.tolist()):
        if budgets[q] < 0:
            by.setdefault(q, set()).add(x)
    return by, budgets, margin, r.stats[:, 7].astype(bool)


@pytest.mark.parametrize("name", ["tiny", "ood"])
def test_learned_routing_matches_oracle(name):
    c = case(name)
    din = c.w.d + 8
    rng = np.random.default_rng(21)
    params = _rand_params(rng, din, 64, 64, 4)
    params[5] = np.array([-1.0, 0.0, 0.5, 1.5], np.float32)  # later heads: higher recall
    F = oracle.features(c.w.Q, c.w.X, c.g.adj, c.g.entry, c.eps, metric=c.w.metric)
    mu = F.mean(0).astype(np.float32)
    sd = F.std(0)
    inv_sigma = np.where(sd > 1e-6, 1 / np.maximum(sd, 1e-6), 1.0).astype(np.float32)
    target = 0.6
    p = vj.Predictor(din, 64, 64, 4, seed=0)
    p.set_params(**_to_dev(params, mu, inv_sigma))
    vj.vj_index_attach_predictor(c.idx, p, recall_target=target, budgets=BUDGETS)
    res = vj.vj_join(c.idx, c.eps, metric=c.w.metric, hybrid="learned")
    qx, _ = res.export(sorted=True)
    qx = qx.cpu().numpy()
    got = {}
    for q, x in qx.tolist():
        got.setdefault(q, set()).add(x)
    st = res.stats().cpu().numpy()
    want, budgets, margin, fragile = _oracle_learned(c, params, mu, inv_sigma, target)
    routed = budgets < 0
    vals, cnts = np.unique(budgets, return_counts=True)
    print(f"[learned] {name}: budgets {dict(zip(vals.tolist(), cnts.tolist()))}", flush=True)
    assert 0 < routed.sum() < len(budgets)  # both paths exercised
    ok = (margin > 1e-3) & ~fragile
    print(f"[learned] {name}: compared {ok.sum()} of {len(ok)} queries (others fragile)", flush=True)
    assert ok.sum() >= 0.3 * len(ok) and (ok & routed).sum() > 0
    bad = [q for q in np.nonzero(ok)[0].tolist() if got.get(q, set()) != want.get(q, set())]
    assert not bad, f"{len(bad)} queries differ, e.g. {bad[:5]}"
    assert np.all((st[ok, 7] & 2 > 0) == routed[ok])
    vj.vj_index_attach_predictor(c.idx, None)


def test_learned_pipeline_trains_and_routes():
    # records from the library's own joins: per query, the recall of a
    # budget-mode join at each budget against the exact join, then training,
    # attaching and a learned join; recall must not fall below plain BFS
    c = case("tiny")
    n = c.w.Q.shape[0]
    F = vj.vj_join_features(c.idx, c.eps)
    gt, _ = vj.vj_bruteforce_join(torch.from_numpy(c.w.Q).cuda(), torch.from_numpy(c.w.X).cuda(),
                                  c.eps).export()
    gtc = torch.bincount(gt[:, 0].long(), minlength=n).float()
    Y = []
    for b in BUDGETS:
        r = vj.vj_join(c.idx, c.eps, hybrid="budget",
                       budget=torch.full((n,), b, dtype=torch.int32, device="cuda"))
        cnt = r.stats()[:, 0].float()
        Y.append(torch.where(gtc > 0, cnt / gtc.clamp(min=1), torch.ones_like(cnt)))
    Y = torch.stack(Y, 1).contiguous()
    p = vj.Predictor(c.w.d + 8, 64, 64, 4, seed=2)
    p.fit_normalization(F)
    losses = p.train(F, Y, epochs=40, batch=128, lr=2e-3, seed=4)
    assert losses[-1] < losses[0]
    vj.vj_index_attach_predictor(c.idx, p, recall_target=0.97, budgets=BUDGETS)
    res = vj.vj_join(c.idx, c.eps, hybrid="learned")
    bfs = vj.vj_join(c.idx, c.eps)
    exact = int(gt.shape[0])
    print(f"[learned] pipeline: loss {losses[0]:.4f} -> {losses[-1]:.4f}; recall bfs "
          f"{bfs.count() / exact:.4f} learned {res.count() / exact:.4f}", flush=True)
    assert res.count() >= bfs.count()
    vj.vj_index_attach_predictor(c.idx, None)
