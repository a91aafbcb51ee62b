"""Benchmark of the merged-index epsilon-join on one MI355X.

Workload: X = 1,000,000 and Q = 100,000 integer-valued vectors (stored as
fp32), d = 128, 256-cluster mixture with heavy-tailed per-dimension scales,
L2, eps for a mean of 50 matches per query (calibrated by the CPU oracle on
2,000 sampled queries and stored in tests/golden/eps.json), merged graph
out-degree 32.  A step is one vj_join of all 100,000 queries (self seeding,
BFS expansion) against the GPU-built merged index with inputs resident in
HBM.  Recall is measured against the exact MFMA brute-force join.

Prints one JSON line on stdout; progress goes to stderr.
  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TIER_KERNELS = ("k_join_lds (one wave per query)",
                "k_join_coop (one workgroup per query; LDS, then global tables)",
                "k_join_coop_global (re-run launch on global tables)")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_join_mid_traffic.txt")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2603_16360_amd", "csrc", f)
                  for f in ("join_impl.h", "join_inst.hip")]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_model():
    """The host CPU's model name (as lscpu reports it)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def kernel_source_sha():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(tier):
    """HBM bytes per launch of the tier's kernel from the committed rocprofv3
    counter summary, or None when the kernel source changed since then."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = dict(line.split(":", 1) for line in open(TRAFFIC_FILE) if ":" in line)
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("source_sha") != kernel_source_sha():
        return None
    key = f"tier{tier}_hbm_bytes_per_launch"
    return float(kv[key]) if key in kv else None


def algorithmic_bytes(stats, dp, elem_bytes, R, mask):
    """Bytes the join must move per launch: per query its own row, one
    adjacency row for the probe plus one per expanded node, every evaluated
    row, and 12 bytes per emitted pair (query, data, distance)."""
    st = stats[mask].astype(np.int64)
    pairs, ndist, nexp = st[:, 0], st[:, 1], st[:, 2]
    per_q = dp * 4 + (1 + nexp) * R * 4 + ndist * dp * elem_bytes + pairs * 12
    return int(per_q.sum())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--variants", default="fp32,u8")
    ap.add_argument("--gather-calib", action="store_true",
                    help="run the counter-calibration gather first (2,000,000 random 512-byte rows)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="run a plain 1 GiB device copy first (HBM counter calibration)")
    ap.add_argument("--ood", action="store_true",
                    help="instead of the headline: the OOD inner-product workload (2M x 768, 200k "
                         "queries); plain fp32 modes against learned routing at equal recall")
    ap.add_argument("--ood-scale", type=float, default=1.0,
                    help="1.0 (the stated size) or 0.1 (X = 200k, 20k queries)")
    ap.add_argument("--modes", action="store_true",
                    help="instead of the headline: MI, MI+SWS, MI+HWS on the merged index against "
                         "INLJ, SWS, HWS on separate indexes, on the headline workload")
    ap.add_argument("--highdim", action="store_true",
                    help="instead of the headline: the 1M x 960 workload, fp32 rows against bf16 "
                         "rows with fp32 re-check, error against fp64")
    ap.add_argument("--stream", action="store_true",
                    help="instead of the headline: the batched stream workload (200 batches, "
                         "p50/p99 batch latency)")
    ap.add_argument("--stream-scale", type=float, default=0.1,
                    help="0.1 (X = 1M, 487k queries) or 1.0 (the stated size: X = 10M, 4.87M "
                         "queries)")
    ap.add_argument("--stream-modes", action="store_true",
                    help="with --stream (offline index): also join every batch in MI+Adapt "
                         "(hybrid ADAPT) and hybrid-for-all (FORCE) mode; queries/s and recall")
    ap.add_argument("--stream-insert", action="store_true",
                    help="with --stream: the index starts over X alone and each batch is "
                         "inserted (vj_index_insert_queries) right before its join; batch "
                         "latency = insertion + join")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the join shards by query id; see the design notes)", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads
    from paper_2603_16360_amd import vj

    if args.stream:
        return stream_main(args, torch, workloads, vj)
    if args.modes:
        return modes_main(args, torch, workloads, vj)
    if args.ood:
        return ood_main(args, torch, workloads, vj)
    if args.highdim:
        return highdim_main(args, torch, workloads, vj)

    t0 = time.time()
    w = workloads.config_mid()
    golden = json.load(open(os.path.join(ROOT, "tests", "golden", "eps.json")))["mid"]
    for key, arr in (("Q_sha", w.Q), ("X_sha", w.X)):
        sha = hashlib.sha256(np.ascontiguousarray(arr).tobytes()).hexdigest()[:16]
        if sha != golden[key]:
            raise SystemExit(f"generated data differs from the calibrated data ({key})")
    eps = float(golden["eps"])
    nq, nx, d, R = w.Q.shape[0], w.X.shape[0], w.d, w.R
    log(f"data {nq} x {nx} x {d} generated in {time.time() - t0:.1f}s, eps={eps}")

    dev = torch.device("cuda:0")
    if args.copy_calib:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)  # reads and writes exactly 1 GiB
        torch.cuda.synchronize()
        del a, b
        log("copy calibration: 1 GiB device-to-device copy done")
    if args.gather_calib:
        # 2,000,000 distinct random rows of 4,000,000 x 128 fp32 (2 GB, far
        # beyond the caches), read with the join's row-read layout: the rows
        # move exactly 1,024,000,000 bytes; ids and output 16,000,000 more
        g = torch.Generator(device=dev)
        g.manual_seed(5)
        rows = torch.rand((4_000_000, 128), device=dev, generator=g)
        ids = torch.randperm(4_000_000, device=dev, generator=g)[:2_000_000].to(torch.int32)
        torch.cuda.synchronize()
        vj.vj_calib_gather(rows, ids)
        torch.cuda.synchronize()
        del rows, ids
        log("gather calibration: 2,000,000 rows of 512 bytes read")
    Q = torch.from_numpy(w.Q).to(dev)
    X = torch.from_numpy(w.X).to(dev)
    torch.cuda.synchronize()

    t = time.time()
    idx = vj.vj_build_merged_index(Q, X, metric="l2", R=R)
    torch.cuda.synchronize()
    build_s = time.time() - t
    info = idx.info()
    log(f"merged index built in {build_s:.2f}s (entry {info['entry']})")

    t = time.time()
    gt = vj.vj_bruteforce_join(Q, X, eps, precision="bf16")
    torch.cuda.synchronize()
    gt_s = time.time() - t
    gt_qx, _ = gt.export(sorted=True)
    gt_keys = gt_qx[:, 0].to(torch.int64) * nx + gt_qx[:, 1].to(torch.int64)
    n_gt = int(gt_keys.numel())
    log(f"ground truth: {n_gt} pairs in {gt_s:.2f}s (exact MFMA tiles + fp64 re-check)")

    results = {}
    for variant in args.variants.split(","):
        for _ in range(args.warmup):
            vj.vj_join(idx, eps, precision=variant)
        torch.cuda.synchronize()
        walls, tier_ms, tier_ln = [], np.zeros(4), np.zeros(4)
        res = None
        for _ in range(args.steps):
            res = None  # the previous result is released outside the timed region
            torch.cuda.synchronize()
            ts = time.perf_counter()
            res = vj.vj_join(idx, eps, precision=variant)
            torch.cuda.synchronize()
            walls.append(time.perf_counter() - ts)
            tiers = res.tiers()
            tier_ms += [t["ms"] for t in tiers]
            tier_ln += [t["launches"] for t in tiers]
        tier_ms /= args.steps
        tier_ln /= args.steps
        tiers = res.tiers()
        qx, _ = res.export(sorted=True)
        keys = qx[:, 0].to(torch.int64) * nx + qx[:, 1].to(torch.int64)
        precise = bool(torch.isin(keys, gt_keys).all().item())
        recall = keys.numel() / max(1, n_gt)
        st = res.stats().cpu().numpy()
        fl = st[:, 7]
        # the launch that completed each query: one-wave tier, workgroup tier
        # (LDS or, promoted within the launch, global tables), re-run launch
        done_on = [(fl & 1) == 0, ((fl & 1) == 1) & ((fl & 16) == 0), (fl & 16) > 0]
        eb = 1 if variant == "u8" else 4
        per_tier = []
        for t in range(3):
            ms = float(tier_ms[t] + (tier_ms[3] if t == 2 else 0.0))
            ln = float(tier_ln[t] + (tier_ln[3] if t == 2 else 0.0))
            nbytes = algorithmic_bytes(st, 128, eb, R, done_on[t])
            per_tier.append({"kernel": TIER_KERNELS[t], "ms": ms, "launches": ln,
                             "queries_launched": int(tiers[t]["queries"] + (tiers[3]["queries"] if t == 2 else 0)),
                             "queries_completed": int(done_on[t].sum()),
                             "algorithmic_bytes": nbytes,
                             "achieved_gbs": nbytes / (ms * 1e-3) / 1e9 if ms > 0 else 0.0})
        dom = int(np.argmax([pt["ms"] for pt in per_tier]))
        all_bytes = algorithmic_bytes(st, 128, eb, R, np.ones(len(st), bool))
        dev_ms = float(tier_ms.sum())
        results[variant] = {
            "qps": nq / float(np.mean(walls)),
            "ms_per_step": 1000.0 * float(np.mean(walls)),
            "device_ms": dev_ms, "recall": recall, "precision_is_one": precise,
            "pairs": int(keys.numel()), "tiers": per_tier, "dominant_tier": dom,
            "algorithmic_bytes_all": all_bytes,
            "traversal_gbs": all_bytes / (dev_ms * 1e-3) / 1e9,
            "mean_dist_evals": float(st[:, 1].mean()), "mean_expanded": float(st[:, 2].mean()),
        }
        log(f"{variant}: {results[variant]}")

    head = results.get("fp32") or next(iter(results.values()))
    cpu = None
    if not args.no_cpu:
        import oracle
        adj, _, _ = idx.export_graph()
        adj = adj.cpu().numpy()
        cores = len(os.sched_getaffinity(0))
        reps, cpu_s, npairs = 0, 0.0, 0
        while cpu_s < 10.0 and reps < 30:  # the whole query set, repeated to >= 10 s
            t = time.time()
            counts = oracle.join_self_counts(w.Q, w.X, adj, info["entry"], eps)
            cpu_s += time.time() - t
            npairs = int(counts.sum())
            reps += 1
        # the ground truth on the CPU: the fp64 nested-loop join on a fixed
        # 2,000-query sample, extrapolated linearly to all queries
        gt_sample = np.sort(np.random.default_rng(203).choice(nq, size=2000, replace=False))
        t = time.time()
        gt_counts = oracle.nlj_counts(w.Q[gt_sample], w.X, eps)
        nlj_s = time.time() - t
        cpu = {"value": reps * nq / cpu_s, "unit": "queries/s", "cores": cores,
               "kind": "oracle", "cpu_model": cpu_model(),
               "sample": f"all {nq} queries x {reps} repetitions ({cpu_s:.1f}s): self-seeded BFS "
                         f"merged-index join in fp64 with OpenMP over queries, same graph and eps; "
                         f"{npairs} pairs per repetition",
               "nlj_ground_truth": {
                   "sample_queries": int(gt_sample.size), "sample_s": nlj_s,
                   "sample_pairs": int(gt_counts.sum()),
                   "extrapolated_s_all_queries": nlj_s * nq / gt_sample.size,
                   "note": "fp64 nested-loop join (OpenMP) on a fixed 2,000-query sample (seed "
                           "203), extrapolated linearly to all queries"}}
        log(f"cpu baseline: {cpu}")

    dom = head["tiers"][head["dominant_tier"]]
    traffic = measured_traffic(head["dominant_tier"])
    line = {
        "metric": "join queries/sec at recall>=0.95 (1Mx128 fp32); achieved HBM GB/s vs peak",
        "value": head["qps"],
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "X=1,000,000 Q=100,000 d=128 integer-valued 256-cluster mixture, "
                               "L2, eps for mean 50 matches, merged graph R=32, self-seeded BFS",
                   "eps": eps, "global_batch": nq},
        "recall": head["recall"],
        "roofline": {"bound": "hbm", "kernel": dom["kernel"], "achieved": dom["achieved_gbs"],
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": dom["achieved_gbs"] / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": dom["algorithmic_bytes"] / max(1.0, dom["launches"]),
                     "avg_launch_ms": dom["ms"] / max(1.0, dom["launches"])},
        "cpu_baseline": cpu,
        "variants": results,
        "build_s": build_s,
        "ground_truth_s": gt_s,
        "ground_truth_pairs": n_gt,
    }
    print(json.dumps(line), flush=True)


def modes_main(args, torch, workloads, vj):
    """The paper's execution modes on the headline workload (Sections 2.2 and
    4.1-4.3): INLJ, HWS and SWS on separate indexes (G_X over X, G_Q over Q;
    best-first greedy from the entry of G_X) against MI, MI+SWS and MI+HWS on
    the merged index, at the same eps.  Soft / hard modes run one launch per
    MST depth level (parents before children), so their launch count is the
    MST depth."""
    w = workloads.config_mid()
    eps = float(json.load(open(os.path.join(ROOT, "tests", "golden", "eps.json")))["mid"]["eps"])
    nq, nx = w.Q.shape[0], w.X.shape[0]
    dev = torch.device("cuda:0")
    Q = torch.from_numpy(w.Q).to(dev)
    X = torch.from_numpy(w.X).to(dev)
    t = time.time()
    merged = vj.vj_build_merged_index(Q, X, R=w.R)
    torch.cuda.synchronize()
    bm = time.time() - t
    t = time.time()
    sep = vj.vj_build_separate_index(Q, X, R=w.R)
    torch.cuda.synchronize()
    bs = time.time() - t
    t = time.time()
    sep.build_nnmap()
    torch.cuda.synchronize()
    bn = time.time() - t
    # HNSW-style upper layers over the data graph: each separate-index query
    # may start its greedy phase where a descent through them ends
    t = time.time()
    vj.vj_index_build_layers(sep, R=w.R, seed=1)
    torch.cuda.synchronize()
    bl = time.time() - t
    layers = [int(ids.numel()) for ids, _, _ in vj.vj_index_layers(sep)]
    log(f"merged index {bm:.2f}s, separate indexes {bs:.2f}s, NN-Map {bn:.2f}s, "
        f"upper layers {layers} {bl:.2f}s")
    gt_qx, _ = vj.vj_bruteforce_join(Q, X, eps, precision="bf16").export(sorted=True)
    gt_keys = gt_qx[:, 0].to(torch.int64) * nx + gt_qx[:, 1].to(torch.int64)
    n_gt = int(gt_keys.numel())
    modes = {
        "MI": (merged, {}), "MI+SWS": (merged, {"work_sharing": "soft"}),
        "MI+HWS": (merged, {"work_sharing": "hard"}),
        "INLJ": (sep, {"work_sharing": "none"}), "SWS": (sep, {"work_sharing": "soft"}),
        "HWS": (sep, {"work_sharing": "hard"}),
        "NN-Map": (sep, {"work_sharing": "nnmap"}),
        "INLJ, layer seeds": (sep, {"work_sharing": "none", "layer_seeds": 1}),
        "SWS, layer seeds": (sep, {"work_sharing": "soft", "layer_seeds": 1}),
        "HWS, layer seeds": (sep, {"work_sharing": "hard", "layer_seeds": 1}),
    }
    out = {}
    for name, (idx, kw) in modes.items():
        for _ in range(args.warmup):
            vj.vj_join(idx, eps, **kw)
        torch.cuda.synchronize()
        walls = []
        res = None
        for _ in range(args.steps):
            res = None
            torch.cuda.synchronize()
            ts = time.perf_counter()
            res = vj.vj_join(idx, eps, **kw)
            torch.cuda.synchronize()
            walls.append(time.perf_counter() - ts)
        qx, _ = res.export(sorted=True)
        keys = qx[:, 0].to(torch.int64) * nx + qx[:, 1].to(torch.int64)
        st = res.stats().cpu().numpy()
        tiers = res.tiers()
        out[name] = {"qps": nq / float(np.mean(walls)), "ms": 1000 * float(np.mean(walls)),
                     "recall": keys.numel() / max(1, n_gt),
                     "precision_is_one": bool(torch.isin(keys, gt_keys).all().item()),
                     "launches": int(sum(tt["launches"] for tt in tiers)),
                     "mean_dist_evals": float(st[:, 1].mean()),
                     "mean_greedy_pops": float(st[:, 4].mean()) if idx is sep else 0.0}
        log(f"{name}: {out[name]}")
    line = {"metric": "join queries/sec by execution mode (1Mx128, 100k queries, same eps)",
            "unit": "queries/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "data": "synthetic",
            "config": {"workload": "X=1,000,000 Q=100,000 d=128 integer-valued 256-cluster "
                                   "mixture, L2, eps for mean 50 matches, R=32", "eps": eps},
            "build_s": {"merged": bm, "separate": bs, "nnmap": bn, "upper_layers": bl},
            "upper_layer_sizes": layers, "ground_truth_pairs": n_gt,
            "modes": out}
    print(json.dumps(line), flush=True)


def ood_main(args, torch, workloads, vj):
    """OOD queries (30 % from shifted means), inner product, at the stated
    size by default (--ood-scale 0.1 for the 1/10 workload).  The plain fp32
    join's family is the paper's MI (BFS), MI+Adapt (d1/d2 rule) and the
    hybrid search for every query at three queue bounds; the learned family
    is the router trained on separate training queries indexed in their own
    merged graph (records: per-query recall of budget-mode joins against the
    exact join) at three recall targets, in fp32 and with low-precision rows.
    For each learned point the fastest plain point with at least its recall
    gives the speed ratio at equal recall.  OOD queries' recall is reported
    on its own."""
    key = "ood_full" if args.ood_scale >= 1.0 else "ood"
    golden = json.load(open(os.path.join(ROOT, "tests", "golden", "eps.json")))[key]
    scale = golden["scale"]
    t0 = time.time()
    w = workloads.config_ood(scale=scale)
    wt = workloads.config_ood(scale=scale, train=True)
    for k, arr in (("Q_sha", w.Q), ("X_sha", w.X)):
        sha = hashlib.sha256(np.ascontiguousarray(arr).tobytes()).hexdigest()[:16]
        if sha != golden[k]:
            raise SystemExit(f"generated data differs from the calibrated data ({k})")
    eps = golden["eps"]
    nq, nt, d = w.Q.shape[0], wt.Q.shape[0], w.d
    log(f"ood: X {w.X.shape}, {nq} test and {nt} training queries, eps={eps} ({time.time() - t0:.1f}s)")
    dev = torch.device("cuda:0")
    X = torch.from_numpy(w.X).to(dev)
    Qt = torch.from_numpy(w.Q).to(dev)
    Qr = torch.from_numpy(wt.Q).to(dev)
    del w.X
    t = time.time()
    idx = vj.vj_build_merged_index(Qt, X, metric="ip", R=w.R)
    torch.cuda.synchronize()
    build_s = time.time() - t
    log(f"test index built in {build_s:.1f}s")
    t = time.time()
    idx_tr = vj.vj_build_merged_index(Qr, X, metric="ip", R=wt.R)
    torch.cuda.synchronize()
    log(f"training index built in {time.time() - t:.1f}s")
    budgets = (0, 16, 64, 256)
    # training records
    t = time.time()
    F = vj.vj_join_features(idx_tr, eps, metric="ip")
    gt_tr, _ = vj.vj_bruteforce_join(Qr, X, eps, metric="ip", precision="bf16").export()
    gtc = torch.bincount(gt_tr[:, 0].long(), minlength=nt).float()
    del gt_tr
    Y = []
    for b in budgets:
        r = vj.vj_join(idx_tr, eps, metric="ip", hybrid="budget",
                       budget=torch.full((nt,), b, dtype=torch.int32, device=dev))
        cnt = r.stats()[:, 0].float()
        Y.append(torch.where(gtc > 0, cnt / gtc.clamp(min=1), torch.ones_like(cnt)))
        del r
    Y = torch.stack(Y, 1).contiguous()
    del idx_tr
    records_s = time.time() - t
    pred = vj.Predictor(d + 8, 256, 256, len(budgets), seed=1)
    pred.fit_normalization(F)
    torch.cuda.synchronize()
    ts = time.time()
    epochs = 40
    losses = pred.train(F, Y, epochs=epochs, batch=512, lr=1e-3, seed=2)
    torch.cuda.synchronize()
    train_s = time.time() - ts
    log(f"records {records_s:.1f}s ({nt} queries x {len(budgets)} budgets), training {train_s:.1f}s "
        f"({epochs} epochs, loss {losses[0]:.4f} -> {losses[-1]:.4f})")
    gt, _ = vj.vj_bruteforce_join(Qt, X, eps, metric="ip", precision="bf16").export()
    n_gt = int(gt.shape[0])
    is_ood = torch.from_numpy(w.meta["is_ood"]).to(dev)
    gt_ood = int(is_ood[gt[:, 0].long()].sum().item())
    del gt

    def measure(name, kw, target=None):
        if target is not None:
            vj.vj_index_attach_predictor(idx, pred, recall_target=target, budgets=budgets)
        for _ in range(max(1, args.warmup)):
            vj.vj_join(idx, eps, metric="ip", **kw)
        torch.cuda.synchronize()
        walls = []
        res = None
        for _ in range(args.steps):
            res = None
            torch.cuda.synchronize()
            ts = time.perf_counter()
            res = vj.vj_join(idx, eps, metric="ip", **kw)
            torch.cuda.synchronize()
            walls.append(time.perf_counter() - ts)
        qx, _ = res.export()
        st = res.stats().cpu().numpy()
        found_ood = int(is_ood[qx[:, 0].long()].sum().item())
        r = {"qps": nq / float(np.mean(walls)), "ms": 1000 * float(np.mean(walls)),
             "recall": int(qx.shape[0]) / max(1, n_gt),
             "recall_ood_queries": found_ood / gt_ood if gt_ood else None,
             "recall_in_distribution_queries": (int(qx.shape[0]) - found_ood) / max(1, n_gt - gt_ood),
             "hybrid_queries": int(st[:, 5].sum()), "routed_exact": int(((st[:, 7] & 2) > 0).sum()),
             "precision": kw.get("precision", "fp32")}
        if target is not None:
            r["recall_target"] = target
        log(f"{name}: {r}")
        return r

    plain = {"MI (BFS)": measure("MI (BFS)", {}),
             "MI+Adapt": measure("MI+Adapt", {"hybrid": "adapt"})}
    for beam in (16, 64, 256):
        name = f"hybrid for all, B={beam}"
        plain[name] = measure(name, {"hybrid": "force", "hybrid_beam": beam})
    # the exact join reaches any recall: the plain point beyond the graph modes
    for prec in ("fp32", "bf16"):
        name = f"exact join ({prec} tiles)"
        torch.cuda.synchronize()
        ts = time.perf_counter()
        n_ex = vj.vj_bruteforce_join(Qt, X, eps, metric="ip", precision=prec).count()
        torch.cuda.synchronize()
        el = time.perf_counter() - ts
        plain[name] = {"qps": nq / el, "ms": 1000 * el, "recall": n_ex / max(1, n_gt),
                       "recall_ood_queries": 1.0, "recall_in_distribution_queries": 1.0,
                       "precision": "fp32"}
        log(f"{name}: {plain[name]}")
    learned = {}
    for target in (0.9, 0.95, 0.98):
        name = f"learned, target {target}"
        learned[name] = measure(name, {"hybrid": "learned"}, target)
    # the learned router with low-precision rows (bf16 and fp8 with their
    # proven margins and fp32 re-checks) at the middle target
    for prec in ("bf16", "fp8"):
        name = f"learned, target 0.95, {prec} rows"
        learned[name] = measure(name, {"hybrid": "learned", "precision": prec}, 0.95)
    # equal recall: the fastest plain point whose recall reaches the learned one's
    compare = {}
    for name, r in learned.items():
        ok = [(p["qps"], pn) for pn, p in plain.items() if p["recall"] >= r["recall"]]
        if ok:
            q, pn = max(ok)
            compare[name] = {"plain": pn, "plain_qps": q, "speedup": r["qps"] / q}
        else:
            compare[name] = {"plain": None, "plain_qps": None, "speedup": None,
                             "note": "no plain fp32 point reaches this recall"}
    best = max(learned.items(), key=lambda kv: (compare[kv[0]]["speedup"] or 0.0))
    line = {"metric": "OOD join queries/sec at equal recall: learned mixed-precision form vs plain fp32 join",
            "value": best[1]["qps"], "unit": "queries/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": best[1]["precision"], "data": "synthetic",
            "config": {"workload": f"OOD{'' if scale >= 1.0 else ' at 1/10 scale'}: X={X.shape[0]:,} "
                                   f"unit vectors d=768 (512-mean vMF mixture); {nq:,} test queries, "
                                   "30 % from means rotated 40 deg (concentrated at mean cosine 0.92); "
                                   f"inner product, eps for 20 mean matches; predictor trained on "
                                   f"{nt:,} separate queries", "eps": eps},
            "best_learned": best[0], "equal_recall": compare, "plain": plain, "learned": learned,
            "build_s": build_s, "records_s": records_s, "train_s": train_s, "train_epochs": epochs,
            "ground_truth_pairs": n_gt, "ground_truth_pairs_of_ood_queries": gt_ood}
    print(json.dumps(line), flush=True)


def highdim_main(args, torch, workloads, vj):
    """High-dimensional data with the precision form: X = 1,000,000 and
    Q = 10,000 vectors of d = 960 in [0, 1] (100-cluster Beta mixture), L2,
    eps for a mean of 10 matches.  The join with fp32 rows against the join
    with bf16 rows (a proven per-row margin, fp32 re-check of every candidate
    inside it), both BFS on the same merged index; recall against the exact
    MFMA brute-force join; the error of every reported distance against
    fp64, max |d - d64| / eps."""
    golden = json.load(open(os.path.join(ROOT, "tests", "golden", "eps.json")))["highdim"]
    t0 = time.time()
    w = workloads.config_highdim()
    for k, arr in (("Q_sha", w.Q), ("X_sha", w.X)):
        sha = hashlib.sha256(np.ascontiguousarray(arr).tobytes()).hexdigest()[:16]
        if sha != golden[k]:
            raise SystemExit(f"generated data differs from the calibrated data ({k})")
    eps = golden["eps"]
    nq = w.Q.shape[0]
    log(f"highdim: X {w.X.shape}, {nq} queries, eps={eps} ({time.time() - t0:.1f}s)")
    dev = torch.device("cuda:0")
    Q = torch.from_numpy(w.Q).to(dev)
    X = torch.from_numpy(w.X).to(dev)
    del w.X
    t = time.time()
    idx = vj.vj_build_merged_index(Q, X, metric="l2", R=w.R, copies=1)
    torch.cuda.synchronize()
    build_s = time.time() - t
    log(f"merged index built in {build_s:.1f}s")
    t = time.time()
    gtr = vj.vj_bruteforce_join(Q, X, eps, precision="bf16")
    torch.cuda.synchronize()
    gt_s = time.time() - t
    gt_qx, gt_d = gtr.export(sorted=True)
    gt_keys = gt_qx[:, 0].to(torch.int64) * X.shape[0] + gt_qx[:, 1].to(torch.int64)
    n_gt = int(gt_keys.numel())

    def err(qx, d):
        """max |d - d64| / eps over the pairs, d64 from the fp32 inputs in fp64"""
        m = 0.0
        for a in range(0, qx.shape[0], 1 << 16):
            q = Q[qx[a:a + (1 << 16), 0].long()].double()
            x = X[qx[a:a + (1 << 16), 1].long()].double()
            d64 = (q - x).pow(2).sum(1).sqrt()
            m = max(m, float((d[a:a + (1 << 16)].double() - d64).abs().max().item()) if d64.numel() else 0.0)
        return m / eps

    out = {}
    sets = {}
    for prec in ("fp32", "bf16"):
        for _ in range(max(1, args.warmup)):
            vj.vj_join(idx, eps, precision=prec)
        torch.cuda.synchronize()
        walls = []
        res = None
        for _ in range(args.steps):
            res = None
            torch.cuda.synchronize()
            ts = time.perf_counter()
            res = vj.vj_join(idx, eps, precision=prec)
            torch.cuda.synchronize()
            walls.append(time.perf_counter() - ts)
        qx, d = res.export(sorted=True)
        keys = qx[:, 0].to(torch.int64) * X.shape[0] + qx[:, 1].to(torch.int64)
        sets[prec] = keys
        out[prec] = {"qps": nq / float(np.mean(walls)), "ms": 1000 * float(np.mean(walls)),
                     "recall": keys.numel() / max(1, n_gt),
                     "precision_is_one": bool(torch.isin(keys, gt_keys).all().item()),
                     "pairs": int(keys.numel()), "rechecked": res.rechecked(),
                     "max_abs_err_over_eps": err(qx, d)}
        log(f"{prec}: {out[prec]}")
    same = bool(sets["fp32"].numel() == sets["bf16"].numel() and torch.equal(sets["fp32"], sets["bf16"]))
    line = {"metric": "high-dim join queries/sec (1Mx960, bf16 rows with fp32 re-check vs fp32 rows)",
            "value": out["bf16"]["qps"], "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "bf16", "data": "synthetic",
            "config": {"workload": "X=1,000,000 Q=10,000 d=960 in [0,1], 100-cluster Beta mixture, L2, "
                                   "eps for mean 10 matches, merged graph R=32, self-seeded BFS",
                       "eps": eps},
            "variants": out, "bf16_pairs_equal_fp32_pairs": same, "build_s": build_s,
            "ground_truth_s": gt_s, "ground_truth_pairs": n_gt,
            "ground_truth_max_abs_err_over_eps": err(gt_qx, gt_d)}
    print(json.dumps(line), flush=True)


def stream_main(args, torch, workloads, vj):
    """The batched stream: 200 join batches, each at its own eps
    (oracle-calibrated, tests/golden/eps.json).

    Offline (default): one merged index over X and every batch's queries,
    then the batches joined one after the other (vj_join_batches) by the
    host runner, the device runner and HIP graph replay.
    --stream-insert: the index starts over X alone; each batch's queries are
    inserted into it (vj_index_insert_queries) and then joined, so a batch's
    latency is its insertion plus its join (every step starts from a fresh
    X-only index, built outside the timed region)."""
    if args.stream_scale not in (0.1, 1.0):
        raise SystemExit("--stream-scale is 0.1 or 1.0")
    key = "stream" if args.stream_scale == 0.1 else "stream_full"
    golden = json.load(open(os.path.join(ROOT, "tests", "golden", "eps.json")))[key]
    t0 = time.time()
    w = workloads.config_stream(scale=golden["scale"], n_batches=golden["n_batches"])
    for k, arr in (("Q_sha", w.Q), ("X_sha", w.X)):
        sha = hashlib.sha256(np.ascontiguousarray(arr).tobytes()).hexdigest()[:16]
        if sha != golden[k]:
            raise SystemExit(f"generated data differs from the calibrated data ({k})")
    batches = workloads.stream_batches(w)
    starts = [b[0] for b in batches]
    counts = [b[1] for b in batches]
    eps = golden["eps"]
    nq = int(sum(counts))
    nx = w.X.shape[0]
    size = f"X={nx:,} x {w.d}"
    log(f"stream: X {w.X.shape}, {len(batches)} batches, {w.Q.shape[0]} queries ({time.time() - t0:.1f}s)")
    dev = torch.device("cuda:0")
    Q = torch.from_numpy(w.Q).to(dev)
    X = torch.from_numpy(w.X).to(dev)
    del w.Q, w.X
    lo, hi = min(counts), max(counts)
    workload = (f"stream at {'the stated size' if key == 'stream_full' else '1/10 scale'}: {size} "
                f"1,024-cluster Gaussian mixture; 200 batches of {lo:,}..{hi:,} queries "
                f"(log-uniform), eps per batch for 5..200 mean matches")

    def recall(res):
        """Pairs found / exact pairs on every 20th batch (MFMA brute force)."""
        found = exact = 0
        for b in range(0, len(batches), 20):
            qb = Q[starts[b]:starts[b] + counts[b]]
            gt = vj.vj_bruteforce_join(qb, X, eps[b])
            exact += gt.count()
            found += res[b].count()
            del gt
        return found / max(1, exact)

    if args.stream_insert:
        return stream_insert(args, torch, vj, Q, X, starts, counts, eps, nq, workload, recall)

    t = time.time()
    idx = vj.vj_build_merged_index(Q, X, metric="l2", R=w.R)
    torch.cuda.synchronize()
    build_s = time.time() - t
    log(f"merged index over {nq + nx} nodes built in {build_s:.1f}s")
    params, tuned_ms = vj.vj_autotune_join(idx, eps[0], query_ids=torch.arange(
        starts[0], starts[0] + counts[0], dtype=torch.int32, device=dev))
    log(f"autotuned on batch 0: start_tier={params.start_tier} precision={params.precision} "
        f"({tuned_ms:.3f} ms)")

    def run(runner):
        """Timed runs of one batch runner: (results, wall seconds per run,
        per-batch ms of every run).  Earlier results are released before the
        timer starts."""
        for _ in range(max(1, args.warmup)):
            vj.vj_join_batches(idx, starts, counts, eps, params=params, runner=runner)
        torch.cuda.synchronize()
        walls, lat = [], []
        res = None
        for _ in range(args.steps):
            res = None
            torch.cuda.synchronize()
            ts = time.perf_counter()
            res, ms = vj.vj_join_batches(idx, starts, counts, eps, params=params, runner=runner)
            torch.cuda.synchronize()
            walls.append(time.perf_counter() - ts)
            lat.extend(ms)
        return res, walls, np.array(lat)

    res, walls, lat = run("host")
    pairs = sum(r.count() for r in res)
    rec = recall(res)
    # the same batches driven from the device (no host synchronisation
    # between batches): direct launches and HIP graph replay
    dev_runs = {}
    for runner in ("device", "graph"):
        dres, dwalls, dlat = run(runner)
        same = all(a.count() == b.count() for a, b in zip(res, dres))
        dev_runs[runner] = {
            "value": nq / float(np.mean(dwalls)), "unit": "queries/s",
            "ms_per_step": 1000.0 * float(np.mean(dwalls)),
            "batch_device_ms_p50": float(np.percentile(dlat, 50)),
            "batch_device_ms_p99": float(np.percentile(dlat, 99)),
            "pair_counts_equal_host_runner": bool(same)}
        log(f"{runner} runner: {dev_runs[runner]['value']:.0f} queries/s, pair counts equal: {same}")
        del dres
    # the paper's hybrid forms on the same batches (host runner, one timed run
    # each): MI+Adapt routes the queries its d1/d2 rule flags, FORCE all
    hybrid_runs = {}
    if args.stream_modes:
        for mode in ("adapt", "force"):
            p2 = vj.join_params(hybrid=mode, start_tier=params.start_tier)
            p2.precision = params.precision
            vj.vj_join_batches(idx, starts, counts, eps, params=p2)
            torch.cuda.synchronize()
            ts = time.perf_counter()
            hres, hms = vj.vj_join_batches(idx, starts, counts, eps, params=p2)
            torch.cuda.synchronize()
            wall = time.perf_counter() - ts
            hybrid_runs[mode] = {
                "value": nq / wall, "unit": "queries/s", "ms_per_step": 1000.0 * wall,
                "batch_ms_p50": float(np.percentile(hms, 50)),
                "batch_ms_p99": float(np.percentile(hms, 99)),
                "pairs": int(sum(r.count() for r in hres)),
                "recall_sampled_batches": recall(hres)}
            log(f"hybrid {mode}: {hybrid_runs[mode]['value']:.0f} queries/s, recall "
                f"{hybrid_runs[mode]['recall_sampled_batches']:.4f}")
            del hres
    line = {
        "metric": f"stream join queries/sec and batch latency (200 batches, {size})",
        "value": nq / float(np.mean(walls)), "unit": "queries/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1000.0 * float(np.mean(walls)), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": workload, "queries": nq},
        "batch_ms_p50": float(np.percentile(lat, 50)), "batch_ms_p99": float(np.percentile(lat, 99)),
        "batch_ms_max": float(lat.max()), "pairs": int(pairs),
        "recall_sampled_batches": rec, "build_s": build_s,
        "tuned": {"start_tier": params.start_tier, "precision": params.precision},
        "device_runner": dev_runs["device"],
        "graph_replay": dev_runs["graph"],
    }
    if hybrid_runs:
        line["hybrid_modes"] = hybrid_runs
    print(json.dumps(line), flush=True)


def stream_insert(args, torch, vj, Q, X, starts, counts, eps, nq, workload, recall):
    """The stream with insertion: per step a fresh index over X alone (not
    timed), then for each batch its insertion and its join, timed together;
    per-batch wall ms of the insertion and of the join are reported apart."""
    def fresh():
        idx = vj.vj_build_merged_index(Q[:0], X, metric="l2", R=32, build_mst=False)
        torch.cuda.synchronize()
        return idx

    t = time.time()
    idx = fresh()
    build_s = time.time() - t
    log(f"index over X alone built in {build_s:.1f}s")
    params = vj.join_params()

    def one_pass(idx):
        res, ins_ms, join_ms = [], [], []
        for b in range(len(starts)):
            qb = Q[starts[b]:starts[b] + counts[b]]
            torch.cuda.synchronize()
            ts = time.perf_counter()
            idx.insert_queries(qb)
            torch.cuda.synchronize()
            tj = time.perf_counter()
            r, _ = vj.vj_join_batches(idx, [starts[b]], [counts[b]], [eps[b]], params=params)
            torch.cuda.synchronize()
            te = time.perf_counter()
            res.append(r[0])
            ins_ms.append(1000.0 * (tj - ts))
            join_ms.append(1000.0 * (te - tj))
            if (b + 1) % 20 == 0:
                log(f"  batch {b + 1}: insert {sum(ins_ms):.0f} ms, join {sum(join_ms):.0f} ms so far")
        return res, np.array(ins_ms), np.array(join_ms)

    for _ in range(args.warmup):  # a warm-up pass is a whole stream (0 allowed)
        one_pass(idx)
        idx = None
        idx = fresh()
    walls, ins, jn = [], [], []
    res = None
    for s in range(args.steps):
        res = None
        ts = time.perf_counter()
        res, i_ms, j_ms = one_pass(idx)
        walls.append(time.perf_counter() - ts)
        ins.append(i_ms)
        jn.append(j_ms)
        log(f"step {s}: {nq / walls[-1]:.0f} queries/s (insert {i_ms.sum():.0f} ms, join "
            f"{j_ms.sum():.0f} ms)")
        if s + 1 < args.steps:
            idx = None
            idx = fresh()
    ins, jn = np.concatenate(ins), np.concatenate(jn)
    lat = ins + jn
    rec = recall(res)
    pairs = sum(r.count() for r in res)
    line = {
        "metric": "stream with insertion: queries/sec and batch latency (insert + join)",
        "value": nq / float(np.mean(walls)), "unit": "queries/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1000.0 * float(np.mean(walls)), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": workload + "; index over X alone, each batch inserted before "
                   "its join", "queries": nq},
        "batch_ms_p50": float(np.percentile(lat, 50)), "batch_ms_p99": float(np.percentile(lat, 99)),
        "batch_ms_max": float(lat.max()),
        "insert_ms_p50": float(np.percentile(ins, 50)), "insert_ms_p99": float(np.percentile(ins, 99)),
        "join_ms_p50": float(np.percentile(jn, 50)), "join_ms_p99": float(np.percentile(jn, 99)),
        "insert_ms_total": float(ins.sum() / args.steps),
        "join_ms_total": float(jn.sum() / args.steps),
        "pairs": int(pairs), "recall_sampled_batches": rec, "x_only_build_s": build_s,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
