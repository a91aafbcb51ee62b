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
    ap.add_argument("--copy-calib", action="store_true",
                    help="run a plain 1 GiB device copy first (HBM counter calibration)")
    ap.add_argument("--ood", action="store_true",
                    help="instead of the headline: the OOD inner-product workload at 1/10 scale; "
                         "MI-BFS, MI+Adapt, forced hybrid and learned routing compared")
    ap.add_argument("--modes", action="store_true",
                    help="instead of the headline: MI, MI+SWS, MI+HWS on the merged index against "
                         "INLJ, SWS, HWS on separate indexes, on the headline workload")
    ap.add_argument("--stream", action="store_true",
                    help="instead of the headline: the batched stream workload at 1/10 scale "
                         "(200 batches, p50/p99 batch latency)")
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
        cpu = {"value": reps * nq / cpu_s, "unit": "queries/s", "cores": cores,
               "kind": "oracle",
               "sample": f"all {nq} queries x {reps} repetitions ({cpu_s:.1f}s): self-seeded BFS "
                         f"merged-index join in fp64 with OpenMP over queries, same graph and eps; "
                         f"{npairs} pairs per repetition"}
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
    log(f"merged index {bm:.2f}s, separate indexes {bs:.2f}s, NN-Map {bn:.2f}s")
    gt_qx, _ = vj.vj_bruteforce_join(Q, X, eps, precision="bf16").export(sorted=True)
    gt_keys = gt_qx[:, 0].to(torch.int64) * nx + gt_qx[:, 1].to(torch.int64)
    n_gt = int(gt_keys.numel())
    modes = {
        "MI": (merged, {}), "MI+SWS": (merged, {"work_sharing": "soft"}),
        "MI+HWS": (merged, {"work_sharing": "hard"}),
        "INLJ": (sep, {"work_sharing": "none"}), "SWS": (sep, {"work_sharing": "soft"}),
        "HWS": (sep, {"work_sharing": "hard"}),
        "NN-Map": (sep, {"work_sharing": "nnmap"}),
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
            "build_s": {"merged": bm, "separate": bs, "nnmap": bn}, "ground_truth_pairs": n_gt,
            "modes": out}
    print(json.dumps(line), flush=True)


def ood_main(args, torch, workloads, vj):
    """OOD queries (30 % from shifted means), inner product: the paper's MI
    (BFS), MI+Adapt (d1/d2 rule), hybrid for every query, and the learned
    router trained on separate training queries indexed in their own merged
    graph (records: per-query recall of budget-mode joins against the exact
    join)."""
    golden = json.load(open(os.path.join(ROOT, "tests", "golden", "eps.json")))["ood"]
    scale = golden["scale"]
    t0 = time.time()
    w = workloads.config_ood(scale=scale)
    wt = workloads.config_ood(scale=scale, train=True)
    for key, arr in (("Q_sha", w.Q), ("X_sha", w.X)):
        sha = hashlib.sha256(np.ascontiguousarray(arr).tobytes()).hexdigest()[:16]
        if sha != golden[key]:
            raise SystemExit(f"generated data differs from the calibrated data ({key})")
    eps = golden["eps"]
    nq, nt = w.Q.shape[0], wt.Q.shape[0]
    log(f"ood: X {w.X.shape}, {nq} test and {nt} training queries, eps={eps} ({time.time() - t0:.1f}s)")
    dev = torch.device("cuda:0")
    X = torch.from_numpy(w.X).to(dev)
    Qt = torch.from_numpy(w.Q).to(dev)
    Qr = torch.from_numpy(wt.Q).to(dev)
    idx = vj.vj_build_merged_index(Qt, X, metric="ip", R=w.R)
    idx_tr = vj.vj_build_merged_index(Qr, X, metric="ip", R=wt.R)
    torch.cuda.synchronize()
    budgets = (0, 16, 64, 256)
    # training records
    t = time.time()
    F = vj.vj_join_features(idx_tr, eps, metric="ip")
    gt_tr, _ = vj.vj_bruteforce_join(Qr, X, eps, metric="ip", precision="bf16").export()
    gtc = torch.bincount(gt_tr[:, 0].long(), minlength=nt).float()
    Y = []
    for b in budgets:
        r = vj.vj_join(idx_tr, eps, metric="ip", hybrid="budget",
                       budget=torch.full((nt,), b, dtype=torch.int32, device=dev))
        cnt = r.stats()[:, 0].float()
        Y.append(torch.where(gtc > 0, cnt / gtc.clamp(min=1), torch.ones_like(cnt)))
    Y = torch.stack(Y, 1).contiguous()
    pred = vj.Predictor(w.d + 8, 256, 256, len(budgets), seed=1)
    pred.fit_normalization(F)
    torch.cuda.synchronize()
    ts = time.time()
    losses = pred.train(F, Y, epochs=40, batch=512, lr=1e-3, seed=2)
    torch.cuda.synchronize()
    train_s = time.time() - ts
    log(f"records + training: {time.time() - t:.1f}s (training {train_s:.1f}s, "
        f"loss {losses[0]:.4f} -> {losses[-1]:.4f})")
    target = 0.95
    vj.vj_index_attach_predictor(idx, pred, recall_target=target, budgets=budgets)
    gt, _ = vj.vj_bruteforce_join(Qt, X, eps, metric="ip", precision="bf16").export()
    n_gt = int(gt.shape[0])
    is_ood = torch.from_numpy(w.meta["is_ood"]).to(dev)
    gt_ood = int(is_ood[gt[:, 0].long()].sum().item())
    modes = {"MI (BFS)": {}, "MI+Adapt": {"hybrid": "adapt"}, "hybrid for all": {"hybrid": "force"},
             "learned": {"hybrid": "learned"}}
    out = {}
    for name, kw in modes.items():
        for _ in range(max(1, args.warmup)):
            vj.vj_join(idx, eps, metric="ip", **kw)
        torch.cuda.synchronize()
        walls = []
        res = None
        for _ in range(args.steps):
            res = None
            torch.cuda.synchronize()
            t = time.perf_counter()
            res = vj.vj_join(idx, eps, metric="ip", **kw)
            torch.cuda.synchronize()
            walls.append(time.perf_counter() - t)
        qx, _ = res.export()
        st = res.stats().cpu().numpy()
        found_ood = int(is_ood[qx[:, 0].long()].sum().item())
        out[name] = {"qps": nq / float(np.mean(walls)), "ms": 1000 * float(np.mean(walls)),
                     "recall": int(qx.shape[0]) / max(1, n_gt),
                     # null when the exact join has no pair of an OOD query
                     "recall_ood_queries": found_ood / gt_ood if gt_ood else None,
                     "hybrid_queries": int(st[:, 5].sum()), "routed_exact": int(((st[:, 7] & 2) > 0).sum())}
        log(f"{name}: {out[name]}")
    line = {"metric": "OOD join queries/sec and recall by mode (X=200k x 768, IP)",
            "value": out["learned"]["qps"], "unit": "queries/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": "OOD at 1/10 scale: X=200,000 unit vectors d=768 (512-mean vMF "
                                   "mixture); 20,000 test queries, 30 % from means rotated 40 deg; "
                                   "inner product, eps for 20 mean matches; predictor trained on "
                                   "12,500 separate queries", "recall_target": target},
            "modes": out, "train_s": train_s, "ground_truth_pairs": n_gt,
            "ground_truth_pairs_of_ood_queries": gt_ood}
    print(json.dumps(line), flush=True)


def stream_main(args, torch, workloads, vj):
    """The batched stream: one merged index over X and every batch's queries,
    then the batches joined one after the other (vj_join_batches), each at
    its own eps (oracle-calibrated, tests/golden/eps.json)."""
    golden = json.load(open(os.path.join(ROOT, "tests", "golden", "eps.json")))["stream"]
    t0 = time.time()
    w = workloads.config_stream(scale=golden["scale"], n_batches=golden["n_batches"])
    for key, arr in (("Q_sha", w.Q), ("X_sha", w.X)):
        sha = hashlib.sha256(np.ascontiguousarray(arr).tobytes()).hexdigest()[:16]
        if sha != golden[key]:
            raise SystemExit(f"generated data differs from the calibrated data ({key})")
    batches = workloads.stream_batches(w)
    starts = [b[0] for b in batches]
    counts = [b[1] for b in batches]
    eps = golden["eps"]
    log(f"stream: X {w.X.shape}, {len(batches)} batches, {w.Q.shape[0]} queries ({time.time() - t0:.1f}s)")
    dev = torch.device("cuda:0")
    Q = torch.from_numpy(w.Q).to(dev)
    X = torch.from_numpy(w.X).to(dev)
    t = time.time()
    idx = vj.vj_build_merged_index(Q, X, metric="l2", R=w.R)
    torch.cuda.synchronize()
    build_s = time.time() - t
    log(f"merged index over {w.Q.shape[0] + w.X.shape[0]} nodes built in {build_s:.1f}s")
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
    nq = int(sum(counts))
    pairs = sum(r.count() for r in res)
    # recall on every 20th batch against the exact join
    found = exact = 0
    for b in range(0, len(batches), 20):
        qb = Q[starts[b]:starts[b] + counts[b]]
        gt = vj.vj_bruteforce_join(qb, X, eps[b])
        exact += gt.count()
        found += res[b].count()
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
    line = {
        "metric": "stream join queries/sec and batch latency (200 batches, X=1M x 96)",
        "value": nq / float(np.mean(walls)), "unit": "queries/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1000.0 * float(np.mean(walls)), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "stream at 1/10 scale: X=1,000,000 d=96 1,024-cluster Gaussian "
                               "mixture; 200 batches of 100..10,000 queries (log-uniform), eps "
                               "per batch for 5..200 mean matches", "queries": nq},
        "batch_ms_p50": float(np.percentile(lat, 50)), "batch_ms_p99": float(np.percentile(lat, 99)),
        "batch_ms_max": float(lat.max()), "pairs": int(pairs),
        "recall_sampled_batches": found / max(1, exact), "build_s": build_s,
        "tuned": {"start_tier": params.start_tier, "precision": params.precision},
        "device_runner": dev_runs["device"],
        "graph_replay": dev_runs["graph"],
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
