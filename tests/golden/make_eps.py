"""Write tests/golden/eps.json: the threshold of each named workload.

eps is calibrated by the oracle alone (oracle.calibrate_eps) on the
workload's seeded query sample, for the workload's target mean match count;
a checksum of the generated vectors is stored beside it so a change of the
generator is detected.  Run:  python tests/golden/make_eps.py [names...]
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "eps.json")

MAKERS = {
    "tiny": lambda: workloads.config_tiny(),
    "mid": lambda: workloads.config_mid(),
    # the OOD workload at 1/10 scale (X = 200,000 x 768, 20,000 test queries)
    "ood": lambda: workloads.config_ood(scale=0.1),
    # and at its stated size (X = 2,000,000 x 768, 200,000 test queries)
    "ood_full": lambda: workloads.config_ood(scale=1.0),
    # the high-dimensional workload (X = 1,000,000 x 960, 10,000 queries)
    "highdim": lambda: workloads.config_highdim(),
}
SCALES = {"ood": 0.1}

# the batched stream: 200 batches, eps per batch for the batch's target
# mean, calibrated on a few of its queries (seed 504 + batch).  "stream" is
# the 1/10 scale (X = 1,000,000 x 96, batches of 100..10,000 queries, 50
# sampled per batch); "stream_full" the stated size (X = 10,000,000 x 96,
# batches of 1,000..100,000 queries, 20 sampled per batch)
STREAM_SCALE, STREAM_BATCHES, STREAM_SAMPLE = 0.1, 200, 50
STREAM_FULL_SAMPLE = 20


def make_stream(data, scale=STREAM_SCALE, sample=STREAM_SAMPLE, key="stream"):
    t = time.time()
    w = workloads.config_stream(scale=scale, n_batches=STREAM_BATCHES)
    eps = []
    for b, (start, count, target) in enumerate(workloads.stream_batches(w)):
        r = np.random.default_rng(504 + b)
        m = min(count, sample)
        idx = start + np.sort(r.choice(count, size=m, replace=False))
        eps.append(oracle.calibrate_eps(w.Q[idx], w.X, target, w.metric))
    data[key] = {"eps": eps, "scale": scale, "n_batches": STREAM_BATCHES,
                      "sample_per_batch": sample, "metric": w.metric,
                      "Q_sha": checksum(w.Q), "X_sha": checksum(w.X),
                      "nq": int(w.Q.shape[0]), "nx": int(w.X.shape[0]), "d": w.d}
    print(f"{key}: {len(eps)} batches, eps {min(eps):.4f}..{max(eps):.4f} ({time.time() - t:.1f}s)",
          flush=True)


def checksum(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()[:16]


def sample(w):
    r = np.random.default_rng(w.eps_sample_seed)
    n = min(w.eps_sample, w.Q.shape[0])
    return np.sort(r.choice(w.Q.shape[0], size=n, replace=False))


def main(names):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in names:
        if name in ("stream", "stream_full"):
            if name == "stream":
                make_stream(data)
            else:
                make_stream(data, 1.0, STREAM_FULL_SAMPLE, "stream_full")
            with open(OUT, "w") as f:
                json.dump(data, f, indent=1, sort_keys=True)
            continue
        t = time.time()
        w = MAKERS[name]()
        idx = sample(w)
        eps = oracle.calibrate_eps(w.Q[idx], w.X, w.target_matches, w.metric,
                                   integer=bool(w.meta.get("integer")))
        data[name] = {"eps": eps, "metric": w.metric, "target_mean_matches": w.target_matches,
                      "scale": SCALES.get(name, 1.0),
                      "sample_queries": int(idx.size), "sample_seed": w.eps_sample_seed,
                      "Q_sha": checksum(w.Q), "X_sha": checksum(w.X),
                      "nq": int(w.Q.shape[0]), "nx": int(w.X.shape[0]), "d": w.d}
        print(f"{name}: eps={eps!r} ({time.time() - t:.1f}s)", flush=True)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or list(MAKERS) + ["stream", "stream_full"])
