"""Seeded synthetic inputs for the merged-index ε-join.

This module only draws random vectors.  It computes no distance, no
threshold and nothing else of the join method; thresholds (ε) are
calibrated by the oracle from these vectors.  Both the CPU oracle and the
HIP path read their inputs from here, so the two sides always see the same
bytes.

The paper's evaluation uses public ANN-benchmark datasets (SIFT, GIST,
GloVe, the OOD sets COCO/ImageNet/LAION; dataset table of the experiments
section).  None of them is available here, so each generator below is a
stand-in with the same shape (rows, dimension) and the kind of structure
the paper relies on (clustered in-distribution data, heavy-tailed scales,
out-of-distribution query shifts).  No item of any benchmark is reproduced.

Every generator uses ``numpy.random.Generator(PCG64(seed))`` so the output
is identical on every machine with the same numpy build.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "Workload",
    "gaussian_mixture",
    "integer_mixture",
    "beta_mixture",
    "vmf_mixture",
    "stream_batches",
    "config_tiny",
    "config_mid",
    "config_highdim",
    "config_ood",
    "config_stream",
    "vmf_kappa_for_mean_cosine",
    "hub_chain",
    "separated_integer_case",
    "separated_float_case",
]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


@dataclass
class Workload:
    """A query set ``Q`` and a data set ``X`` (float32, row-major)."""

    name: str
    Q: np.ndarray
    X: np.ndarray
    metric: str  # "l2" or "ip"
    R: int  # merged-graph out-degree
    target_matches: float  # mean matches per query that ε is calibrated for
    eps_sample_seed: int
    eps_sample: int  # number of queries the ε calibration samples
    meta: dict

    @property
    def d(self) -> int:
        return int(self.X.shape[1])


# ---------------------------------------------------------------------------
# Mixture generators
# ---------------------------------------------------------------------------

def gaussian_mixture(n: int, means: np.ndarray, sigma: float, seed: int,
                     weights: np.ndarray | None = None,
                     chunk: int = 1 << 20) -> np.ndarray:
    """n points x = mu_c + sigma * N(0, I), c drawn from ``weights``."""
    rng = _rng(seed)
    k, d = means.shape
    p = np.full(k, 1.0 / k) if weights is None else weights
    out = np.empty((n, d), dtype=np.float32)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        c = rng.choice(k, size=hi - lo, p=p)
        noise = rng.standard_normal((hi - lo, d), dtype=np.float32)
        out[lo:hi] = means[c].astype(np.float32) + np.float32(sigma) * noise
    return out


def integer_mixture(n: int, means: np.ndarray, scales: np.ndarray,
                    weights: np.ndarray, seed: int, vmax: int = 218,
                    chunk: int = 1 << 18) -> np.ndarray:
    """Non-negative integer-valued points (stored as float32).

    x_j = clip(round(mu_cj + (s_j/3) N(0,1)), 0, vmax); the per-dimension
    scale s_j is heavy-tailed, so a few dimensions dominate distances, as in
    SIFT-like descriptors.
    """
    rng = _rng(seed)
    k, d = means.shape
    out = np.empty((n, d), dtype=np.float32)
    sd = (scales / 3.0).astype(np.float32)
    mu32 = means.astype(np.float32)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        c = rng.choice(k, size=hi - lo, p=weights)
        noise = rng.standard_normal((hi - lo, d), dtype=np.float32)
        v = np.rint(mu32[c] + sd[None, :] * noise)
        np.clip(v, 0, vmax, out=v)
        out[lo:hi] = v
    return out


def beta_mixture(n: int, a: np.ndarray, b: np.ndarray, seed: int,
                 chunk: int = 1 << 16) -> np.ndarray:
    """Points in [0,1]^d; cluster c has independent Beta(a_cj, b_cj) dims."""
    rng = _rng(seed)
    k, d = a.shape
    out = np.empty((n, d), dtype=np.float32)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        c = rng.integers(0, k, size=hi - lo)
        out[lo:hi] = rng.beta(a[c], b[c]).astype(np.float32)
    return out


def _bessel_ratio(nu: float, x: float, terms: int = 4000) -> float:
    """I_nu(x) / I_{nu-1}(x) from the recurrence R_nu = 1 / (2 nu / x + R_{nu+1})
    evaluated backwards (a continued fraction; no overflow or underflow)."""
    r = 0.0
    for k in range(terms, -1, -1):
        r = 1.0 / (2.0 * (nu + k) / x + r)
    return r


def vmf_kappa_for_mean_cosine(p: int, target: float) -> float:
    """κ of a von Mises-Fisher law on S^{p-1} whose E[cos(x, mu)] = target.

    E[cos] = A_p(κ) = I_{p/2}(κ) / I_{p/2-1}(κ) (Mardia & Jupp, 9.3),
    increasing in κ; solved by bisection.
    """
    lo, hi = 1e-6, 1e7
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if _bessel_ratio(p / 2.0, mid) < target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def _vmf_cosines(rng: np.random.Generator, n: int, p: int, kappa: float) -> np.ndarray:
    """Cosines W to the mean direction, by Wood's (1994) rejection sampler."""
    b = (-2.0 * kappa + math.sqrt(4.0 * kappa * kappa + (p - 1.0) ** 2)) / (p - 1.0)
    x0 = (1.0 - b) / (1.0 + b)
    c = kappa * x0 + (p - 1.0) * math.log(1.0 - x0 * x0)
    out = np.empty(n, dtype=np.float64)
    filled = 0
    while filled < n:
        m = max(16, int((n - filled) * 1.3))
        z = rng.beta((p - 1.0) / 2.0, (p - 1.0) / 2.0, size=m)
        w = (1.0 - (1.0 + b) * z) / (1.0 - (1.0 - b) * z)
        u = rng.random(m)
        ok = kappa * w + (p - 1.0) * np.log(1.0 - x0 * w) - c >= np.log(u)
        w = w[ok][: n - filled]
        out[filled:filled + w.size] = w
        filled += w.size
    return out


def vmf_mixture(n: int, means: np.ndarray, kappa: float, seed: int,
                chunk: int = 1 << 16) -> np.ndarray:
    """Unit vectors from an equal-weight mixture of vMF laws around ``means``."""
    rng = _rng(seed)
    k, p = means.shape
    out = np.empty((n, p), dtype=np.float32)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        m = hi - lo
        c = rng.integers(0, k, size=m)
        mu = means[c]
        w = _vmf_cosines(rng, m, p, kappa)
        v = rng.standard_normal((m, p))
        v -= np.sum(v * mu, axis=1, keepdims=True) * mu
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        x = w[:, None] * mu + np.sqrt(np.maximum(0.0, 1.0 - w * w))[:, None] * v
        x /= np.linalg.norm(x, axis=1, keepdims=True)
        out[lo:hi] = x.astype(np.float32)
    return out


def _random_unit(rng: np.random.Generator, k: int, p: int) -> np.ndarray:
    v = rng.standard_normal((k, p))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def _rotate_away(rng: np.random.Generator, mu: np.ndarray, angle_deg: float) -> np.ndarray:
    """mu' = cos(a) mu + sin(a) u with u a random unit vector orthogonal to mu."""
    u = rng.standard_normal(mu.shape)
    u -= np.sum(u * mu, axis=1, keepdims=True) * mu
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    a = math.radians(angle_deg)
    out = math.cos(a) * mu + math.sin(a) * u
    return out / np.linalg.norm(out, axis=1, keepdims=True)


# ---------------------------------------------------------------------------
# Named workloads.  ``scale`` shrinks row counts (never d) for CPU tests.
# ---------------------------------------------------------------------------

def _scaled(n: int, scale: float) -> int:
    return max(1, int(round(n * scale)))


def config_tiny(scale: float = 1.0) -> Workload:
    """X=10,000, Q=1,000, d=32; one 16-component Gaussian mixture, L2, R=16.

    Means ~ N(0, 4 I) (seed 100), sigma = 1; X seed 101, Q seed 102.
    """
    d, k = 32, 16
    means = 2.0 * _rng(100).standard_normal((k, d))
    X = gaussian_mixture(_scaled(10_000, scale), means, 1.0, 101)
    Q = gaussian_mixture(_scaled(1_000, scale), means, 1.0, 102)
    return Workload("tiny", Q, X, "l2", 16, 10.0, 103, Q.shape[0],
                    {"clusters": k, "sigma": 1.0})


def mid_params(d: int = 128, k: int = 256):
    """Mixture parameters of the mid-size integer workload (seed 200)."""
    rng = _rng(200)
    weights = rng.dirichlet(np.ones(k))
    scales = np.exp(rng.normal(math.log(20.0), 0.75, size=d))
    means = scales[None, :] * rng.exponential(1.0, size=(k, d))
    return weights, scales, means


def config_mid(scale: float = 1.0) -> Workload:
    """X=1,000,000, Q=100,000, d=128 integer entries in [0,218], L2, R=32.

    256 clusters with Dirichlet(1) weights (long-tailed cluster sizes, hence
    long-tailed match counts); per-dimension scale s_j ~ LogNormal(ln 20,
    0.75); mu_cj = s_j Exp(1); x = clip(round(mu_c + (s_j/3) N(0,1)), 0, 218).
    X seed 201, Q seed 202; ε is calibrated on 2,000 queries (seed 203) for
    a mean of 50 matches.  Stands in for SIFT (1M x 128).
    """
    weights, scales, means = mid_params()
    X = integer_mixture(_scaled(1_000_000, scale), means, scales, weights, 201)
    Q = integer_mixture(_scaled(100_000, scale), means, scales, weights, 202)
    return Workload("mid", Q, X, "l2", 32, 50.0, 203, min(2_000, Q.shape[0]),
                    {"clusters": 256, "value_max": 218, "integer": True})


def config_highdim(scale: float = 1.0) -> Workload:
    """X=1,000,000, Q=10,000, d=960 in [0,1]; 100-cluster Beta mixture, L2.

    a_cj, b_cj ~ U(0.5, 5) (seed 300); X seed 301, Q seed 302; ε for a mean
    of 10 matches, calibrated on 1,000 queries (seed 303).  Stands in for
    GIST (1M x 960).
    """
    d, k = 960, 100
    rng = _rng(300)
    a = rng.uniform(0.5, 5.0, size=(k, d))
    b = rng.uniform(0.5, 5.0, size=(k, d))
    X = beta_mixture(_scaled(1_000_000, scale), a, b, 301)
    Q = beta_mixture(_scaled(10_000, scale), a, b, 302)
    return Workload("highdim", Q, X, "l2", 32, 10.0, 303, min(1_000, Q.shape[0]),
                    {"clusters": k})


def config_ood(scale: float = 1.0, train: bool = False, ood_mean_cos: float = 0.92) -> Workload:
    """X=2,000,000 unit vectors, d=768, 512-cluster vMF mixture, inner product.

    Means uniform on the sphere (seed 401); κ gives E[cos to mean] = 0.7.
    Q=200,000: 70% from the same mixture, 30% from means rotated 40 degrees
    away (seed 403), concentrated at E[cos to the shifted mean] =
    ``ood_mean_cos``.  With 0.92 an OOD query's nearest nodes in Q ∪ X are
    other OOD queries (its merged-graph neighbourhood holds no data node),
    yet at the shared ε (pooled mean of 20 matches) it has about as many
    matches as an in-distribution query.  ``train=True`` gives 125,000
    training queries from the same recipe with seed 404 (never the test
    queries).  Stands in for the OOD sets (COCO, ImageNet, LAION).
    """
    d, k = 768, 512
    means = _random_unit(_rng(401), k, d)
    kappa = vmf_kappa_for_mean_cosine(d, 0.7)
    X = vmf_mixture(_scaled(2_000_000, scale), means, kappa, 402)
    nq = _scaled(125_000 if train else 200_000, scale)
    qseed = 404 if train else 403
    n_ood = int(round(0.3 * nq))
    rng = _rng(qseed + 1000)
    shifted = _rotate_away(rng, means, 40.0)
    q_id = vmf_mixture(nq - n_ood, means, kappa, qseed)
    q_ood = vmf_mixture(n_ood, shifted, vmf_kappa_for_mean_cosine(d, ood_mean_cos), qseed + 2000)
    Q = np.concatenate([q_id, q_ood], axis=0)
    is_ood = np.zeros(nq, dtype=bool)
    is_ood[nq - n_ood:] = True
    return Workload("ood", Q, X, "ip", 32, 20.0, 405, min(2_000, nq),
                    {"clusters": k, "kappa": kappa, "is_ood": is_ood, "ood_mean_cos": ood_mean_cos})


def config_stream(scale: float = 1.0, n_batches: int = 200) -> Workload:
    """X=10,000,000, d=96, 1,024-cluster Gaussian mixture (means ~ N(0,4I)).

    Queries arrive in ``n_batches`` batches with sizes log-uniform in
    [1e3, 1e5] (seed 502) and per-batch target mean matches log-uniform in
    [5, 200] (seed 503); batch b's queries use seed 600+b.  All batches are
    concatenated into Q; ``meta['batches']`` holds (start, count, target).
    """
    d, k = 96, 1024
    means = 2.0 * _rng(500).standard_normal((k, d))
    X = gaussian_mixture(_scaled(10_000_000, scale), means, 1.0, 501)
    sizes = np.floor(np.exp(_rng(502).uniform(math.log(1e3), math.log(1e5), size=n_batches)))
    sizes = np.maximum(1, np.round(sizes * scale)).astype(np.int64)
    targets = np.exp(_rng(503).uniform(math.log(5.0), math.log(200.0), size=n_batches))
    parts, batches, start = [], [], 0
    for bi in range(n_batches):
        parts.append(gaussian_mixture(int(sizes[bi]), means, 1.0, 600 + bi))
        batches.append((start, int(sizes[bi]), float(targets[bi])))
        start += int(sizes[bi])
    Q = np.concatenate(parts, axis=0)
    return Workload("stream", Q, X, "l2", 32, float(np.mean(targets)), 504,
                    min(1_000, Q.shape[0]), {"clusters": k, "batches": batches})


def stream_batches(w: Workload):
    """(start, count, target_mean) of each batch of a stream workload."""
    return list(w.meta["batches"])


def width_case(d: int, n_x: int, n_q: int, integer: bool, seed: int,
               vmax: int = 218) -> Workload:
    """Small build-parity inputs of width d: the mid workload's integer
    recipe at width d (16 clusters, values clipped to [0, vmax]) or a
    16-component Gaussian mixture with means ~ N(0, 4 I) and sigma = 1.
    X uses ``seed``, Q ``seed + 1``; R = 16, L2."""
    if integer:
        weights, scales, means = mid_params(d, 16)
        X = integer_mixture(n_x, means, scales, weights, seed, vmax=vmax)
        Q = integer_mixture(n_q, means, scales, weights, seed + 1, vmax=vmax)
    else:
        means = 2.0 * _rng(seed + 2).standard_normal((16, d))
        X = gaussian_mixture(n_x, means, 1.0, seed)
        Q = gaussian_mixture(n_q, means, 1.0, seed + 1)
    return Workload(f"width{d}", Q, X, "l2", 16, 10.0, seed + 3, n_q,
                    {"integer": integer, "value_max": vmax})


def separated_integer_case(n_x: int = 12_000, n_q: int = 1_200, d: int = 64, k: int = 24,
                           sigma: float = 4.0, seed: int = 610) -> Workload:
    """Well-separated integer clusters (a build edge case: most groups of
    nodes are far from most others).  k means uniform in [20, 235]^d
    (seed), points round(mean + sigma N(0, I)) clipped to [0, 255], X with
    seed + 1, Q with seed + 2, equal cluster weights; L2, R = 16.  Every
    squared distance is an integer below 2^24."""
    means = _rng(seed).uniform(20.0, 235.0, size=(k, d))
    scales = np.full(d, 3.0 * sigma)  # integer_mixture draws (scale / 3) N(0, 1)
    weights = np.full(k, 1.0 / k)
    X = integer_mixture(n_x, means, scales, weights, seed + 1, vmax=255)
    Q = integer_mixture(n_q, means, scales, weights, seed + 2, vmax=255)
    return Workload("separated", Q, X, "l2", 16, 10.0, seed + 3, n_q,
                    {"integer": True, "clusters": k, "sigma": sigma})


def separated_float_case(n_x: int = 12_000, n_q: int = 1_200, d: int = 64, k: int = 24,
                         sigma: float = 4.0, seed: int = 620) -> Workload:
    """The same geometry with float32 values: k means uniform in
    [20, 235]^d (seed), points mean + sigma N(0, I) (X seed + 1, Q seed + 2,
    equal weights); L2, R = 16."""
    means = _rng(seed).uniform(20.0, 235.0, size=(k, d))
    X = gaussian_mixture(n_x, means, sigma, seed + 1)
    Q = gaussian_mixture(n_q, means, sigma, seed + 2)
    return Workload("separated_float", Q, X, "l2", 16, 10.0, seed + 3, n_q,
                    {"integer": False, "clusters": k, "sigma": sigma})


def hub_chain(d: int = 1024, window: int = 60, n_queries: int = 8) -> Workload:
    """A graph-build edge case: one hub with more reverse-edge candidates
    than a node usually has (0/1 integer data, exact in every precision).

    X[0] is the origin (the hub); X[1 + t], t = 0..d-1, is the 0/1 vector
    with ones at the ``window`` cyclically consecutive coordinates starting
    at t.  Every chain vector lies at the same distance sqrt(window) from
    the hub, and two chain vectors at cyclic offset k differ in 2 min(k,
    window) coordinates.  Q holds ``n_queries`` far-away points (value 200 in
    one coordinate).  No randomness.
    """
    X = np.zeros((1 + d, d), np.float32)
    for t in range(d):
        X[1 + t, (t + np.arange(window)) % d] = 1.0
    Q = np.zeros((n_queries, d), np.float32)
    for i in range(n_queries):
        Q[i, (i * 97) % d] = 200.0
    return Workload("hub_chain", Q, X, "l2", 32, 1.0, 0, n_queries,
                    {"window": window, "integer": True})
