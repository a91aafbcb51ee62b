"""FP64 CPU oracle for the merged-index ε-join (ctypes wrapper of oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may use it; the library under
``paper_2603_16360_amd`` never does, and shares no code with it.

Every function states the passage of the paper it follows; see oracle.c for
the readings of the points the paper leaves open.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

METRICS = {"l2": 0, "ip": 1}
WS = {"self": 0, "none": 0, "soft": 1, "hard": 2, "nnmap": 3}
HYB = {"off": 0, "force": 1, "adapt": 2, "budget": 3}
STAT_FIELDS = ("pairs", "n_dist", "n_expanded", "h_pops", "ood", "hybrid",
               "visited_data", "fragile")


def build(verbose: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (plain -O2, no fast-math)."""
    from .build import build_oracle
    return build_oracle(verbose=verbose)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = C.CDLL(_LIB_PATH)
        _declare(_lib)
    return _lib


_f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_i64, _int, _dbl = C.c_int64, C.c_int, C.c_double


class _Cfg(C.Structure):
    _fields_ = [("work_sharing", C.c_int32), ("hybrid", C.c_int32),
                ("hybrid_beam", C.c_int32), ("conv_threshold", C.c_int32),
                ("ood_ratio", C.c_double), ("uncertain_policy", C.c_int32),
                ("uncertain_rel", C.c_double), ("shuffle_seed", C.c_uint64),
                ("fragile_rel", C.c_double), ("merged", C.c_int32), ("greedy_beam", C.c_int32)]


def _declare(L):
    L.or_nlj.restype = _i64
    L.or_nlj.argtypes = [_f32p, _i64, _f32p, _i64, _int, _int, _dbl, _i64, _i32p, _i32p, _f64p]
    L.or_nlj_counts.restype = None
    L.or_nlj_counts.argtypes = [_f32p, _i64, _f32p, _i64, _int, _int, _dbl, _i64p]
    L.or_pair_dists.restype = None
    L.or_pair_dists.argtypes = [_f32p, _f32p, _int, _int, _i64, _i32p, _i32p, _f64p]
    L.or_dist_matrix.restype = None
    L.or_dist_matrix.argtypes = [_f32p, _i64, _f32p, _i64, _int, _int, _f64p]
    L.or_pooled_kth.restype = _int
    L.or_pooled_kth.argtypes = [_f32p, _i64, _f32p, _i64, _int, _int, _i64, _i64,
                                C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.or_knn.restype = None
    L.or_knn.argtypes = [_f32p, _i64, _int, _int, _i32p, _f64p]
    L.or_rng_prune.restype = _int
    L.or_rng_prune.argtypes = [_f32p, _int, _i64, _i32p, _f64p, _int, _int, _i32p]
    L.or_build_merged.restype = _i64
    L.or_build_merged.argtypes = [_f32p, _i64, _int, _int, _int, _i32p, _f64p,
                                  C.POINTER(C.c_int32)]
    L.or_mst_parents.restype = _dbl
    L.or_mst_parents.argtypes = [_f32p, _i64, _i64, _int, _i32p, _int, C.c_int32,
                                 _i32p, _i32p]
    L.or_join.restype = _i64
    L.or_join.argtypes = [_f32p, _i64, _i64, _int, _int, _i32p, _int, C.c_int32,
                          C.c_void_p, _i32p, _i64, _dbl, C.POINTER(_Cfg), C.c_void_p,
                          C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                          _i64, _i32p, _i32p, _f64p, _i32p]
    L.or_splitmix64.restype = C.c_uint64
    L.or_splitmix64.argtypes = [C.c_uint64, C.c_uint64]
    L.or_levels.restype = None
    L.or_levels.argtypes = [_i64, C.c_uint64, _int, np.ctypeslib.ndpointer(np.int8, flags="C_CONTIGUOUS")]
    L.or_descend.restype = None
    L.or_descend.argtypes = [_f32p, _i64, _i64, _int, _int, _int, _i64p, _i32p, _i32p, _int,
                             _i32p, _i32p, _i64, _i32p, _i32p]
    L.or_insert_batch.restype = _i64
    L.or_insert_batch.argtypes = [_f32p, _i64, _i64, _int, _int, _int, _i32p, _f64p, C.c_int32]
    L.or_nnmap.restype = None
    L.or_nnmap.argtypes = [_f32p, _i64, _i64, _int, _int, _i32p, _int, _dbl, _i32p, _f64p,
                           np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")]
    L.or_join_self_counts.restype = None
    L.or_join_self_counts.argtypes = [_f32p, _i64, _i64, _int, _int, _i32p, _int,
                                      C.c_int32, _i32p, _i64, _dbl, _i64p]
    L.or_features.restype = None
    L.or_features.argtypes = [_f32p, _i64, _i64, _int, _int, _i32p, _int, C.c_int32, _i32p,
                              _i64, _dbl, _f64p]
    L.or_mlp_forward.restype = None
    L.or_mlp_forward.argtypes = [_int] * 5 + [_f64p] * 7 + [_f64p]
    L.or_mlp_bce_backward.restype = _dbl
    L.or_mlp_bce_backward.argtypes = ([_int] * 5 + [_f64p] * 7 + [_f64p, C.c_void_p]
                                      + [_f64p] * 6)
    L.or_adam_step.restype = None
    L.or_adam_step.argtypes = [_i64, _f64p, _f64p, _f64p, _f64p, _i64, _dbl, _dbl, _dbl, _dbl]


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


# ---------------------------------------------------------------------------
# O1: Definition 1, the exact join
# ---------------------------------------------------------------------------

def nlj(Q, X, eps: float, metric: str = "l2"):
    """Exact join {(i, j): dist(Q_i, X_j) < eps} in (i, j) order.

    Returns (qi int32, xj int32, dist float64)."""
    Q, X = _f32(Q), _f32(X)
    L = lib()
    e = np.empty(0, np.int32)
    cnt = L.or_nlj(Q, Q.shape[0], X, X.shape[0], Q.shape[1], METRICS[metric], eps,
                   0, e, e, np.empty(0, np.float64))
    oq = np.empty(cnt, np.int32)
    ox = np.empty(cnt, np.int32)
    od = np.empty(cnt, np.float64)
    L.or_nlj(Q, Q.shape[0], X, X.shape[0], Q.shape[1], METRICS[metric], eps, cnt,
             oq, ox, od)
    return oq, ox, od


def nlj_counts(Q, X, eps: float, metric: str = "l2") -> np.ndarray:
    Q, X = _f32(Q), _f32(X)
    out = np.empty(Q.shape[0], np.int64)
    lib().or_nlj_counts(Q, Q.shape[0], X, X.shape[0], Q.shape[1], METRICS[metric],
                        eps, out)
    return out


def pair_dists(Q, X, qi, xj, metric: str = "l2") -> np.ndarray:
    """Exact fp64 distance of each listed pair."""
    Q, X = _f32(Q), _f32(X)
    qi = np.ascontiguousarray(qi, np.int32)
    xj = np.ascontiguousarray(xj, np.int32)
    out = np.empty(qi.shape[0], np.float64)
    lib().or_pair_dists(Q, X, Q.shape[1], METRICS[metric], qi.shape[0], qi, xj, out)
    return out


def dist_matrix(A, B, metric: str = "l2") -> np.ndarray:
    A, B = _f32(A), _f32(B)
    out = np.empty((A.shape[0], B.shape[0]), np.float64)
    lib().or_dist_matrix(A, A.shape[0], B, B.shape[0], A.shape[1], METRICS[metric], out)
    return out


def pooled_kth(Q, X, k: int, metric: str = "l2", M: int | None = None):
    """k-th and (k+1)-th smallest of all pooled pair distances (1-based)."""
    Q, X = _f32(Q), _f32(X)
    M = M or max(64, min(X.shape[0], 8 * (k // max(1, Q.shape[0]) + 1)))
    L = lib()
    while True:
        vk, vk1 = C.c_double(), C.c_double()
        rc = L.or_pooled_kth(Q, Q.shape[0], X, X.shape[0], Q.shape[1], METRICS[metric],
                             k, M, C.byref(vk), C.byref(vk1))
        if rc == 0 or M >= X.shape[0]:
            return vk.value, vk1.value
        if rc == 2:
            raise MemoryError("or_pooled_kth")
        M = min(X.shape[0], M * 4)


def calibrate_eps(Q, X, target_mean: float, metric: str = "l2",
                  integer: bool = False) -> float:
    """ε for a target mean match count over the queries Q (a sample).

    Real-valued data: the midpoint of the k-th and (k+1)-th smallest pooled
    distances, k = round(target * |Q|).  Integer data (L2): with D_k the k-th
    smallest squared distance (an integer), ε = sqrt(D_k + 0.5), so that no
    squared distance ever equals ε².
    """
    k = int(round(target_mean * Q.shape[0]))
    vk, vk1 = pooled_kth(Q, X, k, metric)
    if integer and metric == "l2":
        dk = round(vk * vk)
        return float(np.sqrt(dk + 0.5))
    return 0.5 * (vk + vk1)


# ---------------------------------------------------------------------------
# O2: merged-graph build (Section 4.3, Appendix C)
# ---------------------------------------------------------------------------

def knn(V, K: int):
    V = _f32(V)
    ids = np.empty((V.shape[0], K), np.int32)
    dd = np.empty((V.shape[0], K), np.float64)
    lib().or_knn(V, V.shape[0], V.shape[1], K, ids, dd)
    return ids, dd


def rng_prune(V, u: int, cand, cd, R: int):
    V = _f32(V)
    cand = np.ascontiguousarray(cand, np.int32)
    cd = np.ascontiguousarray(cd, np.float64)
    out = np.full(R, -1, np.int32)
    k = lib().or_rng_prune(V, V.shape[1], u, cand, cd, cand.shape[0], R, out)
    return out[:k]


@dataclass
class Graph:
    adj: np.ndarray        # [N][R] int32, -1 padded; data ids [0, nx), queries after
    elen: np.ndarray       # [N][R] float64 edge lengths
    entry: int
    repairs: int           # connectivity-repair edges added


def build_merged(Q, X, R: int, Kc: int | None = None) -> Graph:
    """Merged graph over V = [X; Q]: data ids 0..nx-1, query i is node nx+i."""
    V = np.ascontiguousarray(np.concatenate([_f32(X), _f32(Q)], axis=0))
    Kc = Kc or 2 * R
    n = V.shape[0]
    adj = np.empty((n, R), np.int32)
    elen = np.empty((n, R), np.float64)
    ent = C.c_int32()
    rep = lib().or_build_merged(V, n, V.shape[1], R, Kc, adj, elen, C.byref(ent))
    return Graph(adj, elen, int(ent.value), int(rep))


def build_separate(Q, X, R: int, Kc: int | None = None):
    """Separate indexes (cfg.merged = false): the data graph G_X and the
    query graph G_Q, each built by the same recipe as the merged graph over
    its own set alone.  Returns (adj [nx + nq][R] with rows 0..nx-1 = G_X
    in data ids and rows nx.. = G_Q in node ids nx + j, entry of G_X, the
    two Graphs)."""
    gx = build_merged(np.zeros((0, X.shape[1]), np.float32), X, R, Kc)
    gq = build_merged(np.zeros((0, Q.shape[1]), np.float32), Q, R, Kc)
    nx = X.shape[0]
    adjq = np.where(gq.adj >= 0, gq.adj + nx, -1).astype(np.int32)
    return np.ascontiguousarray(np.concatenate([gx.adj, adjq])), gx.entry, gx, gq


def insert_batch(Q_old, X, adj, entry: int, Q_new, R: int | None = None, Kc: int | None = None):
    """Incremental insertion of the query batch Q_new into the merged graph
    adj over [X; Q_old] (see or_insert_batch).  Returns the Graph over
    [X; Q_old; Q_new] (entry unchanged)."""
    V = np.ascontiguousarray(np.concatenate([_f32(X), _f32(Q_old), _f32(Q_new)], axis=0))
    R = R or adj.shape[1]
    Kc = Kc or 2 * R
    n_old = X.shape[0] + Q_old.shape[0]
    n = V.shape[0]
    out = np.full((n, R), -1, np.int32)
    out[:n_old] = adj
    elen = np.empty((n, R), np.float64)
    rep = lib().or_insert_batch(V, n_old, n - n_old, V.shape[1], R, Kc, out, elen, entry)
    return Graph(out, elen, int(entry), int(rep))


def mst_parents(Q, X, adj, entry: int):
    """MST parents of the query nodes (node id, or -1 for the root s), BFS
    order of query indices, and the total tree weight."""
    V = np.ascontiguousarray(np.concatenate([_f32(X), _f32(Q)], axis=0))
    nq, nx = Q.shape[0], X.shape[0]
    adj = np.ascontiguousarray(adj, np.int32)
    parent = np.empty(nq, np.int32)
    order = np.empty(nq, np.int32)
    w = lib().or_mst_parents(V, nx, nq, V.shape[1], adj, adj.shape[1], entry, parent, order)
    return parent, order, w


# ---------------------------------------------------------------------------
# O3: the merged-index join (Algorithms 1-8)
# ---------------------------------------------------------------------------

@dataclass
class JoinResult:
    qi: np.ndarray
    xj: np.ndarray
    dist: np.ndarray
    stats: np.ndarray  # [n][8], columns STAT_FIELDS, row i = query_ids[i]

    def pairs(self) -> set:
        return set(zip(self.qi.tolist(), self.xj.tolist()))


def join(Q, X, adj, entry: int, eps: float, metric: str = "l2", query_ids=None,
         work_sharing: str = "self", hybrid: str = "off", hybrid_beam: int = 256,
         conv_threshold: int = 10, ood_ratio: float = 1.5, parent=None,
         budget=None, uncertain: str = "plain", uncertain_rel: float = 1e-5,
         shuffle_seed: int = 0, fragile_rel: float | None = None, merged: bool = True,
         greedy_beam: int = 256, nnmap=None, qseed=None) -> JoinResult:
    """The join of Algorithm 1 on a merged graph (merged=True: adj is [N][R]
    over X then Q) or on separate indexes (merged=False: adj rows 0..nx-1
    are the data graph G_X with entry `entry`, rows nx.. the query graph
    G_Q in node ids, used only by the MST; work_sharing "none" is INLJ).
    qseed: optional [nq] per-query seed replacing the entry (the node an
    upper-layer descent reached, see descend())."""
    V = np.ascontiguousarray(np.concatenate([_f32(X), _f32(Q)], axis=0))
    nq, nx, d = Q.shape[0], X.shape[0], Q.shape[1]
    adj = np.ascontiguousarray(adj, np.int32)
    R = adj.shape[1]
    qids = np.arange(nq, dtype=np.int32) if query_ids is None else np.ascontiguousarray(query_ids, np.int32)
    n = qids.shape[0]
    if not merged and work_sharing == "self":
        raise ValueError("self mode needs the merged index (use 'none' for INLJ)")
    cfg = _Cfg(WS[work_sharing], HYB[hybrid], hybrid_beam, conv_threshold, ood_ratio,
               {"plain": 0, "out": 1, "in": 2}[uncertain], uncertain_rel, shuffle_seed,
               4.0 * d * 2.0 ** -24 if fragile_rel is None else fragile_rel, int(merged),
               greedy_beam)
    par = None
    nnw = nnd = nno = None
    if work_sharing == "nnmap":
        if merged or nnmap is None:
            raise ValueError("NN-Map joins run on separate indexes with the map from nnmap()")
        nnw = np.ascontiguousarray(nnmap.w, np.int32)
        nnd = np.ascontiguousarray(nnmap.dist, np.float64)
        nno = np.ascontiguousarray(nnmap.ood, np.uint8)
    elif work_sharing not in ("self", "none"):
        if parent is None:
            raise ValueError("work sharing needs MST parents")
        par = np.ascontiguousarray(parent, np.int32)
    bud = None
    if hybrid == "budget":
        bud = np.ascontiguousarray(budget, np.int32)
        assert bud.shape[0] == n
    qs = None
    if qseed is not None:
        qs = np.ascontiguousarray(qseed, np.int32)
        assert qs.shape[0] == nq and np.all((qs >= 0) & (qs < nx))
    stats = np.zeros((n, len(STAT_FIELDS)), np.int32)
    L = lib()
    args = (V, nx, nq, d, METRICS[metric], adj, R, entry,
            par.ctypes.data if par is not None else None, qids, n, eps, C.byref(cfg),
            bud.ctypes.data if bud is not None else None,
            nnw.ctypes.data if nnw is not None else None,
            nnd.ctypes.data if nnd is not None else None,
            nno.ctypes.data if nno is not None else None,
            qs.ctypes.data if qs is not None else None)
    e32, e64 = np.empty(0, np.int32), np.empty(0, np.float64)
    cnt = L.or_join(*args, 0, e32, e32, e64, stats)
    oq, ox, od = np.empty(cnt, np.int32), np.empty(cnt, np.int32), np.empty(cnt, np.float64)
    L.or_join(*args, cnt, oq, ox, od, stats)
    return JoinResult(oq, ox, od, stats)


@dataclass
class NNMap:
    w: np.ndarray     # [nq] int32 nearest data node of each query
    dist: np.ndarray  # [nq] float64 its distance (join metric)
    ood: np.ndarray   # [nq] uint8 OOD bit


def nnmap(Q, X, adj, metric: str = "l2", ratio: float = 1.5) -> NNMap:
    """NN-Map of Section 6: exact nearest data node of every query (fp64,
    ties to the smaller id), its distance and the OOD bit from the witness
    and its data-graph edges (adj rows 0..nx-1; see or_nnmap)."""
    V = np.ascontiguousarray(np.concatenate([_f32(X), _f32(Q)], axis=0))
    nq, nx, d = Q.shape[0], X.shape[0], Q.shape[1]
    adj = np.ascontiguousarray(adj, np.int32)
    w = np.empty(nq, np.int32)
    dist = np.empty(nq, np.float64)
    ood = np.empty(nq, np.uint8)
    lib().or_nnmap(V, nx, nq, d, METRICS[metric], adj, adj.shape[1], ratio, w, dist, ood)
    return NNMap(w, dist, ood)


def join_self_counts(Q, X, adj, entry: int, eps: float, metric: str = "l2",
                     query_ids=None) -> np.ndarray:
    """Per-query match counts of the self-mode BFS join, OpenMP over queries
    (the same steps as ``join`` in self/off mode; used for CPU timing)."""
    V = np.ascontiguousarray(np.concatenate([_f32(X), _f32(Q)], axis=0))
    nq, nx, d = Q.shape[0], X.shape[0], Q.shape[1]
    adj = np.ascontiguousarray(adj, np.int32)
    qids = np.arange(nq, dtype=np.int32) if query_ids is None else np.ascontiguousarray(query_ids, np.int32)
    out = np.empty(qids.shape[0], np.int64)
    lib().or_join_self_counts(V, nx, nq, d, METRICS[metric], adj, adj.shape[1], entry,
                              qids, qids.shape[0], eps, out)
    return out


# ---------------------------------------------------------------------------
# O5: the difficulty MLP in fp64
# ---------------------------------------------------------------------------

FEATURE_NAMES = ("eps", "dist_s", "min_dist_A", "d1", "d2", "d1_over_d2", "frac_A",
                 "frac_A_in_range")


def features(Q, X, adj, entry: int, eps: float, metric: str = "l2", query_ids=None):
    """[n][d + 8]: each query's vector and the 8 post-probe features
    (FEATURE_NAMES; see or_features)."""
    V = np.ascontiguousarray(np.concatenate([_f32(X), _f32(Q)], axis=0))
    nq, nx, d = Q.shape[0], X.shape[0], Q.shape[1]
    adj = np.ascontiguousarray(adj, np.int32)
    qids = np.arange(nq, dtype=np.int32) if query_ids is None else np.ascontiguousarray(query_ids, np.int32)
    out = np.empty((qids.shape[0], d + 8), np.float64)
    lib().or_features(V, nx, nq, d, METRICS[metric], adj, adj.shape[1], entry, qids,
                      qids.shape[0], eps, out)
    return out

def mlp_forward(params, Xin):
    W1, b1, W2, b2, W3, b3 = [np.ascontiguousarray(p, np.float64) for p in params]
    Xin = np.ascontiguousarray(Xin, np.float64)
    n, din = Xin.shape
    out = np.empty((n, W3.shape[0]), np.float64)
    lib().or_mlp_forward(n, din, W1.shape[0], W2.shape[0], W3.shape[0], Xin,
                         W1, b1, W2, b2, W3, b3, out)
    return out


def mlp_bce_backward(params, Xin, Y, mask=None):
    """(loss, [gW1, gb1, gW2, gb2, gW3, gb3]) of mean BCE-with-logits."""
    W1, b1, W2, b2, W3, b3 = [np.ascontiguousarray(p, np.float64) for p in params]
    Xin = np.ascontiguousarray(Xin, np.float64)
    Y = np.ascontiguousarray(Y, np.float64)
    n, din = Xin.shape
    m = None if mask is None else np.ascontiguousarray(mask, np.float64)
    grads = [np.empty_like(p) for p in (W1, b1, W2, b2, W3, b3)]
    loss = lib().or_mlp_bce_backward(n, din, W1.shape[0], W2.shape[0], W3.shape[0], Xin,
                                     W1, b1, W2, b2, W3, b3, Y,
                                     m.ctypes.data if m is not None else None, *grads)
    return loss, grads


def adam_step(p, g, m, v, t: int, lr: float, b1: float = 0.9, b2: float = 0.999,
              eps: float = 1e-8):
    """One fp64 Adam step (Kingma and Ba 2015, Algorithm 1) at step number t
    >= 1, in place on the float64 arrays p, m, v (g is read)."""
    for a in (p, m, v):
        assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    g = np.ascontiguousarray(g, np.float64)
    assert p.shape == g.shape == m.shape == v.shape
    lib().or_adam_step(p.size, p.reshape(-1), g.reshape(-1), m.reshape(-1), v.reshape(-1),
                       int(t), lr, b1, b2, eps)


# ---------------------------------------------------------------------------
# HNSW-style upper layers (Section 5, varying index type)
# ---------------------------------------------------------------------------

def splitmix64(seed: int, k: int) -> int:
    """Output k (k >= 1) of SplitMix64 seeded with `seed`."""
    return int(lib().or_splitmix64(seed, k))


def levels(n: int, seed: int, max_levels: int = 8) -> np.ndarray:
    """Level of each of n data nodes: trailing zero 4-bit digits of its
    SplitMix64 output, capped at max_levels (P(level >= l) = 16^-l)."""
    out = np.empty(n, np.int8)
    lib().or_levels(n, seed, max_levels, out)
    return out


@dataclass
class Layers:
    lvl: np.ndarray    # [nx] int8 level of each data node
    ids: list          # per layer (layer 1 first): sorted data ids
    adj: list          # per layer: [n_l][R] int32 data ids, -1 padded
    entry: list        # per layer: entry data id


def build_layers(X, R: int, seed: int = 1, max_levels: int = 8, Kc: int | None = None) -> Layers:
    """Upper layers over the data nodes: layer l holds the nodes of level
    >= l and its graph is the merged-graph recipe over them alone; layers
    stop before the first one with fewer than two nodes."""
    X = _f32(X)
    lvl = levels(X.shape[0], seed, max_levels)
    ids, adjs, entries = [], [], []
    for l in range(1, max_levels + 1):
        sel = np.nonzero(lvl >= l)[0].astype(np.int32)
        if sel.size < 2:
            break
        g = build_merged(np.zeros((0, X.shape[1]), np.float32), X[sel], R, Kc)
        adjs.append(np.where(g.adj >= 0, sel[np.maximum(g.adj, 0)], -1).astype(np.int32))
        ids.append(sel)
        entries.append(int(sel[g.entry]))
    return Layers(lvl, ids, adjs, entries)


def descend(Q, X, layers: Layers, metric: str = "l2", query_ids=None):
    """Greedy descent of each query through the upper layers; returns
    (seed [n] data ids, moves [n]).  No layers: the seeds are -1."""
    nq, nx, d = Q.shape[0], X.shape[0], Q.shape[1]
    qids = np.arange(nq, dtype=np.int32) if query_ids is None else np.ascontiguousarray(query_ids, np.int32)
    n = qids.shape[0]
    nl = len(layers.ids)
    if nl == 0:
        return np.full(n, -1, np.int32), np.zeros(n, np.int32)
    R = layers.adj[0].shape[1]
    off = np.zeros(nl, np.int64)
    for j in range(1, nl):
        off[j] = off[j - 1] + layers.ids[j - 1].size
    pos = np.full((nl, nx), -1, np.int32)
    for j, sel in enumerate(layers.ids):
        pos[j, sel] = np.arange(sel.size, dtype=np.int32)
    adj = np.ascontiguousarray(np.concatenate(layers.adj), np.int32)
    V = np.ascontiguousarray(np.concatenate([_f32(X), _f32(Q)], axis=0))
    seed = np.empty(n, np.int32)
    moves = np.empty(n, np.int32)
    lib().or_descend(V, nx, nq, d, METRICS[metric], nl, off, np.ascontiguousarray(pos), adj, R,
                     np.asarray(layers.entry, np.int32), qids, n, seed, moves)
    return seed, moves
