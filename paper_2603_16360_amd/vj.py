"""ctypes binding of libvj (include/vj.h): argument marshalling only.

Every function here calls the C ABI of the same name; all computation runs
in the library's HIP kernels.  PyTorch provides device memory and streams.
If libvj.so is missing the import fails loudly: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvj.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with "
                      "`python -c 'import __graft_entry__ as g; g.build()'`")

_lib = C.CDLL(LIB_PATH)

VJ_OK = 0
STATUS = {0: "VJ_OK", 1: "VJ_ERR_INVALID_ARG", 2: "VJ_ERR_METRIC_MISMATCH", 3: "VJ_ERR_OOM",
          4: "VJ_ERR_HIP", 5: "VJ_ERR_INTERNAL", 6: "VJ_ERR_UNSUPPORTED", 7: "VJ_ERR_IO"}
METRIC = {"l2": 0, "ip": 1}
WORK_SHARING = {"self": 0, "none": 0, "soft": 1, "hard": 2,  # "none": no sharing (INLJ)
                "nnmap": 3}
HYBRID = {"off": 0, "force": 1, "adapt": 2, "budget": 3, "learned": 4}
PRECISION = {"fp32": 0, "bf16": 1, "fp8": 2, "u8": 3, "auto": 4}
STAT_FIELDS = ("pairs", "n_dist", "n_expanded", "h_pops", "ood", "hybrid",
               "visited_data", "flags")


class VJError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class vj_build_params(C.Structure):
    _fields_ = [("R", C.c_int32), ("K_cand", C.c_int32), ("build_mst", C.c_int32),
                ("copies", C.c_int32)]


class vj_join_params(C.Structure):
    _fields_ = [("work_sharing", C.c_int32), ("hybrid", C.c_int32),
                ("hybrid_beam", C.c_int32), ("conv_threshold", C.c_int32),
                ("ood_ratio", C.c_float), ("precision", C.c_int32),
                ("budget", C.c_void_p), ("start_tier", C.c_int32),
                ("coop_tables", C.c_int32), ("pair_capacity", C.c_int64),
                ("dense_first", C.c_int32), ("greedy_beam", C.c_int32),
                ("persistent", C.c_int32), ("layer_seeds", C.c_int32)]


_vp, _i64, _i32, _f32 = C.c_void_p, C.c_int64, C.c_int32, C.c_float
_PP = C.POINTER(C.c_void_p)

_SIGS = {
    "vj_default_build_params": (None, [C.POINTER(vj_build_params)]),
    "vj_default_join_params": (None, [C.POINTER(vj_join_params)]),
    "vj_build_merged_index": (C.c_int, [_vp, _i64, _vp, _i64, _i32, C.c_int,
                                        C.POINTER(vj_build_params), _vp, _PP]),
    "vj_index_from_graph": (C.c_int, [_vp, _i64, _vp, _i64, _i32, C.c_int, _vp, _i32, _i32,
                                      _vp, _vp, _PP]),
    "vj_build_separate_index": (C.c_int, [_vp, _i64, _vp, _i64, _i32, C.c_int,
                                          C.POINTER(vj_build_params), _vp, _PP]),
    "vj_index_from_separate_graphs": (C.c_int, [_vp, _i64, _vp, _i64, _i32, C.c_int, _vp, _i32,
                                                _i32, _vp, _vp, _PP]),
    "vj_index_swap_roles": (C.c_int, [_vp, _i32, _vp, _PP]),
    "vj_index_insert_queries": (C.c_int, [_vp, _vp, _i64, _i32, _vp]),
    "vj_build_nnmap": (C.c_int, [_vp, _f32, _vp]),
    "vj_index_export_nnmap": (C.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "vj_index_export_graph": (C.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "vj_index_info": (C.c_int, [_vp] + [_vp] * 6),
    "vj_index_build_stats": (C.c_int, [_vp] + [_vp] * 5),
    "vj_index_free": (None, [_vp]),
    "vj_index_save": (C.c_int, [_vp, C.c_char_p]),
    "vj_index_load": (C.c_int, [C.c_char_p, _vp, _PP]),
    "vj_predictor_save": (C.c_int, [_vp, C.c_char_p]),
    "vj_predictor_load": (C.c_int, [C.c_char_p, _vp, _PP]),
    "vj_predictor_info": (C.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "vj_join": (C.c_int, [_vp, _vp, _i64, _f32, C.c_int, C.POINTER(vj_join_params), _vp, _PP]),
    "vj_bruteforce_join": (C.c_int, [_vp, _i64, _vp, _i64, _i32, _f32, C.c_int, C.c_int,
                                     _vp, _PP]),
    "vj_bruteforce_join_noalloc": (C.c_int, [_vp, _i64, _vp, _i64, _i32, _f32, C.c_int, C.c_int,
                                             _vp, _vp, _i64, C.POINTER(_i64), _vp]),
    "vj_pairs_count": (_i64, [_vp]),
    "vj_pairs_export": (C.c_int, [_vp, _vp, _vp, C.c_int, _vp]),
    "vj_pairs_stats": (C.c_int, [_vp, _vp, _vp]),
    "vj_pairs_timing": (C.c_int, [_vp, _vp, _vp, _vp]),
    "vj_pairs_tiers": (C.c_int, [_vp, _vp, _vp, _vp]),
    "vj_pairs_rechecked": (C.c_int, [_vp, _vp]),
    "vj_pairs_free": (None, [_vp]),
    "vj_join_features": (C.c_int, [_vp, _vp, _i64, _f32, C.c_int, _vp, _vp]),
    "vj_join_batches": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _i32, C.c_int, C.POINTER(vj_join_params),
                                  _vp, _vp, _vp]),
    "vj_join_batches_device": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _i32, C.c_int,
                                         C.POINTER(vj_join_params), C.c_int, _vp, _vp, _vp]),
    "vj_autotune_join": (C.c_int, [_vp, _vp, _i64, _f32, C.c_int, C.POINTER(vj_join_params),
                                   _vp, _vp]),
    "vj_predictor_create": (C.c_int, [_i32, _i32, _i32, _i32, C.c_uint64, _vp, _PP]),
    "vj_predictor_free": (None, [_vp]),
    "vj_predictor_set_params": (C.c_int, [_vp] + [_vp] * 8 + [_vp]),
    "vj_predictor_get_params": (C.c_int, [_vp] + [_vp] * 8 + [_vp]),
    "vj_predictor_fit_normalization": (C.c_int, [_vp, _vp, _i64, _vp]),
    "vj_predictor_forward": (C.c_int, [_vp, _vp, _i64, _vp, _vp]),
    "vj_predictor_loss_grad": (C.c_int, [_vp, _vp, _vp, _vp, _i64, C.POINTER(C.c_double)]
                               + [_vp] * 6 + [_vp]),
    "vj_predictor_train": (C.c_int, [_vp, _vp, _vp, _i64, _i32, _i32, _f32, C.c_uint64, _vp, _vp]),
    "vj_predictor_adam_step": (C.c_int, [_vp, _vp, _f32, _vp]),
    "vj_predictor_get_adam_state": (C.c_int, [_vp, _vp, _vp, C.POINTER(_i64), _vp]),
    "vj_index_attach_predictor": (C.c_int, [_vp, _vp, _f32, _vp]),
    "vj_last_error": (C.c_char_p, []),
    "vj_trim_memory": (C.c_int, [C.POINTER(_i64)]),
    "vj_calib_gather": (C.c_int, [_vp, _i64, _i32, _vp, _i64, _vp, _vp]),
    "vj_index_build_layers": (C.c_int, [_vp, _i32, C.c_uint64, _i32, _vp]),
    "vj_index_layers_info": (C.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "vj_index_export_layer": (C.c_int, [_vp, _i32, _vp, _vp, _vp]),
    "vj_index_descend": (C.c_int, [_vp, _vp, _i64, _vp, _vp, _vp]),
}
for _name, (_res, _args) in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args

EXPORTED = tuple(_SIGS)


def _check(status: int):
    if status != VJ_OK:
        raise VJError(status, _lib.vj_last_error().decode())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t: torch.Tensor, dtype, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    return t.contiguous()


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else C.c_void_p(0)


# ------------------------------------------------------------------ objects --

class Pairs:
    """A join result held by the library (vj_pairs)."""

    def __init__(self, handle: int, n_queries: int):
        self._h = C.c_void_p(handle)
        self.n_queries = n_queries

    def __del__(self):
        if getattr(self, "_h", None) and self._h.value and _lib is not None:
            _lib.vj_pairs_free(self._h)
            self._h = C.c_void_p(0)

    def count(self) -> int:
        return int(_lib.vj_pairs_count(self._h))

    def export(self, sorted: bool = True):
        """(qx int32 [count, 2], dist float32 [count]) as CUDA tensors."""
        n = self.count()
        qx = torch.empty((n, 2), dtype=torch.int32, device="cuda")
        dist = torch.empty(n, dtype=torch.float32, device="cuda")
        _check(_lib.vj_pairs_export(self._h, _ptr(qx), _ptr(dist), int(sorted), _stream()))
        return qx, dist

    def timing(self) -> dict:
        """Device time of the traversal launches (HIP events on the stream)."""
        k, sp, ns = C.c_float(), C.c_float(), C.c_int64()
        _check(_lib.vj_pairs_timing(self._h, C.byref(k), C.byref(sp), C.byref(ns)))
        return {"kernel_ms": k.value, "spill_ms": sp.value, "n_spilled": ns.value}

    def rechecked(self) -> int:
        """Candidates re-decided at full precision (see vj_pairs_rechecked)."""
        n = C.c_int64()
        _check(_lib.vj_pairs_rechecked(self._h, C.byref(n)))
        return n.value

    def tiers(self) -> list:
        """Per storage tier 0..3: device ms, launches, queries launched."""
        ms, ln, nq = (C.c_float * 4)(), (C.c_int32 * 4)(), (C.c_int64 * 4)()
        _check(_lib.vj_pairs_tiers(self._h, ms, ln, nq))
        return [{"ms": ms[t], "launches": ln[t], "queries": nq[t]} for t in range(4)]

    def stats(self) -> torch.Tensor:
        """Per-query counters [n, 8] int32 (columns STAT_FIELDS)."""
        st = torch.empty((self.n_queries, 8), dtype=torch.int32, device="cuda")
        if self.n_queries:
            _check(_lib.vj_pairs_stats(self._h, _ptr(st), _stream()))
        return st


class Index:
    """A merged index (vj_index) over Q (queries) and X (data)."""

    def __init__(self, handle: int):
        self._h = C.c_void_p(handle)

    def __del__(self):
        if getattr(self, "_h", None) and self._h.value and _lib is not None:
            _lib.vj_index_free(self._h)
            self._h = C.c_void_p(0)

    def info(self) -> dict:
        nq, nx = C.c_int64(), C.c_int64()
        d, R, e, m = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        _check(_lib.vj_index_info(self._h, C.byref(nq), C.byref(nx), C.byref(d), C.byref(R),
                                  C.byref(e), C.byref(m)))
        return {"nq": nq.value, "nx": nx.value, "d": d.value, "R": R.value,
                "entry": e.value, "metric": m.value}

    def build_stats(self) -> dict:
        """Work counters of the last build or insertion (vj_index_build_stats)."""
        v = [C.c_int64() for _ in range(5)]
        _check(_lib.vj_index_build_stats(self._h, *[C.byref(x) for x in v]))
        return dict(zip(("tiles_first", "tiles_second", "tiles_all", "repairs",
                         "repairs_listed"), (x.value for x in v)))

    def export_graph(self, with_parent: bool = True):
        """(adj int32 [N, R], elen float32 [N, R], parent int32 [nq] or None
        without an MST) on the GPU."""
        i = self.info()
        N = i["nq"] + i["nx"]
        adj = torch.empty((N, i["R"]), dtype=torch.int32, device="cuda")
        elen = torch.empty((N, i["R"]), dtype=torch.float32, device="cuda")
        parent = torch.empty(i["nq"], dtype=torch.int32, device="cuda")
        _check(_lib.vj_index_export_graph(self._h, _ptr(adj), _ptr(elen),
                                          _ptr(parent) if with_parent else None, _stream()))
        return adj, elen, parent if with_parent else None

    def swap_roles(self, build_mst: bool = False) -> "Index":
        """The role-switched merged index (vj_index_swap_roles): joins on it
        return (old data index, old query index) pairs."""
        h = C.c_void_p()
        _check(_lib.vj_index_swap_roles(self._h, int(build_mst), _stream(), C.byref(h)))
        return Index(h.value)

    def insert_queries(self, Q: torch.Tensor, K_cand: int = 0):
        """Append the query batch Q [n, d] (vj_index_insert_queries); the new
        queries get the next query indexes."""
        Q = _dev(Q, torch.float32, "Q")
        _check(_lib.vj_index_insert_queries(self._h, _ptr(Q), Q.shape[0], int(K_cand), _stream()))

    def build_nnmap(self, ood_ratio: float = 1.5):
        """NN-Map of the queries (vj_build_nnmap; separate indexes)."""
        _check(_lib.vj_build_nnmap(self._h, float(ood_ratio), _stream()))

    def export_nnmap(self):
        """(w int32 [nq], dist float64 [nq], ood uint8 [nq]) on the GPU."""
        nq = self.info()["nq"]
        w = torch.empty(nq, dtype=torch.int32, device="cuda")
        dist = torch.empty(nq, dtype=torch.float64, device="cuda")
        ood = torch.empty(nq, dtype=torch.uint8, device="cuda")
        _check(_lib.vj_index_export_nnmap(self._h, _ptr(w), _ptr(dist), _ptr(ood), _stream()))
        return w, dist, ood

    def save(self, path: str):
        """Write the index to a file (vj_index_save)."""
        _check(_lib.vj_index_save(self._h, os.fsencode(path)))


def vj_index_load(path: str) -> Index:
    """Read an index file written by Index.save (vj_index_load)."""
    h = C.c_void_p()
    _check(_lib.vj_index_load(os.fsencode(path), _stream(), C.byref(h)))
    return Index(h.value)


# ---------------------------------------------------------------- functions --

def join_params(work_sharing="self", hybrid="off", hybrid_beam=256, conv_threshold=10,
                ood_ratio=1.5, precision="fp32", budget=None, start_tier=1, coop_tables=0,
                pair_capacity=0, dense_first=1, greedy_beam=256, persistent=0, layer_seeds=0):
    p = vj_join_params()
    _lib.vj_default_join_params(C.byref(p))
    p.work_sharing = WORK_SHARING[work_sharing]
    p.hybrid = HYBRID[hybrid]
    p.hybrid_beam = hybrid_beam
    p.conv_threshold = conv_threshold
    p.ood_ratio = ood_ratio
    p.precision = PRECISION[precision]
    p.budget = budget.data_ptr() if budget is not None else None
    p.start_tier = start_tier
    p.coop_tables = coop_tables
    p.pair_capacity = pair_capacity
    p.dense_first = dense_first
    p.greedy_beam = greedy_beam
    p.persistent = persistent
    p.layer_seeds = layer_seeds
    return p


def vj_build_merged_index(Q: torch.Tensor, X: torch.Tensor, metric: str = "l2", R: int = 32,
                          K_cand: int = 0, build_mst: bool = True, copies: int = 0) -> Index:
    Q = _dev(Q, torch.float32, "Q")
    X = _dev(X, torch.float32, "X")
    bp = vj_build_params()
    _lib.vj_default_build_params(C.byref(bp))
    bp.R, bp.K_cand, bp.build_mst, bp.copies = R, K_cand, int(build_mst), copies
    h = C.c_void_p()
    _check(_lib.vj_build_merged_index(_ptr(Q), Q.shape[0], _ptr(X), X.shape[0], X.shape[1],
                                      METRIC[metric], C.byref(bp), _stream(), C.byref(h)))
    return Index(h.value)


def vj_build_separate_index(Q: torch.Tensor, X: torch.Tensor, metric: str = "l2", R: int = 32,
                            K_cand: int = 0, build_mst: bool = True, copies: int = 0) -> Index:
    """Separate indexes G_X and G_Q (cfg.merged = false)."""
    Q = _dev(Q, torch.float32, "Q")
    X = _dev(X, torch.float32, "X")
    bp = vj_build_params()
    _lib.vj_default_build_params(C.byref(bp))
    bp.R, bp.K_cand, bp.build_mst, bp.copies = R, K_cand, int(build_mst), copies
    h = C.c_void_p()
    _check(_lib.vj_build_separate_index(_ptr(Q), Q.shape[0], _ptr(X), X.shape[0], X.shape[1],
                                        METRIC[metric], C.byref(bp), _stream(), C.byref(h)))
    return Index(h.value)


def vj_index_from_separate_graphs(Q: torch.Tensor, X: torch.Tensor, adj: torch.Tensor,
                                  entry: int, metric: str = "l2",
                                  parent: torch.Tensor | None = None) -> Index:
    Q = _dev(Q, torch.float32, "Q")
    X = _dev(X, torch.float32, "X")
    adj = _dev(adj, torch.int32, "adj")
    if parent is not None:
        parent = _dev(parent, torch.int32, "parent")
    h = C.c_void_p()
    _check(_lib.vj_index_from_separate_graphs(_ptr(Q), Q.shape[0], _ptr(X), X.shape[0], X.shape[1],
                                              METRIC[metric], _ptr(adj), adj.shape[1], entry,
                                              _ptr(parent) if parent is not None else C.c_void_p(0),
                                              _stream(), C.byref(h)))
    return Index(h.value)


def vj_index_from_graph(Q: torch.Tensor, X: torch.Tensor, adj: torch.Tensor, entry: int,
                        metric: str = "l2", parent: torch.Tensor | None = None) -> Index:
    Q = _dev(Q, torch.float32, "Q")
    X = _dev(X, torch.float32, "X")
    adj = _dev(adj, torch.int32, "adj")
    if parent is not None:
        parent = _dev(parent, torch.int32, "parent")
    h = C.c_void_p()
    _check(_lib.vj_index_from_graph(_ptr(Q), Q.shape[0], _ptr(X), X.shape[0], X.shape[1],
                                    METRIC[metric], _ptr(adj), adj.shape[1], entry,
                                    _ptr(parent) if parent is not None else C.c_void_p(0),
                                    _stream(), C.byref(h)))
    return Index(h.value)


def vj_join(index: Index, eps: float, metric: str = "l2", query_ids: torch.Tensor | None = None,
            params: vj_join_params | None = None, **kw) -> Pairs:
    if params is None:
        params = join_params(**kw)
    n = index.info()["nq"] if query_ids is None else int(query_ids.numel())
    qp = C.c_void_p(0)
    if query_ids is not None:
        query_ids = _dev(query_ids, torch.int32, "query_ids")
        qp = _ptr(query_ids)
    h = C.c_void_p()
    _check(_lib.vj_join(index._h, qp, n, float(eps), METRIC[metric], C.byref(params),
                        _stream(), C.byref(h)))
    return Pairs(h.value, n)


def vj_bruteforce_join(Q: torch.Tensor, X: torch.Tensor, eps: float, metric: str = "l2",
                       precision: str = "fp32") -> Pairs:
    Q = _dev(Q, torch.float32, "Q")
    X = _dev(X, torch.float32, "X")
    h = C.c_void_p()
    _check(_lib.vj_bruteforce_join(_ptr(Q), Q.shape[0], _ptr(X), X.shape[0], X.shape[1],
                                   float(eps), METRIC[metric], PRECISION[precision],
                                   _stream(), C.byref(h)))
    return Pairs(h.value, 0)


def vj_bruteforce_join_noalloc(Q: torch.Tensor, X: torch.Tensor, eps: float, qx: torch.Tensor,
                               dist: torch.Tensor | None = None, metric: str = "l2",
                               precision: str = "fp32") -> int:
    """vj_bruteforce_join into the caller's qx [cap, 2] int32 and dist [cap]
    float32 (may be None) with no device allocation by the library; returns
    the pair count (if above cap, only cap pairs were written)."""
    Q = _dev(Q, torch.float32, "Q")
    X = _dev(X, torch.float32, "X")
    if not (qx.is_cuda and qx.dtype == torch.int32 and qx.dim() == 2 and qx.shape[1] == 2
            and qx.is_contiguous()):
        raise TypeError("qx must be a contiguous CUDA int32 tensor of shape [cap, 2]")
    cap = qx.shape[0]
    if dist is not None and not (dist.is_cuda and dist.dtype == torch.float32
                                 and dist.is_contiguous() and dist.numel() >= cap):
        raise TypeError("dist must be a contiguous CUDA float32 tensor of at least cap values")
    cnt = C.c_int64()
    _check(_lib.vj_bruteforce_join_noalloc(_ptr(Q), Q.shape[0], _ptr(X), X.shape[0], X.shape[1],
                                           float(eps), METRIC[metric], PRECISION[precision],
                                           _ptr(qx), _ptr(dist) if dist is not None else None,
                                           cap, C.byref(cnt), _stream()))
    return cnt.value


def vj_join_batches(index: Index, starts, counts, eps_list, metric: str = "l2",
                    query_ids: torch.Tensor | None = None, params: vj_join_params | None = None,
                    runner: str = "host", **kw):
    """Run the batches back to back; returns (list of Pairs, ms per batch).

    runner="host": vj_join_batches, one vj_join per batch, wall ms per batch.
    runner="device" / "graph": vj_join_batches_device (self mode, no host
    synchronisation between batches) with direct launches / HIP graph
    replay, device ms per batch."""
    if params is None:
        params = join_params(**kw)
    if runner not in ("host", "device", "graph"):
        raise ValueError(f"runner must be host, device or graph, not {runner!r}")
    nb = len(starts)
    st = (C.c_int64 * nb)(*[int(v) for v in starts])
    ct = (C.c_int64 * nb)(*[int(v) for v in counts])
    ep = (C.c_float * nb)(*[float(v) for v in eps_list])
    out = (C.c_void_p * nb)()
    ms = (C.c_float * nb)()
    qp = C.c_void_p(0)
    if query_ids is not None:
        query_ids = _dev(query_ids, torch.int32, "query_ids")
        qp = _ptr(query_ids)
    if runner == "host":
        _check(_lib.vj_join_batches(index._h, qp, st, ct, ep, nb, METRIC[metric], C.byref(params),
                                    _stream(), out, ms))
    else:
        _check(_lib.vj_join_batches_device(index._h, qp, st, ct, ep, nb, METRIC[metric],
                                           C.byref(params), int(runner == "graph"), _stream(), out,
                                           ms))
    return [Pairs(out[b], int(counts[b])) for b in range(nb)], list(ms)


def vj_autotune_join(index: Index, eps: float, metric: str = "l2",
                     query_ids: torch.Tensor | None = None, params: vj_join_params | None = None,
                     **kw):
    """(tuned vj_join_params, best device ms) on the given sample."""
    if params is None:
        params = join_params(**kw)
    n = index.info()["nq"] if query_ids is None else int(query_ids.numel())
    qp = C.c_void_p(0)
    if query_ids is not None:
        query_ids = _dev(query_ids, torch.int32, "query_ids")
        qp = _ptr(query_ids)
    best = C.c_float()
    _check(_lib.vj_autotune_join(index._h, qp, n, float(eps), METRIC[metric], C.byref(params),
                                 C.byref(best), _stream()))
    return params, best.value


def vj_join_features(index: Index, eps: float, metric: str = "l2",
                     query_ids: torch.Tensor | None = None) -> torch.Tensor:
    """[n][d + 8] float32 post-probe features (see vj_join_features)."""
    info = index.info()
    n = info["nq"] if query_ids is None else int(query_ids.numel())
    out = torch.empty((n, info["d"] + 8), dtype=torch.float32, device="cuda")
    qp = C.c_void_p(0)
    if query_ids is not None:
        query_ids = _dev(query_ids, torch.int32, "query_ids")
        qp = _ptr(query_ids)
    _check(_lib.vj_join_features(index._h, qp, n, float(eps), METRIC[metric], _ptr(out), _stream()))
    return out


class Predictor:
    """The difficulty MLP (vj_predictor): din -> h1 -> h2 -> k."""

    def __init__(self, din: int, h1: int = 256, h2: int = 256, k: int = 4, seed: int = 0):
        h = C.c_void_p()
        _check(_lib.vj_predictor_create(din, h1, h2, k, seed, _stream(), C.byref(h)))
        self._h = h
        self.shapes = {"W1": (h1, din), "b1": (h1,), "W2": (h2, h1), "b2": (h2,),
                       "W3": (k, h2), "b3": (k,), "mu": (din,), "inv_sigma": (din,)}
        self.din, self.k = din, k

    def __del__(self):
        if getattr(self, "_h", None) and self._h.value and _lib is not None:
            _lib.vj_predictor_free(self._h)
            self._h = C.c_void_p(0)

    NAMES = ("W1", "b1", "W2", "b2", "W3", "b3", "mu", "inv_sigma")

    def get_params(self) -> dict:
        out = {k: torch.empty(v, dtype=torch.float32, device="cuda") for k, v in self.shapes.items()}
        _check(_lib.vj_predictor_get_params(self._h, *[_ptr(out[k]) for k in self.NAMES], _stream()))
        return out

    def set_params(self, **kw):
        ts = {k: _dev(v, torch.float32, k) for k, v in kw.items()}
        for k, v in ts.items():
            if tuple(v.shape) != self.shapes[k]:
                raise ValueError(f"{k} must have shape {self.shapes[k]}")
        _check(_lib.vj_predictor_set_params(self._h, *[_ptr(ts[k]) if k in ts else C.c_void_p(0)
                                                       for k in self.NAMES], _stream()))

    def fit_normalization(self, X: torch.Tensor):
        X = _dev(X, torch.float32, "X")
        _check(_lib.vj_predictor_fit_normalization(self._h, _ptr(X), X.shape[0], _stream()))

    def forward(self, X: torch.Tensor) -> torch.Tensor:
        X = _dev(X, torch.float32, "X")
        out = torch.empty((X.shape[0], self.k), dtype=torch.float32, device="cuda")
        _check(_lib.vj_predictor_forward(self._h, _ptr(X), X.shape[0], _ptr(out), _stream()))
        return out

    def loss_grad(self, X: torch.Tensor, Y: torch.Tensor, mask: torch.Tensor | None = None):
        X = _dev(X, torch.float32, "X")
        Y = _dev(Y, torch.float32, "Y")
        m = _dev(mask, torch.float32, "mask") if mask is not None else None
        g = {k: torch.empty(self.shapes[k], dtype=torch.float32, device="cuda")
             for k in ("W1", "b1", "W2", "b2", "W3", "b3")}
        loss = C.c_double()
        _check(_lib.vj_predictor_loss_grad(self._h, _ptr(X), _ptr(Y), _ptr(m), X.shape[0],
                                           C.byref(loss), *[_ptr(g[k]) for k in g], _stream()))
        return loss.value, g

    def train(self, X: torch.Tensor, Y: torch.Tensor, epochs: int = 10, batch: int = 1024,
              lr: float = 1e-3, seed: int = 0):
        X = _dev(X, torch.float32, "X")
        Y = _dev(Y, torch.float32, "Y")
        losses = (C.c_float * max(1, epochs))()
        _check(_lib.vj_predictor_train(self._h, _ptr(X), _ptr(Y), X.shape[0], epochs, batch,
                                       float(lr), seed, losses, _stream()))
        return list(losses)[:epochs]

    PARAMS = ("W1", "b1", "W2", "b2", "W3", "b3")

    def save(self, path: str):
        """Write parameters, normalisation and optimizer state (vj_predictor_save)."""
        _check(_lib.vj_predictor_save(self._h, os.fsencode(path)))

    @classmethod
    def load(cls, path: str) -> "Predictor":
        """Read a predictor file (vj_predictor_load)."""
        h = C.c_void_p()
        _check(_lib.vj_predictor_load(os.fsencode(path), _stream(), C.byref(h)))
        p = cls.__new__(cls)
        p._h = h
        p._read_shapes()
        return p

    def _read_shapes(self):
        din, h1, h2, k = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        _check(_lib.vj_predictor_info(self._h, C.byref(din), C.byref(h1), C.byref(h2), C.byref(k)))
        din, h1, h2, k = din.value, h1.value, h2.value, k.value
        self.shapes = {"W1": (h1, din), "b1": (h1,), "W2": (h2, h1), "b2": (h2,),
                       "W3": (k, h2), "b3": (k,), "mu": (din,), "inv_sigma": (din,)}
        self.din, self.k = din, k

    @property
    def n_params(self) -> int:
        return sum(int(np.prod(self.shapes[k])) for k in self.PARAMS)

    def adam_step(self, grad: torch.Tensor, lr: float = 1e-3):
        """One Adam step with the caller's gradient: every parameter back to
        back (order W1 b1 W2 b2 W3 b3), n_params floats."""
        g = _dev(grad, torch.float32, "grad").reshape(-1)
        if g.numel() != self.n_params:
            raise ValueError(f"grad must hold {self.n_params} floats")
        _check(_lib.vj_predictor_adam_step(self._h, _ptr(g), float(lr), _stream()))

    def adam_state(self):
        """(m, v, steps): the optimizer's moments (flat, layout of adam_step)
        and its step count."""
        m = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        v = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        t = C.c_int64()
        _check(_lib.vj_predictor_get_adam_state(self._h, _ptr(m), _ptr(v), C.byref(t), _stream()))
        return m, v, t.value


def vj_index_attach_predictor(index: Index, pred: Predictor | None, recall_target: float = 0.95,
                              budgets=(0, 16, 64, 256)):
    b = (C.c_int32 * len(budgets))(*budgets)
    _check(_lib.vj_index_attach_predictor(index._h, pred._h if pred is not None else None,
                                          float(recall_target), b))
    index._pred = pred  # keep the predictor alive while attached


def vj_last_error() -> str:
    return _lib.vj_last_error().decode()


def vj_trim_memory() -> int:
    """Return the library's kept device blocks of the current device to the
    runtime (see include/vj.h); the bytes returned."""
    n = _i64(0)
    _check(_lib.vj_trim_memory(C.byref(n)))
    return n.value


def vj_index_build_layers(index: Index, R: int = 16, seed: int = 1, max_levels: int = 8):
    """HNSW-style upper layers over the data nodes (see include/vj.h)."""
    _check(_lib.vj_index_build_layers(index._h, R, seed, max_levels, _stream()))


def vj_index_layers(index: Index):
    """[(data ids, adjacency [n][R], entry)] of each upper layer, layer 1 first."""
    nl, R = C.c_int32(), C.c_int32()
    _check(_lib.vj_index_layers_info(index._h, C.byref(nl), C.byref(R), None, None))
    counts = (C.c_int64 * max(1, nl.value))()
    entries = (C.c_int32 * max(1, nl.value))()
    _check(_lib.vj_index_layers_info(index._h, C.byref(nl), C.byref(R), counts, entries))
    out = []
    for j in range(nl.value):
        ids = torch.empty(counts[j], dtype=torch.int32, device="cuda")
        adj = torch.empty((counts[j], R.value), dtype=torch.int32, device="cuda")
        _check(_lib.vj_index_export_layer(index._h, j + 1, _ptr(ids), _ptr(adj), _stream()))
        out.append((ids, adj, entries[j]))
    return out


def vj_index_descend(index: Index, query_ids: torch.Tensor | None = None):
    """(seed, moves) of each listed query's descent through the upper layers."""
    n = index.info()["nq"] if query_ids is None else int(query_ids.numel())
    qp = C.c_void_p(0)
    if query_ids is not None:
        query_ids = _dev(query_ids, torch.int32, "query_ids")
        qp = _ptr(query_ids)
    seed = torch.empty(n, dtype=torch.int32, device="cuda")
    moves = torch.empty(n, dtype=torch.int32, device="cuda")
    _check(_lib.vj_index_descend(index._h, qp, n, _ptr(seed), _ptr(moves), _stream()))
    return seed, moves


def vj_calib_gather(rows: torch.Tensor, ids: torch.Tensor) -> torch.Tensor:
    """Counter calibration: the sum of each listed row, read with the join's
    row-read layout (see include/vj.h)."""
    rows = _dev(rows, torch.float32, "rows")
    ids = _dev(ids, torch.int32, "ids")
    out = torch.empty(ids.numel(), dtype=torch.float32, device=rows.device)
    _check(_lib.vj_calib_gather(_ptr(rows), rows.shape[0], rows.shape[1], _ptr(ids), ids.numel(),
                                _ptr(out), _stream()))
    return out
