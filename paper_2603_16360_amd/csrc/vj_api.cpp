// C ABI of libvj: argument checks, index objects, the join driver and the
// result objects.  Every entry point converts internal errors to vj_status.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <numeric>
#include <vector>

#include "build.h"
#include "predictor.h"
#include "tiles.h"
#include "util.h"
#include "vj_internal.h"

struct vj_index { vj::Index impl; };
struct vj_pairs { vj::Pairs impl; };
struct vj_predictor { vj::Predictor impl; };

namespace vj {

static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }
const char *last_error() { return g_err.c_str(); }

int padded_dim(int d) {
    static const int dims[] = {32, 64, 96, 128, 192, 256, 384, 512, 768, 1024};
    for (int x : dims)
        if (d <= x) return x;
    return -1;
}

static int ceil_log2(int64_t v) {
    int l = 0;
    while ((int64_t(1) << l) < v) ++l;
    return l;
}

// ----------------------------------------------------------------- index --

// exact low-precision copies of the padded rows in ix.vec, join state
static void finish_vectors(Index &ix, hipStream_t s) {
    DevBuf flag(sizeof(int32_t));
    VJ_HIP(hipMemsetAsync(flag.p, 0, sizeof(int32_t), s));
    ix.vec_u8.alloc((size_t)ix.N * ix.dp);
    launch_quantize(ix.vec.as<float>(), ix.N, ix.dp, ix.vec_u8.as<uint8_t>(), nullptr,
                    flag.as<int32_t>(), s);
    int32_t h = 0;
    VJ_HIP(hipMemcpyAsync(&h, flag.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    VJ_HIP(hipStreamSynchronize(s));
    ix.integer_u8 = (h & 1) == 0;
    if (!ix.integer_u8) ix.vec_u8.release();
    const size_t nq = (size_t)std::max<int64_t>(ix.nq, 1);
    ix.cache.alloc(nq * sizeof(int32_t));
    ix.inb.alloc(nq * sizeof(int32_t));
    ix.seg.alloc(nq * sizeof(int64_t));
    ix.segn.alloc(nq * sizeof(int32_t));
    ix.done.alloc(nq * sizeof(int32_t));
    VJ_HIP(hipMemsetAsync(ix.done.p, 0, ix.done.bytes, s));
    VJ_HIP(hipMemsetAsync(ix.cache.p, 0xff, ix.cache.bytes, s));
    VJ_HIP(hipMemsetAsync(ix.inb.p, 0, ix.inb.bytes, s));
    VJ_HIP(hipMemsetAsync(ix.seg.p, 0, ix.seg.bytes, s));
    VJ_HIP(hipMemsetAsync(ix.segn.p, 0, ix.segn.bytes, s));
}

// copy + pad the vectors, exact low-precision copies, join state
static void init_vectors(Index &ix, const float *Q, const float *X, hipStream_t s) {
    ix.vec.alloc((size_t)ix.N * ix.dp * sizeof(float));
    launch_pad_rows(X, ix.nx, ix.d, ix.vec.as<float>(), ix.dp, s);
    launch_pad_rows(Q, ix.nq, ix.d, ix.vec.as<float>() + (size_t)ix.nx * ix.dp, ix.dp, s);
    finish_vectors(ix, s);
}

void ensure_bf16(Index &ix, hipStream_t s) {
    if (ix.vec_bf16.p) return;
    ix.vec_bf16.alloc((size_t)ix.N * ix.dp * sizeof(uint16_t));
    DevBuf flag(sizeof(int32_t));
    VJ_HIP(hipMemsetAsync(flag.p, 0, sizeof(int32_t), s));
    launch_quantize(ix.vec.as<float>(), ix.N, ix.dp, nullptr, ix.vec_bf16.as<uint16_t>(),
                    flag.as<int32_t>(), s);
    int32_t h = 0;
    VJ_HIP(hipMemcpyAsync(&h, flag.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    VJ_HIP(hipStreamSynchronize(s));
    ix.bf16_exact = (h & 2) == 0;
}

void ensure_f8(Index &ix, hipStream_t s) {
    if (ix.vec_f8.p) return;
    ix.vec_f8.alloc((size_t)ix.N * ix.dp);
    ix.f8meta.alloc((size_t)ix.N * sizeof(float2));
    launch_quantize_f8(ix.vec.as<float>(), ix.N, ix.dp, ix.vec_f8.as<uint8_t>(),
                       ix.f8meta.as<float2>(), s);
    VJ_HIP(hipStreamSynchronize(s));
}

// MST over the query nodes plus (s, q) edges, rooted at s (Section 3.2);
// Kruskal with ties on (w, min id, max id); weights are fp32 L2 lengths.
void compute_mst(Index &ix, hipStream_t s) {
    const int64_t nq = ix.nq, nx = ix.nx;
    const int R = ix.R;
    std::vector<int32_t> adjq((size_t)nq * R);
    std::vector<float> elq((size_t)nq * R), ds((size_t)nq);
    if (nq > 0) {
        VJ_HIP(hipMemcpyAsync(adjq.data(), ix.adj.as<int32_t>() + (size_t)nx * R,
                              adjq.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        VJ_HIP(hipMemcpyAsync(elq.data(), ix.elen.as<float>() + (size_t)nx * R,
                              elq.size() * sizeof(float), hipMemcpyDeviceToHost, s));
        DevBuf dd((size_t)nq * sizeof(float));
        launch_dist_to_node(ix.vec.as<float>(), ix.dp, nx, nq, ix.entry, dd.as<float>(), s);
        VJ_HIP(hipMemcpyAsync(ds.data(), dd.p, ds.size() * sizeof(float), hipMemcpyDeviceToHost, s));
        VJ_HIP(hipStreamSynchronize(s));
    }
    struct E { float w; int32_t a, b; };
    std::vector<E> es;
    es.reserve((size_t)nq * (R + 1));
    const int32_t sn = ix.entry;
    for (int64_t i = 0; i < nq; ++i) {
        const int32_t u = (int32_t)(nx + i);
        for (int j = 0; j < R; ++j) {
            const int32_t v = adjq[(size_t)i * R + j];
            if (v < nx || v == u) continue;
            es.push_back({elq[(size_t)i * R + j], std::min(u, v), std::max(u, v)});
        }
        if (u != sn) es.push_back({ds[i], std::min(u, sn), std::max(u, sn)});
    }
    std::sort(es.begin(), es.end(), [](const E &x, const E &y) {
        if (x.w != y.w) return x.w < y.w;
        if (x.a != y.a) return x.a < y.a;
        return x.b < y.b;
    });
    // vertices: query indices 0..nq-1, plus slot nq for s when s is a data node
    auto vid = [&](int32_t node) -> int64_t { return node >= nx ? node - nx : nq; };
    std::vector<int64_t> uf((size_t)nq + 1);
    std::iota(uf.begin(), uf.end(), 0);
    auto find = [&](int64_t x) {
        while (uf[x] != x) { uf[x] = uf[uf[x]]; x = uf[x]; }
        return x;
    };
    std::vector<std::vector<int32_t>> tree((size_t)nq + 1);
    for (const E &e : es) {
        int64_t ra = find(vid(e.a)), rb = find(vid(e.b));
        if (ra == rb) continue;
        uf[std::max(ra, rb)] = std::min(ra, rb);
        tree[vid(e.a)].push_back(e.b);
        tree[vid(e.b)].push_back(e.a);
    }
    std::vector<int32_t> parent((size_t)std::max<int64_t>(nq, 1), -1), depth((size_t)std::max<int64_t>(nq, 1), 0);
    std::vector<uint8_t> seen((size_t)nq + 1, 0);
    std::vector<int32_t> queue;
    queue.reserve((size_t)nq + 1);
    queue.push_back(sn);
    seen[vid(sn)] = 1;
    for (size_t h = 0; h < queue.size(); ++h) {
        const int32_t u = queue[h];
        auto &kids = tree[vid(u)];
        std::sort(kids.begin(), kids.end());
        for (int32_t v : kids) {
            if (seen[vid(v)]) continue;
            seen[vid(v)] = 1;
            const int64_t qi = v - nx;
            parent[qi] = (u == sn) ? -1 : u;
            depth[qi] = (u == sn) ? 0 : depth[u - nx] + 1;
            queue.push_back(v);
        }
    }
    ix.parent.alloc((size_t)std::max<int64_t>(nq, 1) * sizeof(int32_t));
    ix.depth.alloc((size_t)std::max<int64_t>(nq, 1) * sizeof(int32_t));
    VJ_HIP(hipMemcpyAsync(ix.parent.p, parent.data(), (size_t)nq * sizeof(int32_t), hipMemcpyHostToDevice, s));
    VJ_HIP(hipMemcpyAsync(ix.depth.p, depth.data(), (size_t)nq * sizeof(int32_t), hipMemcpyHostToDevice, s));
    VJ_HIP(hipStreamSynchronize(s));
    ix.has_mst = true;
}

static void set_parents(Index &ix, const int32_t *parent, hipStream_t s) {
    const int64_t nq = ix.nq;
    std::vector<int32_t> par((size_t)std::max<int64_t>(nq, 1), -1), depth((size_t)std::max<int64_t>(nq, 1), -1);
    if (nq > 0) {
        VJ_HIP(hipMemcpyAsync(par.data(), parent, (size_t)nq * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        VJ_HIP(hipStreamSynchronize(s));
    }
    for (int64_t i = 0; i < nq; ++i) {
        const int32_t p = par[i];
        VJ_CHECK(p == -1 || (p >= ix.nx && p < ix.N && p != ix.nx + i), VJ_ERR_INVALID_ARG,
                 "parent ids must be query node ids or -1");
    }
    // depth by walking up (the parents must form a forest rooted at the entry)
    for (int64_t i = 0; i < nq; ++i) {
        std::vector<int64_t> chain;
        int64_t c = i;
        while (c >= 0 && depth[c] < 0) {
            chain.push_back(c);
            VJ_CHECK((int64_t)chain.size() <= nq, VJ_ERR_INVALID_ARG, "parent ids contain a cycle");
            c = par[c] >= 0 ? par[c] - ix.nx : -1;
        }
        int32_t d0 = c >= 0 ? depth[c] : -1;
        for (auto it = chain.rbegin(); it != chain.rend(); ++it) depth[*it] = ++d0;
    }
    ix.parent.alloc((size_t)std::max<int64_t>(nq, 1) * sizeof(int32_t));
    ix.depth.alloc((size_t)std::max<int64_t>(nq, 1) * sizeof(int32_t));
    VJ_HIP(hipMemcpyAsync(ix.parent.p, par.data(), (size_t)nq * sizeof(int32_t), hipMemcpyHostToDevice, s));
    VJ_HIP(hipMemcpyAsync(ix.depth.p, depth.data(), (size_t)nq * sizeof(int32_t), hipMemcpyHostToDevice, s));
    VJ_HIP(hipStreamSynchronize(s));
    ix.has_mst = true;
}

static void check_shape(const float *Q, int64_t nq, const float *X, int64_t nx, int32_t d) {
    VJ_CHECK(nq >= 0 && nx >= 1, VJ_ERR_INVALID_ARG, "need nq >= 0 and nx >= 1");
    VJ_CHECK(X != nullptr && (nq == 0 || Q != nullptr), VJ_ERR_INVALID_ARG, "null vector pointer");
    VJ_CHECK(d >= 1, VJ_ERR_INVALID_ARG, "d must be >= 1");
    VJ_CHECK(d <= 1024, VJ_ERR_UNSUPPORTED, "d must be <= 1024");
    VJ_CHECK(nq + nx < ((int64_t)1 << 31) - 1, VJ_ERR_UNSUPPORTED, "nq + nx must be < 2^31 - 1");
}

// An index's node ids must stay below 2^30: the workgroup tier of the join
// carries a flag in bit 30 of the node ids it stages.
static void check_index_size(int64_t nq, int64_t nx) {
    VJ_CHECK(nq + nx < ((int64_t)1 << 30), VJ_ERR_UNSUPPORTED, "an index needs nq + nx < 2^30");
}

// ------------------------------------------------------------------ join --

// Processing order: the caller's order in self mode; in soft / hard mode the
// queries sorted by MST depth, one launch per depth so that every parent
// finished in an earlier launch (any parent-before-child order gives the
// same result, Algorithm 3 reads only the parent's cache).
struct Order {
    DevBuf &qlist, &qpos;
    std::vector<int64_t> level_start;  // boundaries of the launches, last = n
};

static void make_order(Index &ix, const int32_t *ids, int64_t n, int ws, bool dense_first,
                       hipStream_t s, Order &o) {
    o.qlist.reserve(n * sizeof(int32_t));
    o.qpos.reserve(n * sizeof(int32_t));
    o.level_start.clear();
    if (ws == VJ_WS_SELF || ws == VJ_WS_NNMAP) {
        // queries are independent: any order gives the same result
        if (dense_first) {
            JoinWorkspace &jw = ix.jw;
            order_by_density(ix.adj.as<int32_t>(), ix.elen.as<float>(), ix.R, ix.nx, ix.nq, ids, n,
                             o.qlist.as<int32_t>(), o.qpos.as<int32_t>(), jw.sort_keys, jw.sort_tmp,
                             s);
        } else {
            if (ids) VJ_HIP(hipMemcpyAsync(o.qlist.p, ids, n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
            else iota_i32(o.qlist.as<int32_t>(), n, s);
            iota_i32(o.qpos.as<int32_t>(), n, s);
        }
        o.level_start = {0, n};
        return;
    }
    DevBuf tmp;
    order_by_depth(ix.depth.as<int32_t>(), ix.nq, ids, n, o.qlist.as<int32_t>(), o.qpos.as<int32_t>(), tmp, s);
    // depth of every processing slot, to cut the list into levels
    std::vector<int32_t> ql((size_t)n), dep((size_t)ix.nq);
    VJ_HIP(hipMemcpyAsync(ql.data(), o.qlist.p, n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    VJ_HIP(hipMemcpyAsync(dep.data(), ix.depth.p, ix.nq * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    VJ_HIP(hipStreamSynchronize(s));
    o.level_start.push_back(0);
    for (int64_t i = 1; i < n; ++i) {
        const int32_t a = ql[i - 1], b = ql[i];
        VJ_CHECK(a >= 0 && a < ix.nq && b >= 0 && b < ix.nq, VJ_ERR_INVALID_ARG, "query id out of range");
        if (dep[b] != dep[a]) o.level_start.push_back(i);
    }
    o.level_start.push_back(n);
}

// The join's arguments other than its outputs; ctr: the join counters
static JoinArgs make_args(const Index &ix, int prec, const vj_join_params &p, int beam, float eps,
                          const int32_t *budget, int32_t *ctr) {
    JoinArgs a{};
    a.rows = prec == VJ_PREC_U8     ? ix.vec_u8.p
             : prec == VJ_PREC_BF16 ? ix.vec_bf16.p
             : prec == VJ_PREC_FP8  ? ix.vec_f8.p
                                    : ix.vec.p;
    a.f8meta = prec == VJ_PREC_FP8 ? ix.f8meta.as<float2>() : nullptr;
    // RNE to bf16 has relative error <= 2^-8 of |x|, i.e. <= 2^-8 / (1 - 2^-8) of |bf16(x)|
    a.bf_u = prec == VJ_PREC_BF16 && !ix.bf16_exact ? 0.00392157f : 0.f;
    a.nrecheck = reinterpret_cast<unsigned long long *>(ctr + 6);
    a.rows32 = ix.vec.as<float>();
    a.adj = ix.adj.as<int32_t>();
    a.elen = ix.elen.as<float>();
    a.nx = ix.nx;
    a.nq = ix.nq;
    a.R = ix.R;
    a.dp = ix.dp;
    a.entry = ix.entry;
    a.metric = ix.metric;
    a.eps = eps;
    a.eps2 = (float)((double)eps * (double)eps);
    a.ws = p.work_sharing;
    a.hyb = p.hybrid;
    a.merged = ix.separate ? 0 : 1;
    a.gbeam = p.greedy_beam;
    a.qseed = p.layer_seeds && ix.separate && ix.lay_n > 0 ? ix.lay_seed.as<int32_t>() : nullptr;
    a.nn_w = ix.has_nnmap ? ix.nn_w.as<int32_t>() : nullptr;
    a.nn_d = ix.has_nnmap ? ix.nn_d.as<double>() : nullptr;
    a.nn_ood = ix.has_nnmap ? ix.nn_ood.as<uint8_t>() : nullptr;
    a.beam = beam;
    a.conv = p.conv_threshold;
    a.ood_ratio = p.ood_ratio;
    a.gen = ix.gen;
    a.parent = ix.has_mst ? ix.parent.as<int32_t>() : nullptr;
    a.inb = ix.inb.as<int32_t>();
    a.cache = ix.cache.as<int32_t>();
    a.seg = ix.seg.as<int64_t>();
    a.segn = ix.segn.as<int32_t>();
    a.budget = budget;
    a.out_count = reinterpret_cast<unsigned long long *>(ctr);
    a.err = ctr + 3;
    return a;
}

// Row type of a join: AUTO takes exact u8 rows when the data allows them
static int join_precision(Index &ix, int prec, hipStream_t s) {
    if (prec == VJ_PREC_AUTO) prec = ix.integer_u8 ? VJ_PREC_U8 : VJ_PREC_FP32;
    VJ_CHECK(prec != VJ_PREC_U8 || ix.integer_u8, VJ_ERR_INVALID_ARG,
             "u8 precision needs integer data in [0, 255]");
    VJ_CHECK(prec == VJ_PREC_FP32 || prec == VJ_PREC_U8 || prec == VJ_PREC_BF16 ||
                 prec == VJ_PREC_FP8,
             VJ_ERR_UNSUPPORTED, "precision not supported by the traversal");
    if (prec == VJ_PREC_BF16) ensure_bf16(ix, s);
    if (prec == VJ_PREC_FP8) ensure_f8(ix, s);
    return prec;
}

// the seeds of the listed queries (ids: query indexes, null = all) from the
// greedy descent through the index's upper layers, into ix.lay_seed[qi]
static void layer_seeds(Index &ix, const int32_t *ids, int64_t n, int32_t *seed_i, int32_t *moves,
                        hipStream_t s) {
    DevBuf err(sizeof(int32_t));
    VJ_HIP(hipMemsetAsync(err.p, 0, sizeof(int32_t), s));
    descend(ix.vec.as<float>(), ix.dp, ix.nx, ix.metric, ix.lay_n, ix.lay_offd.as<int64_t>(),
            ix.lay_offd.as<int64_t>() + ix.lay_n, ix.lay_pos.as<int32_t>(), ix.lay_adj.as<int32_t>(),
            ix.lay_R, ix.lay_entry.back(), ids, n, seed_i, seed_i ? nullptr : ix.lay_seed.as<int32_t>(),
            moves, err.as<int32_t>(), s);
    int32_t e = 0;
    VJ_HIP(hipMemcpyAsync(&e, err.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    VJ_HIP(hipStreamSynchronize(s));
    VJ_CHECK(e == 0, VJ_ERR_INTERNAL, "upper layers are not nested");
}

static void run_join(Index &ix, const int32_t *ids, int64_t n, float eps, const vj_join_params &p,
                     const int32_t *budget, hipStream_t s, Pairs &r) {
    if (p.layer_seeds && ix.separate && ix.lay_n > 0) layer_seeds(ix, ids, n, nullptr, nullptr, s);
    const int ws = p.work_sharing, hyb = p.hybrid;
    const int prec = join_precision(ix, p.precision, s);
    // bf16 rows run on the workgroup tiers (they carry the margin re-check)
    // bf16 rows and separate indexes run on the workgroup tiers (they carry
    // the margin re-check, resp. the greedy phase)
    const int start_tier = prec == VJ_PREC_BF16 || prec == VJ_PREC_FP8 || ix.separate
                               ? std::max(1, (int)p.start_tier)
                               : (int)p.start_tier;
    const int beam = (hyb != VJ_HYB_OFF) ? p.hybrid_beam : 0;
    VJ_CHECK(beam <= 256, VJ_ERR_UNSUPPORTED, "hybrid_beam must be <= 256");
    // persistent launch of the workgroup tier (the one-wave tier is not
    // persistent: a request for it falls back to per-level launches)
    const bool persist = p.persistent != 0 && start_tier == 1;

    JoinWorkspace &jw = ix.jw;
    Order ord{jw.qlist, jw.qpos, {}};
    // densest first reads the stored lengths of a query's edges to data
    // nodes: the merged graph's (a separate query graph has none)
    make_order(ix, ids, n, ws, p.dense_first != 0 && !ix.separate, s, ord);
    const int32_t *qlist = ord.qlist.as<int32_t>(), *qpos = ord.qpos.as<int32_t>();

    // counters: [0..1] out_count (u64), [2] ovf_count, [3] err, [4] global regions taken,
    // [6..7] bf16 re-checks (u64)
    jw.counters.reserve(64);
    jw.args.reserve(sizeof(JoinArgs));
    jw.ovf.reserve((size_t)std::max<int64_t>(n, 1) * sizeof(int32_t));
    DevBuf &counters = jw.counters, &argsbuf = jw.args, &ovf = jw.ovf, &sl = jw.slots;
    DevBuf &out_q = jw.out_q, &out_x = jw.out_x, &out_d = jw.out_d;
    DevBuf gh, gil, gild, q2, p2;
    r.stats.alloc((size_t)std::max<int64_t>(n, 1) * 8 * sizeof(int32_t));
    int32_t *ctr = counters.as<int32_t>();

    int64_t cap = p.pair_capacity > 0
                      ? p.pair_capacity
                      : std::max<int64_t>({1 << 16, n * 64, (int64_t)(out_q.bytes / sizeof(int32_t))});
    if (!jw.ev0) VJ_HIP(hipEventCreate(&jw.ev0));
    if (!jw.ev1) VJ_HIP(hipEventCreate(&jw.ev1));
    if (!jw.pinned) VJ_HIP(hipHostMalloc(&jw.pinned, 4096, hipHostMallocDefault));
    hipEvent_t ev0 = jw.ev0, ev1 = jw.ev1;
    // pinned host staging: [0, 64) the counters read back, [256, ...) the arguments
    int32_t *hctr = static_cast<int32_t *>(jw.pinned);
    JoinArgs *args_h = reinterpret_cast<JoinArgs *>(static_cast<char *>(jw.pinned) + 256);
    static_assert(sizeof(JoinArgs) <= 4096 - 256, "JoinArgs exceeds the pinned staging area");
    for (int attempt = 0; attempt < 4; ++attempt) {
        r.kernel_ms = 0.f;
        r.spill_ms = 0.f;
        r.n_spilled = 0;
        for (int t = 0; t < 4; ++t) {
            r.tier_ms[t] = 0.f;
            r.tier_launches[t] = 0;
            r.tier_queries[t] = 0;
        }
        out_q.reserve((size_t)cap * sizeof(int32_t));
        out_x.reserve((size_t)cap * sizeof(int32_t));
        out_d.reserve((size_t)cap * sizeof(float));
        ix.gen += 1;
        VJ_HIP(hipMemsetAsync(counters.p, 0, 64, s));
        if (ws == VJ_WS_SOFT || ws == VJ_WS_HARD)
            stamp_batch(ix.inb.as<int32_t>(), ix.nq, ids, n, ix.gen, ctr + 3, s);

        JoinArgs a = make_args(ix, prec, p, beam, eps, budget, ctr);
        a.out_q = out_q.as<int32_t>();
        a.out_x = out_x.as<int32_t>();
        a.out_d = out_d.as<float>();
        a.cap = cap;
        a.out_count = reinterpret_cast<unsigned long long *>(ctr);
        a.stats = r.stats.as<int32_t>();
        a.err = ctr + 3;
        a.done = persist && (ws == VJ_WS_SOFT || ws == VJ_WS_HARD) ? ix.done.as<int32_t>() : nullptr;
        *args_h = a;
        VJ_HIP(hipMemcpyAsync(argsbuf.p, args_h, sizeof(a), hipMemcpyHostToDevice, s));
        std::memset(hctr, 0, 64);
        // One launch (or a sequence of chunks, global tiers) of `cnt` slots
        // of the lists lq/lp on tier `tier`; returns the device time.
        auto run_tier = [&](int tier, const int32_t *lq, const int32_t *lp, int64_t cnt) -> float {
            JoinLaunch L{};
            L.args = argsbuf.as<JoinArgs>();
            L.qlist = lq;
            L.qpos = lp;
            L.dp = ix.dp;
            L.prec = prec;
            L.tier = std::min(tier, 2);
            L.coop_small = p.coop_tables == 1;
            // the greedy phase of separate indexes keeps its queue in the
            // out-range queue's arrays
            L.hyb = beam > 0 || ix.separate;
            L.ovf = ovf.as<int32_t>();
            L.ovf_count = ctr + 2;
            int64_t chunk = cnt;
            // global tables: 2^16 visited slots (32,768 nodes) and 32,768
            // pairs per region (smaller for small data sets), kept in the
            // index; tier 3 tables are as large as the data set
            const int hl2 = std::min(16, ceil_log2(2 * ix.nx));
            const int ilc2 = (int)std::min<int64_t>(ix.nx, 1 << 15);
            auto global_regions = [&](int64_t regions, int hl, int ilc) {
                ix.ws_gh.reserve((size_t)regions * ((size_t)1 << hl) * sizeof(int32_t));
                ix.ws_gil.reserve((size_t)regions * ilc * sizeof(int32_t));
                ix.ws_gild.reserve((size_t)regions * ilc * sizeof(float));
                L.gh = ix.ws_gh.as<int32_t>();
                L.gil = ix.ws_gil.as<int32_t>();
                L.gild = ix.ws_gild.as<float>();
                L.hash_log2 = hl;
                L.il_cap = ilc;
            };
            if (tier == 1) {
                // regions a query that outgrows LDS may take within the launch;
                // the small LDS tables overflow more often, so they get more
                // (and smaller: 2^15 slots, 16,384 pairs) regions
                if (L.coop_small) {
                    L.promo_cap = (int)std::min<int64_t>(4096, std::max<int64_t>(64, cnt / 16));
                    global_regions(L.promo_cap, std::min(15, ceil_log2(2 * ix.nx)),
                                   (int)std::min<int64_t>(ix.nx, 1 << 14));
                } else {
                    // about 1.5 % of the queries outgrow the large LDS tables
                    L.promo_cap = (int)std::min<int64_t>(4096, std::max<int64_t>(64, cnt / 32));
                    global_regions(L.promo_cap, hl2, ilc2);
                }
                L.promo_next = ctr + 4;
                VJ_HIP(hipMemsetAsync(ctr + 4, 0, sizeof(int32_t), s));
                if (persist) {
                    // resident workgroups (four per CU) claim the slots in order
                    L.claim = ctr + 5;
                    L.grid = (int)std::min<int64_t>(cnt, (int64_t)num_cus() * 4);
                    VJ_HIP(hipMemsetAsync(ctr + 5, 0, sizeof(int32_t), s));
                }
            } else if (tier == 2) {
                chunk = 1024;
                global_regions(std::min(chunk, cnt), hl2, ilc2);
            } else if (tier == 3) {
                L.hash_log2 = ceil_log2(2 * ix.nx);
                L.il_cap = (int)ix.nx;
                chunk = 16;
                gh.reserve((size_t)std::min(chunk, cnt) * ((size_t)1 << L.hash_log2) * sizeof(int32_t));
                gil.reserve((size_t)std::min(chunk, cnt) * L.il_cap * sizeof(int32_t));
                gild.reserve((size_t)std::min(chunk, cnt) * L.il_cap * sizeof(float));
                L.gh = gh.as<int32_t>();
                L.gil = gil.as<int32_t>();
                L.gild = gild.as<float>();
            }
            // one launch: the caller's synchronisation completes the events; a
            // sequence of chunks synchronises per chunk (they share the scratch)
            float total_ms = 0.f;
            const bool single = chunk >= cnt;
            for (int64_t c0 = 0; c0 < cnt; c0 += chunk) {
                L.first = (int)c0;
                L.count = (int)std::min<int64_t>(chunk, cnt - c0);
                VJ_HIP(hipEventRecord(ev0, s));
                VJ_CHECK(launch_join(L, s), VJ_ERR_UNSUPPORTED, "no join kernel for this row width");
                VJ_HIP(hipGetLastError());
                VJ_HIP(hipEventRecord(ev1, s));
                if (!single) {
                    VJ_HIP(hipStreamSynchronize(s));
                    float ms = 0.f;
                    VJ_HIP(hipEventElapsedTime(&ms, ev0, ev1));
                    total_ms += ms;
                }
                r.tier_launches[tier] += 1;
            }
            r.tier_queries[tier] += cnt;
            return single ? -1.f : total_ms;
        };
        // Runs `pending` slots of lq / lp on tier `tier`, then the queries that
        // outgrew it, in processing order, on the next tiers (up to tier
        // `last`); on return lq / lp / pending hold what is left.
        auto chain = [&](int tier, const int32_t *&lq, const int32_t *&lp, int64_t &pending,
                         int last) {
            for (; pending > 0 && tier <= last; ++tier) {
                VJ_CHECK(tier <= 3, VJ_ERR_INTERNAL, "join tiers exhausted");
                VJ_HIP(hipMemsetAsync(ctr + 2, 0, sizeof(int32_t), s));
                float ms = run_tier(tier, lq, lp, pending);
                VJ_HIP(hipMemcpyAsync(hctr, ctr, 64, hipMemcpyDeviceToHost, s));
                VJ_HIP(hipStreamSynchronize(s));
                if (ms < 0.f) VJ_HIP(hipEventElapsedTime(&ms, ev0, ev1));
                r.tier_ms[tier] += ms;
                if (tier == start_tier) r.kernel_ms += ms;
                else r.spill_ms += ms;
                VJ_CHECK(!(hctr[3] & 8), VJ_ERR_INVALID_ARG, "query id out of range");
                pending = hctr[2];
                if (pending == 0) break;
                r.n_spilled += tier == start_tier ? pending : 0;
                std::vector<int32_t> slots_h((size_t)pending);
                VJ_HIP(hipMemcpyAsync(slots_h.data(), ovf.p, pending * sizeof(int32_t), hipMemcpyDeviceToHost, s));
                VJ_HIP(hipStreamSynchronize(s));
                std::sort(slots_h.begin(), slots_h.end());
                sl.reserve(pending * sizeof(int32_t));
                VJ_HIP(hipMemcpyAsync(sl.p, slots_h.data(), pending * sizeof(int32_t), hipMemcpyHostToDevice, s));
                DevBuf nq2(pending * sizeof(int32_t)), np2(pending * sizeof(int32_t));
                gather_slots(lq, lp, sl.as<int32_t>(), pending, nq2.as<int32_t>(), np2.as<int32_t>(), s);
                VJ_HIP(hipStreamSynchronize(s));
                q2 = std::move(nq2);
                p2 = std::move(np2);
                lq = q2.as<int32_t>();
                lp = p2.as<int32_t>();
            }
            VJ_CHECK(!(hctr[3] & 16), VJ_ERR_INTERNAL, "visited-set probe exceeded the table size");
            VJ_CHECK(!(hctr[3] & 32), VJ_ERR_INTERNAL, "a worklist entry is not a data node id");
            VJ_CHECK(!(hctr[3] & 128), VJ_ERR_INTERNAL, "a join wave waited past its bound");
            VJ_CHECK(!(hctr[3] & 256), VJ_ERR_INTERNAL, "a query waited past its bound for its parent");
        };
        if (persist) {
            // one persistent launch over every slot (all MST levels: children
            // wait on the device for their parents), then the queries that
            // outgrew it, level by level in processing order
            const int32_t *lq = qlist, *lp = qpos;
            int64_t pending = n;
            chain(1, lq, lp, pending, 1);
            if (pending > 0) {
                std::vector<int64_t> cuts{0};
                if (ws == VJ_WS_SOFT || ws == VJ_WS_HARD) {
                    std::vector<int32_t> ql((size_t)pending), dep((size_t)ix.nq);
                    VJ_HIP(hipMemcpyAsync(ql.data(), lq, pending * sizeof(int32_t), hipMemcpyDeviceToHost, s));
                    VJ_HIP(hipMemcpyAsync(dep.data(), ix.depth.p, ix.nq * sizeof(int32_t), hipMemcpyDeviceToHost, s));
                    VJ_HIP(hipStreamSynchronize(s));
                    for (int64_t i = 1; i < pending; ++i)
                        if (dep[ql[i]] != dep[ql[i - 1]]) cuts.push_back(i);
                }
                cuts.push_back(pending);
                // the overflow list outlives the chains below (they replace q2 / p2)
                DevBuf keep_q = std::move(q2), keep_p = std::move(p2);
                const int32_t *bq = keep_q.as<int32_t>(), *bp = keep_p.as<int32_t>();
                for (size_t c = 0; c + 1 < cuts.size(); ++c) {
                    const int32_t *cq = bq + cuts[c], *cp = bp + cuts[c];
                    int64_t cn = cuts[c + 1] - cuts[c];
                    chain(2, cq, cp, cn, 3);
                }
            }
        } else {
            for (size_t lv = 0; lv + 1 < ord.level_start.size(); ++lv) {
                // one MST level (all queries, self mode): the first tier, then
                // the queries that outgrew it on the next tiers
                const int64_t first = ord.level_start[lv];
                int64_t pending = ord.level_start[lv + 1] - first;
                const int32_t *lq = qlist + first, *lp = qpos + first;
                chain(start_tier, lq, lp, pending, 3);
            }
        }
        const int64_t total = (int64_t)(((uint64_t)(uint32_t)hctr[1] << 32) | (uint32_t)hctr[0]);
        if (total <= cap) {
            unsigned long long nre = 0;
            std::memcpy(&nre, hctr + 6, sizeof(nre));  // read back with the last counters
            // the result owns exact-size copies (one allocation for the three
            // arrays); the workspace keeps its buffers
            const size_t m = (size_t)std::max<int64_t>(total, 1);
            DevBuf block(m * (2 * sizeof(int32_t) + sizeof(float)));
            r.x = DevBuf::view(block.as<char>() + m * sizeof(int32_t), m * sizeof(int32_t));
            r.dist = DevBuf::view(block.as<char>() + 2 * m * sizeof(int32_t), m * sizeof(float));
            r.q = std::move(block);
            r.q.bytes = m * sizeof(int32_t);
            if (total > 0) {
                VJ_HIP(hipMemcpyAsync(r.q.p, out_q.p, total * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
                VJ_HIP(hipMemcpyAsync(r.x.p, out_x.p, total * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
                VJ_HIP(hipMemcpyAsync(r.dist.p, out_d.p, total * sizeof(float), hipMemcpyDeviceToDevice, s));
            }
            VJ_HIP(hipStreamSynchronize(s));
            r.n_candidates = (int64_t)nre;
            r.count = total;
            r.n_queries = n;
            return;
        }
        cap = total + total / 16 + 1024;
    }
    VJ_CHECK(false, VJ_ERR_INTERNAL, "result capacity did not converge");
}

// VJ_HYB_LEARNED: features after the probe -> the attached MLP -> the
// smallest budget whose predicted recall reaches the target; the join then
// runs in budget mode, and the queries no budget satisfies (budget -1) are
// joined exactly on the MFMA tiles, their pairs appended.
static void learned_join(Index &ix, const int32_t *ids, int64_t n, float eps, vj_join_params p,
                         hipStream_t s, Pairs &r) {
    const Predictor &P = *ix.pred;
    VJ_CHECK(P.din == ix.d + kFeatures, VJ_ERR_INVALID_ARG, "predictor input width is not d + 8");
    std::vector<int32_t> ids_h((size_t)n);
    if (ids) {
        VJ_HIP(hipMemcpyAsync(ids_h.data(), ids, n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        VJ_HIP(hipStreamSynchronize(s));
        for (int32_t q : ids_h) VJ_CHECK(q >= 0 && q < ix.nq, VJ_ERR_INVALID_ARG, "query id out of range");
    } else {
        for (int64_t i = 0; i < n; ++i) ids_h[(size_t)i] = (int32_t)i;
    }
    DevBuf ql((size_t)n * sizeof(int32_t));
    VJ_HIP(hipMemcpyAsync(ql.p, ids_h.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, s));
    DevBuf feat((size_t)n * (ix.d + kFeatures) * sizeof(float)), logits((size_t)n * P.k * sizeof(float)),
        bud((size_t)n * sizeof(int32_t));
    compute_features(ix, ql.as<int32_t>(), n, eps, ix.d + kFeatures, feat.as<float>(), s);
    predictor_forward(P, feat.as<float>(), n, logits.as<float>(), s);
    select_budgets(logits.as<float>(), n, P.k, ix.pred_budgets.as<int32_t>(), ix.pred_target,
                   bud.as<int32_t>(), s);
    std::vector<int32_t> bud_h((size_t)n), routed;
    VJ_HIP(hipMemcpyAsync(bud_h.data(), bud.p, n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    VJ_HIP(hipStreamSynchronize(s));
    p.hybrid = VJ_HYB_BUDGET;
    // no query got out-range pops: the kernels without the out-range queue
    // run it (budget 0 is BFS; routed queries are skipped either way)
    if (*std::max_element(bud_h.begin(), bud_h.end()) <= 0) p.hybrid_beam = 0;
    run_join(ix, ids, n, eps, p, bud.as<int32_t>(), s, r);
    // queries routed to the exact join
    for (int64_t i = 0; i < n; ++i)
        if (bud_h[(size_t)i] < 0) routed.push_back(ids_h[(size_t)i]);
    if (routed.empty()) return;
    const int64_t nr = (int64_t)routed.size();
    DevBuf rl((size_t)nr * sizeof(int32_t)), rows((size_t)nr * ix.dp * sizeof(float));
    VJ_HIP(hipMemcpyAsync(rl.p, routed.data(), nr * sizeof(int32_t), hipMemcpyHostToDevice, s));
    gather_rows(ix.vec.as<float>() + (size_t)ix.nx * ix.dp, ix.dp, rl.as<int32_t>(), nr,
                rows.as<float>(), s);
    // the exact join on MFMA tiles: with low-precision rows the one-term bf16
    // tiles (a proven margin, fp64 re-check; a third of the fp32 form's
    // MFMA work), else the three-term form; both give the exact pair set
    const vj_precision rp = p.precision == VJ_PREC_BF16 || p.precision == VJ_PREC_FP8
                                ? VJ_PREC_BF16 : VJ_PREC_FP32;
    Pairs bp;
    bruteforce_join(rows.as<float>(), nr, ix.vec.as<float>(), ix.nx, ix.dp, eps, ix.metric, rp, s,
                    bp);
    if (bp.count == 0) return;
    remap_ids(bp.q.as<int32_t>(), bp.count, rl.as<int32_t>(), s);
    const int64_t tot = r.count + bp.count;
    DevBuf q2((size_t)tot * sizeof(int32_t)), x2((size_t)tot * sizeof(int32_t)),
        d2((size_t)tot * sizeof(float));
    auto cat = [&](DevBuf &dst, const DevBuf &a, const DevBuf &b, size_t el) {
        if (r.count) VJ_HIP(hipMemcpyAsync(dst.p, a.p, (size_t)r.count * el, hipMemcpyDeviceToDevice, s));
        VJ_HIP(hipMemcpyAsync(dst.as<char>() + (size_t)r.count * el, b.p, (size_t)bp.count * el,
                              hipMemcpyDeviceToDevice, s));
    };
    cat(q2, r.q, bp.q, sizeof(int32_t));
    cat(x2, r.x, bp.x, sizeof(int32_t));
    cat(d2, r.dist, bp.dist, sizeof(float));
    VJ_HIP(hipStreamSynchronize(s));
    r.q = std::move(q2);
    r.x = std::move(x2);
    r.dist = std::move(d2);
    r.count = tot;
}

// arguments shared by the two batch runners
static void check_batches(const vj_index *idx, const int32_t *query_ids, const int64_t *st,
                          const int64_t *ct, const float *eps, int32_t nb, vj_pairs **out) {
    VJ_CHECK(idx != nullptr && out != nullptr && st != nullptr && ct != nullptr && eps != nullptr &&
                 nb >= 0,
             VJ_ERR_INVALID_ARG, "null pointer or negative batch count");
    for (int32_t b = 0; b < nb; ++b) {
        VJ_CHECK(st[b] >= 0 && ct[b] >= 0, VJ_ERR_INVALID_ARG, "batch ranges must be >= 0");
        VJ_CHECK(query_ids != nullptr ? true : st[b] + ct[b] <= idx->impl.nq, VJ_ERR_INVALID_ARG,
                 "batch range beyond the queries");
        VJ_CHECK(std::isfinite(eps[b]), VJ_ERR_INVALID_ARG, "eps must be finite");
    }
}

// ---------------------------------------------------- device batch runner --
// The steps of a batch (self mode) run with no host synchronisation between
// batches, their parameters read from descriptors in device memory: start (eps, stats rows,
// counters, the batch's query list and d1 buckets) -> densest
// neighbourhoods first (bucket scan and scatter; or the caller's order) ->
// the workgroup tier with in-launch promotion -> the queries it could not
// hold, read through its overflow list, on global tables (a fixed grid
// looping over a count on the device) -> the queries those could not hold,
// on tables as large as the data set
// -> end (pair range, clock, cursor).  The steps are launched directly, or
// captured as a HIP graph of up to kSteps steps that is replayed (and kept
// for the next call of the same launch shape).  Two replay slots,
// each with its own state, graph and stream, take the even and the odd
// batches, so that one batch's tail overlaps the next batch's start; within
// a slot batches run in order, so the pairs of each batch are contiguous in
// its slot's output.
namespace {

constexpr int kSlots = 2;
constexpr int kSteps = 16;

}  // namespace

static void run_batches_device(Index &ix, const int32_t *ids, const int64_t *st_h,
                               const int64_t *ct_h, const float *eps_h, int32_t nb,
                               const vj_join_params &p, bool graph, hipStream_t s,
                               std::vector<std::unique_ptr<vj_pairs>> &res, float *batch_ms) {
    VJ_CHECK(p.work_sharing == VJ_WS_SELF, VJ_ERR_UNSUPPORTED,
             "the device batch runner joins in self mode only");
    VJ_CHECK(p.hybrid == VJ_HYB_OFF || p.hybrid == VJ_HYB_FORCE || p.hybrid == VJ_HYB_ADAPT,
             VJ_ERR_UNSUPPORTED, "the device batch runner takes hybrid off, force or adapt");
    const int prec = join_precision(ix, p.precision, s);
    const int beam = (p.hybrid != VJ_HYB_OFF) ? p.hybrid_beam : 0;
    VJ_CHECK(beam <= 256, VJ_ERR_UNSUPPORTED, "hybrid_beam must be <= 256");

    int64_t nmax = 0, total_q = 0;
    std::vector<int64_t> stats_off((size_t)nb);
    for (int32_t b = 0; b < nb; ++b) {
        stats_off[(size_t)b] = total_q;
        total_q += ct_h[b];
        if (!(ix.metric == VJ_L2 && eps_h[b] <= 0.0f)) nmax = std::max<int64_t>(nmax, ct_h[b]);
    }
    auto stats = std::make_shared<DevBuf>((size_t)std::max<int64_t>(total_q, 1) * 8 * sizeof(int32_t));
    VJ_HIP(hipMemsetAsync(stats->p, 0, stats->bytes, s));
    // descriptors of each slot (batch b goes to slot b % 2, entry b / 2),
    // padded to whole graphs with batches that run nothing; a batch with
    // nothing to find (L2, eps <= 0) runs nothing either
    const int nsl = nb > 1 ? kSlots : 1;
    std::vector<BatchDesc> desc[kSlots];
    for (int32_t b = 0; b < nb; ++b) {
        BatchDesc d{};
        d.ids = ids;
        d.stats = stats->as<int32_t>() + stats_off[(size_t)b] * 8;
        d.start = st_h[b];
        d.count = (ix.metric == VJ_L2 && eps_h[b] <= 0.0f) ? 0 : (int32_t)ct_h[b];
        d.eps = eps_h[b];
        d.eps2 = (float)((double)eps_h[b] * (double)eps_h[b]);
        desc[b % kSlots].push_back(d);
    }
    const int64_t per_slot = (nb + nsl - 1) / nsl;
    // steps per submission: a graph of up to kSteps, or one step launched directly
    const int steps = graph ? (int)std::min<int64_t>(kSteps, std::max<int64_t>(per_slot, 1)) : 1;
    int launches[kSlots] = {0, 0};
    for (int k = 0; k < nsl; ++k) {
        launches[k] = (int)((desc[k].size() + steps - 1) / steps);
        BatchDesc pad{};
        pad.stats = stats->as<int32_t>();
        desc[k].resize((size_t)launches[k] * steps, pad);
    }
    JoinWorkspace &jw = ix.jw;
    int hz = 0;  // device wall clock, kHz
    VJ_HIP(hipDeviceGetAttribute(&hz, hipDeviceAttributeWallClockRate, ix.device));
    // results: slot k's pairs sit at base[k] in the block of all pairs
    auto make_results = [&](const std::shared_ptr<DevBuf> &block, int64_t total, const int64_t *base,
                            const std::vector<uint64_t> *rec) {
        const size_t m = (size_t)std::max<int64_t>(total, 1);
        for (int32_t b = 0; b < nb; ++b) {
            const int k = b % kSlots;
            const BatchDesc &d = desc[k][(size_t)(b / kSlots)];
            auto h = std::make_unique<vj_pairs>();
            Pairs &r = h->impl;
            r.n_queries = ct_h[b];
            r.stats = DevBuf::view(d.stats, (size_t)ct_h[b] * 8 * sizeof(int32_t));
            r.keep.push_back(stats);
            if (block) {
                const uint64_t *rb = rec[k].data() + (size_t)(b / kSlots) * kBatchRec;
                const int64_t begin = base[k] + (int64_t)rb[0], cnt = (int64_t)(rb[1] - rb[0]);
                r.count = cnt;
                r.q = DevBuf::view(block->as<int32_t>() + begin, cnt * sizeof(int32_t));
                r.x = DevBuf::view(block->as<int32_t>() + m + begin, cnt * sizeof(int32_t));
                r.dist = DevBuf::view(block->as<float>() + 2 * m + begin, cnt * sizeof(float));
                r.keep.push_back(block);
                r.n_candidates = (int64_t)(rb[5] - rb[4]);
                r.tier_queries[1] = d.count;
                r.tier_queries[2] = (int64_t)rb[2];
                r.tier_queries[3] = (int64_t)rb[3];
                r.tier_launches[1] = d.count > 0;
                r.tier_launches[2] = rb[2] > 0;
                r.tier_launches[3] = rb[3] > 0;
                r.n_spilled = (int64_t)rb[2];
                const float ms = hz > 0 ? (float)((double)(rb[7] - rb[6]) / (double)hz) : 0.f;
                r.kernel_ms = ms;
                r.tier_ms[1] = ms;
                if (batch_ms) batch_ms[b] = ms;
            } else if (batch_ms) {
                batch_ms[b] = 0.f;
            }
            res[(size_t)b] = std::move(h);
        }
    };
    if (nmax == 0) {
        VJ_HIP(hipStreamSynchronize(s));
        make_results(nullptr, 0, nullptr, nullptr);
        return;
    }

    if (!jw.pinned) VJ_HIP(hipHostMalloc(&jw.pinned, 4096, hipHostMallocDefault));
    if (!jw.capture) VJ_HIP(hipStreamCreateWithFlags(&jw.capture, hipStreamNonBlocking));
    for (auto &e : jw.bev)
        if (!e) VJ_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    // pinned staging: counters of slot k at [64 k, 64 k + 64), arguments at 256 + 1024 k
    static_assert(sizeof(JoinArgs) <= 1024, "JoinArgs exceeds its pinned staging slot");
    int32_t *hctr = static_cast<int32_t *>(jw.pinned);
    const bool dense = p.dense_first != 0;
    const bool small = p.coop_tables == 1;
    const int hl2 = std::min(16, ceil_log2(2 * ix.nx));
    const int ilc2 = (int)std::min<int64_t>(ix.nx, 1 << 15);
    const int hl1 = small ? std::min(15, ceil_log2(2 * ix.nx)) : hl2;
    const int ilc1 = small ? (int)std::min<int64_t>(ix.nx, 1 << 14) : ilc2;
    const int promo_cap = (int)std::min<int64_t>(4096, std::max<int64_t>(64, small ? nmax / 16 : nmax / 32));
    const int g2 = (int)std::min<int64_t>(1024, nmax);
    const int g3 = (int)std::min<int64_t>(16, nmax);
    const int hl3 = ceil_log2(2 * ix.nx);
    // global tables: the promotion regions of the first launch and the
    // regions of the re-run share one buffer (the launches do not overlap)
    const size_t gh_n = std::max(((size_t)promo_cap) << hl1, ((size_t)g2) << hl2);
    const size_t il_n = std::max((size_t)promo_cap * ilc1, (size_t)g2 * ilc2);

    // seven lists of nmax slots per replay slot: the processing list and
    // positions, the overflow list of each launch, the batch's ids in caller
    // order and their density buckets; then the bucket counts and offsets
    struct Lists {
        int32_t *lq1, *lp1, *ovf1, *ovf2, *ovf3, *lq0, *bucket;
        uint32_t *hist, *boff;
    } L[kSlots];
    for (int k = 0; k < nsl; ++k) {
        BatchSlot &S = jw.bslot[k];
        S.args.reserve(sizeof(JoinArgs));
        S.counters.reserve(64);
        S.desc.reserve(desc[k].size() * sizeof(BatchDesc));
        S.rec.reserve(desc[k].size() * kBatchRec * sizeof(uint64_t));
        S.lists.reserve((size_t)nmax * 7 * sizeof(int32_t) + 2 * kOrderBuckets * sizeof(uint32_t));
        S.gh.reserve(gh_n * sizeof(int32_t));
        S.gil.reserve(il_n * sizeof(int32_t));
        S.gild.reserve(il_n * sizeof(float));
        S.gh3.reserve(((size_t)g3 << hl3) * sizeof(int32_t));
        S.gil3.reserve((size_t)g3 * ix.nx * sizeof(int32_t));
        S.gild3.reserve((size_t)g3 * ix.nx * sizeof(float));
        if (!S.stream) VJ_HIP(hipStreamCreateWithFlags(&S.stream, hipStreamNonBlocking));
        Lists &l = L[k];
        l.lq1 = S.lists.as<int32_t>();
        l.lp1 = l.lq1 + nmax;
        l.ovf1 = l.lp1 + nmax;
        l.ovf2 = l.ovf1 + nmax;
        l.ovf3 = l.ovf2 + nmax;
        l.lq0 = l.ovf3 + nmax;
        l.bucket = l.lq0 + nmax;
        l.hist = reinterpret_cast<uint32_t *>(l.bucket + nmax);
        l.boff = l.hist + kOrderBuckets;
    }

    auto launch = [&](BatchSlot &S, int tier, const int32_t *lq, const int32_t *lp,
                      const int32_t *sl, const int32_t *cnt, int32_t *ovf, int32_t *ovf_cnt,
                      hipStream_t cs) {
        JoinLaunch J{};
        J.args = S.args.as<JoinArgs>();
        J.qlist = lq;
        J.qpos = lp;
        J.slots = sl;
        J.first = 0;
        J.count = (int)nmax;
        J.count_dev = cnt;
        J.dp = ix.dp;
        J.prec = prec;
        J.tier = tier;
        J.coop_small = tier == 1 && small;
        J.hyb = beam > 0;
        J.ovf = ovf;
        J.ovf_count = ovf_cnt;
        J.gh = S.gh.as<int32_t>();
        J.gil = S.gil.as<int32_t>();
        J.gild = S.gild.as<float>();
        if (tier == 1) {
            J.hash_log2 = hl1;
            J.il_cap = ilc1;
            J.promo_next = S.counters.as<int32_t>() + 4;
            J.promo_cap = promo_cap;
        } else if (tier == 2) {
            J.hash_log2 = hl2;
            J.il_cap = ilc2;
            J.grid = g2;
        } else {
            J.tier = 2;
            J.gh = S.gh3.as<int32_t>();
            J.gil = S.gil3.as<int32_t>();
            J.gild = S.gild3.as<float>();
            J.hash_log2 = hl3;
            J.il_cap = (int)ix.nx;
            J.grid = g3;
        }
        VJ_CHECK(launch_join(J, cs), VJ_ERR_UNSUPPORTED, "no join kernel for this row width");
    };

    // one batch step of slot k on stream cs
    auto enqueue_step = [&](int k, hipStream_t cs) {
        BatchSlot &S = jw.bslot[k];
        const Lists &l = L[k];
        int32_t *ctr = S.counters.as<int32_t>();
        const BatchDesc *dd = S.desc.as<BatchDesc>();
        uint64_t *rec = S.rec.as<uint64_t>();
        if (dense) {
            batch_start(dd, S.args.as<JoinArgs>(), ctr, rec, nmax, ix.adj.as<int32_t>(),
                        ix.elen.as<float>(), ix.R, ix.nx, ix.nq, l.lq0, l.bucket, l.hist, cs);
            batch_order(l.lq0, ctr, nmax, l.bucket, l.hist, l.boff, l.lq1, l.lp1, cs);
        } else {
            batch_start(dd, S.args.as<JoinArgs>(), ctr, rec, nmax, ix.adj.as<int32_t>(),
                        ix.elen.as<float>(), ix.R, ix.nx, ix.nq, l.lq1, nullptr, nullptr, cs);
        }
        // the re-runs read their queries through the overflow lists (slots
        // of the first list) and append slots of the first list
        launch(S, 1, l.lq1, l.lp1, nullptr, ctr + kBatchCount, l.ovf1, ctr + 2, cs);
        launch(S, 2, l.lq1, l.lp1, l.ovf1, ctr + 2, l.ovf2, ctr + kBatchOvf2, cs);
        launch(S, 3, l.lq1, l.lp1, l.ovf2, ctr + kBatchOvf2, l.ovf3, ctr + kBatchOvf3, cs);
        batch_end(ctr, rec, cs);
    };

    // the graph of each slot: kept while the launch shape and the buffers
    // it names are the same
    hipStream_t cs = jw.capture;
    for (int k = 0; k < nsl && graph; ++k) {
        BatchSlot &S = jw.bslot[k];
        const Lists &l = L[k];
        const std::vector<uint64_t> key = {
            (uint64_t)steps, (uint64_t)nmax, (uint64_t)dense, (uint64_t)small, (uint64_t)prec,
            (uint64_t)beam, (uint64_t)ix.dp, (uint64_t)(uintptr_t)ix.adj.p,
            (uint64_t)(uintptr_t)ix.elen.p, (uint64_t)(uintptr_t)S.args.p,
            (uint64_t)(uintptr_t)S.counters.p, (uint64_t)(uintptr_t)S.desc.p,
            (uint64_t)(uintptr_t)S.rec.p, (uint64_t)(uintptr_t)S.lists.p, (uint64_t)(uintptr_t)S.gh.p,
            (uint64_t)(uintptr_t)S.gil.p, (uint64_t)(uintptr_t)S.gild.p, (uint64_t)(uintptr_t)S.gh3.p,
            (uint64_t)(uintptr_t)S.gil3.p, (uint64_t)(uintptr_t)S.gild3.p};
        if (S.exec && S.key == key) continue;
        if (S.exec) {
            (void)hipGraphExecDestroy(S.exec);
            S.exec = nullptr;
            S.key.clear();
        }
        hipGraph_t g = nullptr;
        VJ_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        try {
            for (int step = 0; step < steps; ++step) enqueue_step(k, cs);
            VJ_HIP(hipGetLastError());
        } catch (...) {
            (void)hipStreamEndCapture(cs, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
        }
        VJ_HIP(hipStreamEndCapture(cs, &g));
        const hipError_t e = hipGraphInstantiate(&S.exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            S.exec = nullptr;
            VJ_HIP(e);
        }
        S.key = key;
    }

    int64_t cap[kSlots];
    // capacity: the caller's, else an estimate, at least what the slot's
    // output buffer already holds (a call that outgrew it grew it)
    for (int k = 0; k < kSlots; ++k)
        cap[k] = p.pair_capacity > 0
                     ? p.pair_capacity
                     : std::max<int64_t>({1 << 16, total_q * 64 / nsl,
                                          (int64_t)(jw.bslot[k].out_q.bytes / sizeof(int32_t))});
    std::vector<uint64_t> rec[kSlots];
    for (int k = 0; k < nsl; ++k) rec[k].assign(desc[k].size() * kBatchRec, 0);
    for (int attempt = 0; attempt < 4; ++attempt) {
        for (int k = 0; k < nsl; ++k) {
            BatchSlot &S = jw.bslot[k];
            int32_t *ctr = S.counters.as<int32_t>();
            S.out_q.reserve((size_t)cap[k] * sizeof(int32_t));
            S.out_x.reserve((size_t)cap[k] * sizeof(int32_t));
            S.out_d.reserve((size_t)cap[k] * sizeof(float));
            JoinArgs *args_h = reinterpret_cast<JoinArgs *>(static_cast<char *>(jw.pinned) + 256 + 1024 * k);
            JoinArgs a = make_args(ix, prec, p, beam, 0.f, nullptr, ctr);
            a.out_q = S.out_q.as<int32_t>();
            a.out_x = S.out_x.as<int32_t>();
            a.out_d = S.out_d.as<float>();
            a.cap = cap[k];
            a.stats = stats->as<int32_t>();
            *args_h = a;
            VJ_HIP(hipMemcpyAsync(S.args.p, args_h, sizeof(a), hipMemcpyHostToDevice, s));
            VJ_HIP(hipMemcpyAsync(S.desc.p, desc[k].data(), desc[k].size() * sizeof(BatchDesc),
                                  hipMemcpyHostToDevice, s));
            VJ_HIP(hipMemsetAsync(ctr, 0, 64, s));  // the cursor starts at the slot's first batch
            if (dense) VJ_HIP(hipMemsetAsync(L[k].hist, 0, kOrderBuckets * sizeof(uint32_t), s));
            else iota_i32(L[k].lp1, nmax, s);
        }
        VJ_HIP(hipEventRecord(jw.bev[0], s));
        for (int k = 0; k < nsl; ++k) VJ_HIP(hipStreamWaitEvent(jw.bslot[k].stream, jw.bev[0], 0));
        // alternate the slots' submissions so that both start early
        for (int i = 0; i < std::max(launches[0], launches[1]); ++i)
            for (int k = 0; k < nsl; ++k) {
                if (i >= launches[k]) continue;
                if (graph) VJ_HIP(hipGraphLaunch(jw.bslot[k].exec, jw.bslot[k].stream));
                else enqueue_step(k, jw.bslot[k].stream);
            }
        VJ_HIP(hipGetLastError());
        for (int k = 0; k < nsl; ++k) {
            VJ_HIP(hipEventRecord(jw.bev[1 + k], jw.bslot[k].stream));
            VJ_HIP(hipStreamWaitEvent(s, jw.bev[1 + k], 0));
        }
        std::memset(hctr, 0, 64 * kSlots);
        for (int k = 0; k < nsl; ++k) {
            VJ_HIP(hipMemcpyAsync(hctr + 16 * k, jw.bslot[k].counters.p, 64, hipMemcpyDeviceToHost, s));
            VJ_HIP(hipMemcpyAsync(rec[k].data(), jw.bslot[k].rec.p, rec[k].size() * sizeof(uint64_t),
                                  hipMemcpyDeviceToHost, s));
        }
        VJ_HIP(hipStreamSynchronize(s));
        int64_t tot[kSlots] = {0, 0};
        bool fits = true;
        for (int k = 0; k < nsl; ++k) {
            const int32_t *hc = hctr + 16 * k;
            VJ_CHECK(!(hc[3] & 8), VJ_ERR_INVALID_ARG, "query id out of range");
            VJ_CHECK(!(hc[3] & 16), VJ_ERR_INTERNAL, "visited-set probe exceeded the table size");
            VJ_CHECK(!(hc[3] & 32), VJ_ERR_INTERNAL, "a worklist entry is not a data node id");
            VJ_CHECK(!(hc[3] & 64), VJ_ERR_INTERNAL, "join tiers exhausted");
            VJ_CHECK(!(hc[3] & 128), VJ_ERR_INTERNAL, "a join wave waited past its bound");
            VJ_CHECK(hc[kBatchCursor] == (int32_t)desc[k].size(), VJ_ERR_INTERNAL,
                     "batch replays incomplete");
            tot[k] = (int64_t)(((uint64_t)(uint32_t)hc[1] << 32) | (uint32_t)hc[0]);
            if (tot[k] > cap[k]) {
                fits = false;
                cap[k] = tot[k] + tot[k] / 16 + 1024;
            }
        }
        if (!fits) continue;
        // one block for the pairs of every batch: q, x and dist arrays, the
        // pairs of slot 0 then those of slot 1
        const int64_t total = tot[0] + tot[1];
        const int64_t base[kSlots] = {0, tot[0]};
        const size_t m = (size_t)std::max<int64_t>(total, 1);
        auto block = std::make_shared<DevBuf>(m * (2 * sizeof(int32_t) + sizeof(float)));
        for (int k = 0; k < nsl; ++k) {
            if (tot[k] == 0) continue;
            const BatchSlot &S = jw.bslot[k];
            VJ_HIP(hipMemcpyAsync(block->as<int32_t>() + base[k], S.out_q.p, tot[k] * sizeof(int32_t),
                                  hipMemcpyDeviceToDevice, s));
            VJ_HIP(hipMemcpyAsync(block->as<int32_t>() + m + base[k], S.out_x.p,
                                  tot[k] * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
            VJ_HIP(hipMemcpyAsync(block->as<float>() + 2 * m + base[k], S.out_d.p,
                                  tot[k] * sizeof(float), hipMemcpyDeviceToDevice, s));
        }
        VJ_HIP(hipStreamSynchronize(s));
        make_results(block, total, base, rec);
        return;
    }
    VJ_CHECK(false, VJ_ERR_INTERNAL, "result capacity did not converge");
}

}  // namespace vj

// =================================================================== C ABI ==

using namespace vj;

#define API_BEGIN try {
#define API_END                                                                    \
    }                                                                              \
    catch (const vj::Error &e) {                                                   \
        vj::set_error(e.msg);                                                      \
        return e.st;                                                               \
    }                                                                              \
    catch (const std::bad_alloc &) {                                               \
        vj::set_error("host allocation failed");                                   \
        return VJ_ERR_OOM;                                                         \
    }                                                                              \
    catch (...) {                                                                  \
        vj::set_error("unexpected exception");                                     \
        return VJ_ERR_INTERNAL;                                                    \
    }                                                                              \
    vj::set_error("");                                                             \
    return VJ_OK;

extern "C" {

void vj_default_build_params(vj_build_params *p) {
    if (!p) return;
    p->R = 32;
    p->K_cand = 0;
    p->build_mst = 1;
    p->copies = 0;
}

void vj_default_join_params(vj_join_params *p) {
    if (!p) return;
    p->work_sharing = VJ_WS_SELF;
    p->hybrid = VJ_HYB_OFF;
    p->hybrid_beam = 256;
    p->conv_threshold = 10;
    p->ood_ratio = 1.5f;
    p->precision = VJ_PREC_FP32;
    p->budget = nullptr;
    p->start_tier = 1;
    p->coop_tables = 0;
    p->dense_first = 1;
    p->pair_capacity = 0;
    p->greedy_beam = 256;
    p->persistent = 0;
    p->layer_seeds = 0;
}

const char *vj_last_error(void) { return vj::last_error(); }

vj_status vj_trim_memory(int64_t *bytes_freed) {
    API_BEGIN
    const size_t n = vj::trim_block_cache();
    if (bytes_freed) *bytes_freed = (int64_t)n;
    API_END
}

vj_status vj_calib_gather(const float *rows, int64_t nrows, int32_t dp, const int32_t *ids,
                          int64_t n, float *out, void *stream) {
    API_BEGIN
    VJ_CHECK(n >= 0 && nrows >= 0, VJ_ERR_INVALID_ARG, "n and nrows must be >= 0");
    VJ_CHECK(dp > 0 && dp % 32 == 0, VJ_ERR_INVALID_ARG, "dp must be a positive multiple of 32");
    VJ_CHECK(n == 0 || (rows && ids && out), VJ_ERR_INVALID_ARG, "null pointer");
    calib_gather(rows, nrows, dp, ids, n, out, (hipStream_t)stream);
    API_END
}

// output k (k >= 1) of SplitMix64 seeded with `seed` (Steele, Lea and Flood 2014)
static uint64_t splitmix64_at(uint64_t seed, uint64_t k) {
    uint64_t z = seed + k * 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

vj_status vj_index_build_layers(vj_index *idx, int32_t R, uint64_t seed, int32_t max_levels,
                                void *stream) {
    API_BEGIN
    VJ_CHECK(idx != nullptr, VJ_ERR_INVALID_ARG, "null index");
    VJ_CHECK(R >= 1 && R <= 64, VJ_ERR_INVALID_ARG, "R must be in [1, 64]");
    VJ_CHECK(max_levels >= 1 && max_levels <= 16, VJ_ERR_INVALID_ARG, "max_levels in [1, 16]");
    Index &ix = idx->impl;
    hipStream_t s = (hipStream_t)stream;
    const int64_t nx = ix.nx;
    // levels: trailing zero 4-bit digits of each data node's output
    std::vector<int> lvl((size_t)nx);
    for (int64_t v = 0; v < nx; ++v) {
        uint64_t z = splitmix64_at(seed, (uint64_t)v + 1);
        int l = 0;
        while (l < max_levels && (z & 15u) == 0) { ++l; z >>= 4; }
        lvl[(size_t)v] = l;
    }
    std::vector<std::vector<int32_t>> sets;
    for (int l = 1; l <= max_levels; ++l) {
        std::vector<int32_t> sel;
        for (int64_t v = 0; v < nx; ++v)
            if (lvl[(size_t)v] >= l) sel.push_back((int32_t)v);
        if (sel.size() < 2) break;
        sets.push_back(std::move(sel));
    }
    const int nl = (int)sets.size();
    ix.lay_n = 0;
    ix.lay_R = R;
    ix.lay_off.assign((size_t)nl, 0);
    ix.lay_cnt.assign((size_t)nl, 0);
    ix.lay_entry.assign((size_t)nl, 0);
    int64_t total = 0;
    for (int j = 0; j < nl; ++j) {
        ix.lay_off[(size_t)j] = total;
        ix.lay_cnt[(size_t)j] = (int64_t)sets[(size_t)j].size();
        total += ix.lay_cnt[(size_t)j];
    }
    if (nl > 0) {
        ix.lay_adj.alloc((size_t)total * R * sizeof(int32_t));
        ix.lay_ids.alloc((size_t)total * sizeof(int32_t));
        ix.lay_pos.alloc((size_t)nl * nx * sizeof(int32_t));
        fill_i32(ix.lay_pos.as<int32_t>(), nl * nx, -1, s);
        const int kc = std::min(2 * R, 112);
        for (int j = 0; j < nl; ++j) {
            const int64_t n = ix.lay_cnt[(size_t)j];
            int32_t *ids = ix.lay_ids.as<int32_t>() + ix.lay_off[(size_t)j];
            VJ_HIP(hipMemcpyAsync(ids, sets[(size_t)j].data(), (size_t)n * sizeof(int32_t),
                                  hipMemcpyHostToDevice, s));
            Index part;
            part.nq = 0; part.nx = n; part.N = n; part.d = ix.d; part.dp = ix.dp; part.R = R;
            part.metric = ix.metric;
            part.vec.alloc((size_t)n * ix.dp * sizeof(float));
            gather_rows_f32(ix.vec.as<float>(), ix.dp, ids, n, part.vec.as<float>(), s);
            build_graph(part, (int)std::min<int64_t>(kc, n - 1), s);
            int32_t *dst = ix.lay_adj.as<int32_t>() + ix.lay_off[(size_t)j] * R;
            VJ_HIP(hipMemcpyAsync(dst, part.adj.p, (size_t)n * R * sizeof(int32_t),
                                  hipMemcpyDeviceToDevice, s));
            map_ids(dst, n * R, ids, s);
            scatter_pos(ix.lay_pos.as<int32_t>() + (int64_t)j * nx, ids, n, s);
            ix.lay_entry[(size_t)j] = sets[(size_t)j][(size_t)part.entry];
            VJ_HIP(hipStreamSynchronize(s));
        }
        std::vector<int64_t> oc(ix.lay_off);
        oc.insert(oc.end(), ix.lay_cnt.begin(), ix.lay_cnt.end());
        ix.lay_offd.alloc(oc.size() * sizeof(int64_t));
        VJ_HIP(hipMemcpyAsync(ix.lay_offd.p, oc.data(), oc.size() * sizeof(int64_t),
                              hipMemcpyHostToDevice, s));
        ix.lay_seed.alloc((size_t)std::max<int64_t>(ix.nq, 1) * sizeof(int32_t));
        fill_i32(ix.lay_seed.as<int32_t>(), std::max<int64_t>(ix.nq, 1), ix.entry, s);
    }
    VJ_HIP(hipStreamSynchronize(s));
    ix.lay_n = nl;
    API_END
}

vj_status vj_index_layers_info(const vj_index *idx, int32_t *n_layers, int32_t *R,
                               int64_t *counts, int32_t *entries) {
    API_BEGIN
    VJ_CHECK(idx != nullptr && n_layers != nullptr, VJ_ERR_INVALID_ARG, "null pointer");
    const Index &ix = idx->impl;
    *n_layers = ix.lay_n;
    if (R) *R = ix.lay_R;
    for (int j = 0; j < ix.lay_n; ++j) {
        if (counts) counts[j] = ix.lay_cnt[(size_t)j];
        if (entries) entries[j] = ix.lay_entry[(size_t)j];
    }
    API_END
}

vj_status vj_index_export_layer(const vj_index *idx, int32_t layer, int32_t *ids, int32_t *adj,
                                void *stream) {
    API_BEGIN
    VJ_CHECK(idx != nullptr, VJ_ERR_INVALID_ARG, "null index");
    const Index &ix = idx->impl;
    VJ_CHECK(layer >= 1 && layer <= ix.lay_n, VJ_ERR_INVALID_ARG, "no such layer");
    hipStream_t s = (hipStream_t)stream;
    const int64_t off = ix.lay_off[(size_t)layer - 1], n = ix.lay_cnt[(size_t)layer - 1];
    if (ids)
        VJ_HIP(hipMemcpyAsync(ids, ix.lay_ids.as<int32_t>() + off, (size_t)n * sizeof(int32_t),
                              hipMemcpyDeviceToDevice, s));
    if (adj)
        VJ_HIP(hipMemcpyAsync(adj, ix.lay_adj.as<int32_t>() + off * ix.lay_R,
                              (size_t)n * ix.lay_R * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    VJ_HIP(hipStreamSynchronize(s));
    API_END
}

vj_status vj_index_descend(vj_index *idx, const int32_t *query_ids, int64_t n, int32_t *seeds,
                           int32_t *moves, void *stream) {
    API_BEGIN
    VJ_CHECK(idx != nullptr && seeds != nullptr, VJ_ERR_INVALID_ARG, "null pointer");
    Index &ix = idx->impl;
    VJ_CHECK(ix.lay_n > 0, VJ_ERR_INVALID_ARG, "the index has no upper layers");
    VJ_CHECK(n >= 0 && (query_ids != nullptr || n == ix.nq), VJ_ERR_INVALID_ARG,
             "n must be nq when query_ids is null");
    if (query_ids != nullptr && n > 0) {
        std::vector<int32_t> h((size_t)n);
        VJ_HIP(hipMemcpy(h.data(), query_ids, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToHost));
        for (int32_t q : h) VJ_CHECK(q >= 0 && q < ix.nq, VJ_ERR_INVALID_ARG, "query id out of range");
    }
    layer_seeds(ix, query_ids, n, seeds, moves, (hipStream_t)stream);
    API_END
}

}  // extern "C"

namespace vj {
// An index around a graph built elsewhere.  separate: adj rows 0..nx-1 are a
// data graph over data ids only, rows nx.. a query graph over query node ids
// only, and the entry is a data node.
static void index_from_graph(const float *Q, int64_t nq, const float *X, int64_t nx, int32_t d,
                             vj_metric metric, const int32_t *adj, int32_t R, int32_t entry,
                             const int32_t *parent, bool separate, hipStream_t s, Index &ix) {
    VJ_CHECK(adj != nullptr, VJ_ERR_INVALID_ARG, "null pointer");
    check_shape(Q, nq, X, nx, d);
    check_index_size(nq, nx);
    VJ_CHECK(metric == VJ_L2 || metric == VJ_IP, VJ_ERR_INVALID_ARG, "unknown metric");
    VJ_CHECK(R >= 1 && R <= 64, VJ_ERR_UNSUPPORTED, "R must be in [1, 64]");
    VJ_CHECK(entry >= 0 && entry < (separate ? nx : nq + nx), VJ_ERR_INVALID_ARG,
             separate ? "the entry of separate indexes is a data node" : "entry out of range");
    ix.nq = nq; ix.nx = nx; ix.N = nq + nx; ix.d = d; ix.dp = padded_dim(d); ix.R = R;
    ix.entry = entry; ix.metric = metric; ix.separate = separate;
    VJ_HIP(hipGetDevice(&ix.device));
    init_vectors(ix, Q, X, s);
    ix.adj.alloc((size_t)ix.N * R * sizeof(int32_t));
    VJ_HIP(hipMemcpyAsync(ix.adj.p, adj, ix.adj.bytes, hipMemcpyDeviceToDevice, s));
    // every id must be -1 or a node id (separate: of the row's own set)
    std::vector<int32_t> ah((size_t)ix.N * R);
    VJ_HIP(hipMemcpyAsync(ah.data(), adj, ah.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    VJ_HIP(hipStreamSynchronize(s));
    for (size_t e = 0; e < ah.size(); ++e) {
        const int32_t v = ah[e];
        VJ_CHECK(v >= -1 && v < ix.N, VJ_ERR_INVALID_ARG, "adjacency id out of range");
        if (separate && v >= 0) {
            const bool data_row = (int64_t)(e / R) < nx;
            VJ_CHECK(data_row == (v < nx), VJ_ERR_INVALID_ARG,
                     "separate indexes: a data row may only hold data ids and a query row "
                     "only query node ids");
        }
    }
    ix.elen.alloc((size_t)ix.N * R * sizeof(float));
    launch_edge_lengths(ix.vec.as<float>(), ix.dp, ix.adj.as<int32_t>(), ix.N, R, ix.elen.as<float>(), s);
    if (parent) set_parents(ix, parent, s);
    else compute_mst(ix, s);
    VJ_HIP(hipStreamSynchronize(s));
}

// The graph of rows [first, first + n) of ix's vectors, built by the merged
// build's recipe over that set alone, into rows [first, first + n) of
// ix.adj with node ids offset by `first`.
static void build_part(Index &ix, int64_t first, int64_t n, int kc, hipStream_t s, int32_t *entry,
                       int64_t *repairs) {
    if (n < 2) {
        fill_i32(ix.adj.as<int32_t>() + (size_t)first * ix.R, n * ix.R, -1, s);
        *entry = (int32_t)first;
        return;
    }
    Index part;
    part.nq = 0; part.nx = n; part.N = n; part.d = ix.d; part.dp = ix.dp; part.R = ix.R;
    part.metric = ix.metric;
    part.vec = DevBuf::view(ix.vec.as<float>() + (size_t)first * ix.dp, (size_t)n * ix.dp * sizeof(float));
    build_graph(part, (int)std::min<int64_t>(kc, n - 1), s);
    int32_t *dst = ix.adj.as<int32_t>() + (size_t)first * ix.R;
    VJ_HIP(hipMemcpyAsync(dst, part.adj.p, (size_t)n * ix.R * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    if (first) offset_ids(dst, n * ix.R, (int32_t)first, s);
    VJ_HIP(hipStreamSynchronize(s));
    *entry = (int32_t)(part.entry + first);
    *repairs += part.repairs;
}
}  // namespace vj

extern "C" {

vj_status vj_index_from_graph(const float *Q, int64_t nq, const float *X, int64_t nx, int32_t d,
                              vj_metric metric, const int32_t *adj, int32_t R, int32_t entry,
                              const int32_t *parent, void *stream, vj_index **out) {
    API_BEGIN
    VJ_CHECK(out != nullptr, VJ_ERR_INVALID_ARG, "null pointer");
    auto h = std::make_unique<vj_index>();
    index_from_graph(Q, nq, X, nx, d, metric, adj, R, entry, parent, false, (hipStream_t)stream,
                     h->impl);
    *out = h.release();
    API_END
}

vj_status vj_index_from_separate_graphs(const float *Q, int64_t nq, const float *X, int64_t nx,
                                        int32_t d, vj_metric metric, const int32_t *adj, int32_t R,
                                        int32_t entry, const int32_t *parent, void *stream,
                                        vj_index **out) {
    API_BEGIN
    VJ_CHECK(out != nullptr, VJ_ERR_INVALID_ARG, "null pointer");
    auto h = std::make_unique<vj_index>();
    index_from_graph(Q, nq, X, nx, d, metric, adj, R, entry, parent, true, (hipStream_t)stream,
                     h->impl);
    *out = h.release();
    API_END
}

vj_status vj_build_separate_index(const float *Q, int64_t nq, const float *X, int64_t nx,
                                  int32_t d, vj_metric metric, const vj_build_params *bp,
                                  void *stream, vj_index **out) {
    API_BEGIN
    VJ_CHECK(out != nullptr, VJ_ERR_INVALID_ARG, "null pointer");
    check_shape(Q, nq, X, nx, d);
    check_index_size(nq, nx);
    VJ_CHECK(nx >= 2, VJ_ERR_INVALID_ARG, "the data graph needs nx >= 2");
    VJ_CHECK(metric == VJ_L2 || metric == VJ_IP, VJ_ERR_INVALID_ARG, "unknown metric");
    vj_build_params p;
    vj_default_build_params(&p);
    if (bp) p = *bp;
    VJ_CHECK(p.R >= 1 && p.R <= 64, VJ_ERR_UNSUPPORTED, "R must be in [1, 64]");
    const int kc = p.K_cand > 0 ? p.K_cand : std::min(2 * p.R, 112);
    VJ_CHECK(kc >= 1 && kc <= 112, VJ_ERR_UNSUPPORTED, "K_cand must be in [1, 112]");
    hipStream_t s = (hipStream_t)stream;
    auto h = std::make_unique<vj_index>();
    Index &ix = h->impl;
    ix.nq = nq; ix.nx = nx; ix.N = nq + nx; ix.d = d; ix.dp = padded_dim(d); ix.R = p.R;
    ix.metric = metric;
    ix.separate = true;
    VJ_HIP(hipGetDevice(&ix.device));
    init_vectors(ix, Q, X, s);
    ix.adj.alloc((size_t)ix.N * ix.R * sizeof(int32_t));
    int32_t ex = 0, eq = 0;
    build_part(ix, 0, nx, kc, s, &ex, &ix.repairs);
    build_part(ix, nx, nq, kc, s, &eq, &ix.repairs);
    ix.entry = ex;
    ix.elen.alloc((size_t)ix.N * ix.R * sizeof(float));
    launch_edge_lengths(ix.vec.as<float>(), ix.dp, ix.adj.as<int32_t>(), ix.N, ix.R,
                        ix.elen.as<float>(), s);
    if (p.copies & 1) ensure_bf16(ix, s);
    if (p.copies & 2) ensure_f8(ix, s);
    if (p.build_mst) compute_mst(ix, s);
    VJ_HIP(hipStreamSynchronize(s));
    *out = h.release();
    API_END
}

vj_status vj_build_merged_index(const float *Q, int64_t nq, const float *X, int64_t nx, int32_t d,
                                vj_metric metric, const vj_build_params *bp, void *stream,
                                vj_index **out) {
    API_BEGIN
    VJ_CHECK(out != nullptr, VJ_ERR_INVALID_ARG, "null pointer");
    check_shape(Q, nq, X, nx, d);
    check_index_size(nq, nx);
    VJ_CHECK(metric == VJ_L2 || metric == VJ_IP, VJ_ERR_INVALID_ARG, "unknown metric");
    vj_build_params p;
    vj_default_build_params(&p);
    if (bp) p = *bp;
    VJ_CHECK(p.R >= 1 && p.R <= 64, VJ_ERR_UNSUPPORTED, "R must be in [1, 64]");
    const int kc = p.K_cand > 0 ? p.K_cand : std::min(2 * p.R, 112);
    VJ_CHECK(kc >= 1 && kc <= 112, VJ_ERR_UNSUPPORTED, "K_cand must be in [1, 112]");
    hipStream_t s = (hipStream_t)stream;
    auto h = std::make_unique<vj_index>();
    Index &ix = h->impl;
    ix.nq = nq; ix.nx = nx; ix.N = nq + nx; ix.d = d; ix.dp = padded_dim(d); ix.R = p.R;
    ix.metric = metric;
    VJ_HIP(hipGetDevice(&ix.device));
    init_vectors(ix, Q, X, s);
    build_graph(ix, (int)std::min<int64_t>(kc, ix.N - 1), s);
    if (p.copies & 1) ensure_bf16(ix, s);
    if (p.copies & 2) ensure_f8(ix, s);
    if (p.build_mst) compute_mst(ix, s);
    VJ_HIP(hipStreamSynchronize(s));
    *out = h.release();
    API_END
}

vj_status vj_index_swap_roles(const vj_index *idx, int32_t build_mst, void *stream,
                              vj_index **out) {
    API_BEGIN
    VJ_CHECK(idx != nullptr && out != nullptr, VJ_ERR_INVALID_ARG, "null pointer");
    const Index &a = idx->impl;
    VJ_CHECK(!a.separate, VJ_ERR_INVALID_ARG, "the role switch is defined on a merged index");
    VJ_CHECK(a.nq >= 1, VJ_ERR_INVALID_ARG, "the role switch needs at least one query");
    hipStream_t s = (hipStream_t)stream;
    auto h = std::make_unique<vj_index>();
    Index &b = h->impl;
    b.nq = a.nx; b.nx = a.nq; b.N = a.N; b.d = a.d; b.dp = a.dp; b.R = a.R;
    b.metric = a.metric;
    b.entry = a.entry < a.nx ? a.entry + (int32_t)a.nq : a.entry - (int32_t)a.nx;
    b.repairs = a.repairs;
    VJ_HIP(hipGetDevice(&b.device));
    // the old query rows come first, then the old data rows
    const size_t rq = (size_t)a.nq, rx = (size_t)a.nx;
    b.vec.alloc((size_t)b.N * b.dp * sizeof(float));
    const size_t vrow = (size_t)a.dp * sizeof(float), arow = (size_t)a.R * sizeof(int32_t);
    VJ_HIP(hipMemcpyAsync(b.vec.p, a.vec.as<char>() + rx * vrow, rq * vrow, hipMemcpyDeviceToDevice, s));
    VJ_HIP(hipMemcpyAsync(b.vec.as<char>() + rq * vrow, a.vec.p, rx * vrow, hipMemcpyDeviceToDevice, s));
    b.adj.alloc((size_t)b.N * arow);
    VJ_HIP(hipMemcpyAsync(b.adj.p, a.adj.as<char>() + rx * arow, rq * arow, hipMemcpyDeviceToDevice, s));
    VJ_HIP(hipMemcpyAsync(b.adj.as<char>() + rq * arow, a.adj.p, rx * arow, hipMemcpyDeviceToDevice, s));
    swap_ids(b.adj.as<int32_t>(), b.N * b.R, (int32_t)a.nx, (int32_t)a.nq, s);
    b.elen.alloc((size_t)b.N * b.R * sizeof(float));
    VJ_HIP(hipMemcpyAsync(b.elen.p, a.elen.as<char>() + rx * arow, rq * arow, hipMemcpyDeviceToDevice, s));
    VJ_HIP(hipMemcpyAsync(b.elen.as<char>() + rq * arow, a.elen.p, rx * arow, hipMemcpyDeviceToDevice, s));
    finish_vectors(b, s);
    if (build_mst) compute_mst(b, s);
    VJ_HIP(hipStreamSynchronize(s));
    *out = h.release();
    API_END
}

vj_status vj_index_insert_queries(vj_index *idx, const float *Q, int64_t n, int32_t K_cand,
                                  void *stream) {
    API_BEGIN
    VJ_CHECK(idx != nullptr, VJ_ERR_INVALID_ARG, "null index");
    Index &ix = idx->impl;
    VJ_CHECK(!ix.separate, VJ_ERR_UNSUPPORTED, "insertion is defined on merged indexes");
    VJ_CHECK(n >= 0, VJ_ERR_INVALID_ARG, "n must be >= 0");
    if (n == 0) return VJ_OK;
    VJ_CHECK(Q != nullptr, VJ_ERR_INVALID_ARG, "null vector pointer");
    check_index_size(ix.nq + n, ix.nx);
    const int kc = K_cand > 0 ? K_cand : std::min(2 * ix.R, 112);
    VJ_CHECK(kc >= 1 && kc <= 112, VJ_ERR_UNSUPPORTED, "K_cand must be in [1, 112]");
    hipStream_t s = (hipStream_t)stream;
    const int64_t n_old = ix.N, N = n_old + n;
    const size_t R = (size_t)ix.R, dp = (size_t)ix.dp;
    // the grown graph is built beside the old one and swapped in at the end
    Index b;
    b.nq = ix.nq + n; b.nx = ix.nx; b.N = N; b.d = ix.d; b.dp = ix.dp; b.R = ix.R;
    b.entry = ix.entry; b.metric = ix.metric; b.device = ix.device;
    b.vec.alloc((size_t)N * dp * sizeof(float));
    VJ_HIP(hipMemcpyAsync(b.vec.p, ix.vec.p, (size_t)n_old * dp * sizeof(float),
                          hipMemcpyDeviceToDevice, s));
    launch_pad_rows(Q, n, ix.d, b.vec.as<float>() + (size_t)n_old * dp, ix.dp, s);
    b.adj.alloc((size_t)N * R * sizeof(int32_t));
    VJ_HIP(hipMemcpyAsync(b.adj.p, ix.adj.p, (size_t)n_old * R * sizeof(int32_t),
                          hipMemcpyDeviceToDevice, s));
    fill_i32(b.adj.as<int32_t>() + (size_t)n_old * R, n * (int64_t)R, -1, s);
    b.elen.alloc((size_t)N * R * sizeof(float));
    VJ_HIP(hipMemcpyAsync(b.elen.p, ix.elen.p, (size_t)n_old * R * sizeof(float),
                          hipMemcpyDeviceToDevice, s));
    // the kNN sweep's group centres, labels of the old nodes and radii go
    // with the graph (on an error they are dropped, and the next insertion
    // labels every node)
    b.piv_rows = std::move(ix.piv_rows);
    b.piv_of = std::move(ix.piv_of);
    b.piv_rad = std::move(ix.piv_rad);
    b.piv_n = ix.piv_n;
    b.piv_cnt = ix.piv_cnt;
    ix.piv_n = 0;
    ix.piv_cnt = 0;
    // so do the kNN lists kept for the repair
    b.knn_id = std::move(ix.knn_id);
    b.knn_d2 = std::move(ix.knn_d2);
    b.knn_cert = std::move(ix.knn_cert);
    b.knn_from = std::move(ix.knn_from);
    b.knn_kc = ix.knn_kc;
    b.knn_rows = ix.knn_rows;
    b.knn_cap = ix.knn_cap;
    ix.knn_rows = ix.knn_cap = 0;
    insert_graph(b, n_old, kc, s);
    // swap in, then the derived state
    ix.vec = std::move(b.vec);
    ix.adj = std::move(b.adj);
    ix.elen = std::move(b.elen);
    ix.piv_rows = std::move(b.piv_rows);
    ix.piv_of = std::move(b.piv_of);
    ix.piv_rad = std::move(b.piv_rad);
    ix.piv_n = b.piv_n;
    ix.piv_cnt = b.piv_cnt;
    ix.knn_id = std::move(b.knn_id);
    ix.knn_d2 = std::move(b.knn_d2);
    ix.knn_cert = std::move(b.knn_cert);
    ix.knn_from = std::move(b.knn_from);
    ix.knn_kc = b.knn_kc;
    ix.knn_rows = b.knn_rows;
    ix.knn_cap = b.knn_cap;
    ix.nq = b.nq;
    ix.N = N;
    ix.repairs += b.repairs;
    for (int k = 0; k < 3; ++k) ix.knn_tiles[k] = b.knn_tiles[k];
    ix.last_repairs = b.last_repairs;
    ix.last_listed = b.last_listed;
    const bool had_bf16 = ix.vec_bf16.p != nullptr, had_f8 = ix.vec_f8.p != nullptr;
    ix.vec_bf16.release();
    ix.vec_f8.release();
    ix.f8meta.release();
    finish_vectors(ix, s);
    if (had_bf16) ensure_bf16(ix, s);
    if (had_f8) ensure_f8(ix, s);
    if (ix.has_mst) compute_mst(ix, s);
    VJ_HIP(hipStreamSynchronize(s));
    API_END
}

vj_status vj_build_nnmap(vj_index *idx, float ood_ratio, void *stream) {
    API_BEGIN
    VJ_CHECK(idx != nullptr, VJ_ERR_INVALID_ARG, "null index");
    Index &ix = idx->impl;
    VJ_CHECK(ix.separate, VJ_ERR_INVALID_ARG, "an NN-Map is built on separate indexes");
    VJ_CHECK(std::isfinite(ood_ratio) && ood_ratio > 0.f, VJ_ERR_INVALID_ARG, "ood_ratio > 0");
    hipStream_t s = (hipStream_t)stream;
    const size_t nq = (size_t)std::max<int64_t>(ix.nq, 1);
    ix.nn_w.alloc(nq * sizeof(int32_t));
    ix.nn_d.alloc(nq * sizeof(double));
    ix.nn_ood.alloc(nq);
    const float *vec = ix.vec.as<float>();
    exact_top1(vec + (size_t)ix.nx * ix.dp, ix.nq, vec, ix.nx, ix.dp, ix.metric,
               ix.nn_w.as<int32_t>(), ix.nn_d.as<double>(), s);
    nn_ood(vec, ix.dp, ix.nx, ix.nq, ix.adj.as<int32_t>(), ix.R, ix.nn_w.as<int32_t>(),
           (double)ood_ratio, ix.nn_ood.as<uint8_t>(), s);
    VJ_HIP(hipStreamSynchronize(s));
    ix.has_nnmap = true;
    API_END
}

vj_status vj_index_export_nnmap(const vj_index *idx, int32_t *w, double *dist, uint8_t *ood,
                                void *stream) {
    API_BEGIN
    VJ_CHECK(idx != nullptr, VJ_ERR_INVALID_ARG, "null index");
    const Index &ix = idx->impl;
    VJ_CHECK(ix.has_nnmap, VJ_ERR_INVALID_ARG, "the index has no NN-Map");
    hipStream_t s = (hipStream_t)stream;
    if (w) VJ_HIP(hipMemcpyAsync(w, ix.nn_w.p, (size_t)ix.nq * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    if (dist) VJ_HIP(hipMemcpyAsync(dist, ix.nn_d.p, (size_t)ix.nq * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (ood) VJ_HIP(hipMemcpyAsync(ood, ix.nn_ood.p, (size_t)ix.nq, hipMemcpyDeviceToDevice, s));
    VJ_HIP(hipStreamSynchronize(s));
    API_END
}

vj_status vj_index_export_graph(const vj_index *idx, int32_t *adj, float *elen, int32_t *parent,
                                void *stream) {
    API_BEGIN
    VJ_CHECK(idx != nullptr, VJ_ERR_INVALID_ARG, "null index");
    const Index &ix = idx->impl;
    hipStream_t s = (hipStream_t)stream;
    if (adj) VJ_HIP(hipMemcpyAsync(adj, ix.adj.p, (size_t)ix.N * ix.R * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    if (elen) VJ_HIP(hipMemcpyAsync(elen, ix.elen.p, (size_t)ix.N * ix.R * sizeof(float), hipMemcpyDeviceToDevice, s));
    if (parent) {
        VJ_CHECK(ix.has_mst, VJ_ERR_INVALID_ARG, "index has no MST");
        VJ_HIP(hipMemcpyAsync(parent, ix.parent.p, (size_t)ix.nq * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    }
    VJ_HIP(hipStreamSynchronize(s));
    API_END
}

vj_status vj_index_info(const vj_index *idx, int64_t *nq, int64_t *nx, int32_t *d, int32_t *R,
                        int32_t *entry, int32_t *metric) {
    API_BEGIN
    VJ_CHECK(idx != nullptr, VJ_ERR_INVALID_ARG, "null index");
    const Index &ix = idx->impl;
    if (nq) *nq = ix.nq;
    if (nx) *nx = ix.nx;
    if (d) *d = ix.d;
    if (R) *R = ix.R;
    if (entry) *entry = ix.entry;
    if (metric) *metric = ix.metric;
    API_END
}

vj_status vj_index_build_stats(const vj_index *idx, int64_t *tiles_first, int64_t *tiles_second,
                               int64_t *tiles_all, int64_t *repairs, int64_t *repairs_listed) {
    API_BEGIN
    VJ_CHECK(idx != nullptr, VJ_ERR_INVALID_ARG, "null index");
    const Index &ix = idx->impl;
    if (tiles_first) *tiles_first = ix.knn_tiles[0];
    if (tiles_second) *tiles_second = ix.knn_tiles[1];
    if (tiles_all) *tiles_all = ix.knn_tiles[2];
    if (repairs) *repairs = ix.last_repairs;
    if (repairs_listed) *repairs_listed = ix.last_listed;
    API_END
}

void vj_index_free(vj_index *idx) { delete idx; }

vj_status vj_index_save(const vj_index *idx, const char *path) {
    API_BEGIN
    VJ_CHECK(idx != nullptr && path != nullptr, VJ_ERR_INVALID_ARG, "null pointer");
    VJ_HIP(hipDeviceSynchronize());
    index_save(idx->impl, path);
    API_END
}

vj_status vj_index_load(const char *path, void *stream, vj_index **out) {
    API_BEGIN
    VJ_CHECK(path != nullptr && out != nullptr, VJ_ERR_INVALID_ARG, "null pointer");
    hipStream_t s = (hipStream_t)stream;
    auto h = std::make_unique<vj_index>();
    index_load(h->impl, path, finish_vectors, s);
    VJ_HIP(hipStreamSynchronize(s));
    *out = h.release();
    API_END
}

vj_status vj_join(vj_index *idx, const int32_t *query_ids, int64_t n, float eps, vj_metric metric,
                  const vj_join_params *pp, void *stream, vj_pairs **out) {
    API_BEGIN
    VJ_CHECK(idx != nullptr && out != nullptr, VJ_ERR_INVALID_ARG, "null pointer");
    Index &ix = idx->impl;
    VJ_CHECK(n >= 0, VJ_ERR_INVALID_ARG, "n must be >= 0");
    VJ_CHECK(query_ids != nullptr || n == ix.nq || n == 0, VJ_ERR_INVALID_ARG,
             "query_ids may be NULL only with n == nq or n == 0");
    VJ_CHECK(n < ((int64_t)1 << 31), VJ_ERR_UNSUPPORTED, "n must be < 2^31");
    VJ_CHECK(std::isfinite(eps), VJ_ERR_INVALID_ARG, "eps must be finite");
    VJ_CHECK(metric == ix.metric, VJ_ERR_METRIC_MISMATCH, "join metric differs from the index metric");
    vj_join_params p;
    vj_default_join_params(&p);
    if (pp) p = *pp;
    VJ_CHECK(p.work_sharing >= VJ_WS_SELF && p.work_sharing <= VJ_WS_NNMAP, VJ_ERR_INVALID_ARG, "work_sharing");
    VJ_CHECK(p.work_sharing != VJ_WS_NNMAP || (ix.separate && ix.has_nnmap), VJ_ERR_INVALID_ARG,
             "NN-Map joins need a separate index with an NN-Map (vj_build_nnmap)");
    VJ_CHECK(p.hybrid >= VJ_HYB_OFF && p.hybrid <= VJ_HYB_LEARNED, VJ_ERR_INVALID_ARG, "hybrid");
    VJ_CHECK(p.hybrid_beam >= 0 && p.hybrid_beam <= 4096, VJ_ERR_INVALID_ARG, "hybrid_beam in [0, 4096]");
    VJ_CHECK((p.work_sharing != VJ_WS_SOFT && p.work_sharing != VJ_WS_HARD) || ix.has_mst,
             VJ_ERR_INVALID_ARG, "work sharing needs the MST");
    VJ_CHECK(p.hybrid != VJ_HYB_BUDGET || p.budget != nullptr, VJ_ERR_INVALID_ARG, "budget mode needs budget[]");
    VJ_CHECK(p.start_tier >= 0 && p.start_tier <= 2, VJ_ERR_INVALID_ARG, "start_tier in [0, 2]");
    VJ_CHECK(p.coop_tables == 0 || p.coop_tables == 1, VJ_ERR_INVALID_ARG, "coop_tables is 0 or 1");
    VJ_CHECK(p.hybrid != VJ_HYB_LEARNED || ix.pred != nullptr, VJ_ERR_INVALID_ARG,
             "learned routing needs an attached predictor");
    VJ_CHECK(!ix.separate || p.hybrid != VJ_HYB_LEARNED, VJ_ERR_INVALID_ARG,
             "learned routing needs the merged index (its features come from the probe of q)");
    VJ_CHECK(p.greedy_beam >= 1 && p.greedy_beam <= 256, VJ_ERR_INVALID_ARG,
             "greedy_beam in [1, 256]");
    VJ_CHECK(p.layer_seeds == 0 || (ix.separate && ix.lay_n > 0), VJ_ERR_INVALID_ARG,
             "layer seeds need a separate index with upper layers (vj_index_build_layers)");
    // the persistent launch faulted the GPU once in soft work-sharing mode
    // and its cause is not established: it is switched off until it is
    VJ_CHECK(p.persistent == 0, VJ_ERR_UNSUPPORTED,
             "persistent launches are switched off (their GPU fault is under investigation)");
    hipStream_t s = (hipStream_t)stream;
    auto h = std::make_unique<vj_pairs>();
    Pairs &r = h->impl;
    r.n_queries = n;
    if (n == 0 || (metric == VJ_L2 && eps <= 0.0f)) {
        r.stats.alloc((size_t)std::max<int64_t>(n, 1) * 8 * sizeof(int32_t));
        VJ_HIP(hipMemsetAsync(r.stats.p, 0, r.stats.bytes, s));
        VJ_HIP(hipStreamSynchronize(s));
        r.count = 0;
        *out = h.release();
        vj::set_error("");
        return VJ_OK;
    }
    if (p.hybrid != VJ_HYB_LEARNED) run_join(ix, query_ids, n, eps, p, p.budget, s, r);
    else learned_join(ix, query_ids, n, eps, p, s, r);
    *out = h.release();
    API_END
}

vj_status vj_bruteforce_join(const float *Q, int64_t nq, const float *X, int64_t nx, int32_t d,
                             float eps, vj_metric metric, vj_precision prec, void *stream,
                             vj_pairs **out) {
    API_BEGIN
    VJ_CHECK(out != nullptr, VJ_ERR_INVALID_ARG, "null pointer");
    check_shape(Q, nq, X, nx, d);
    VJ_CHECK(std::isfinite(eps), VJ_ERR_INVALID_ARG, "eps must be finite");
    VJ_CHECK(metric == VJ_L2 || metric == VJ_IP, VJ_ERR_INVALID_ARG, "unknown metric");
    VJ_CHECK(prec == VJ_PREC_FP32 || prec == VJ_PREC_BF16, VJ_ERR_UNSUPPORTED,
             "brute force supports FP32 (split bf16) and BF16 tiles");
    hipStream_t s = (hipStream_t)stream;
    auto h = std::make_unique<vj_pairs>();
    bruteforce_join(Q, nq, X, nx, d, eps, metric, prec, s, h->impl);
    *out = h.release();
    API_END
}

vj_status vj_bruteforce_join_noalloc(const float *Q, int64_t nq, const float *X, int64_t nx,
                                     int32_t d, float eps, vj_metric metric, vj_precision prec,
                                     int32_t *qx, float *dist, int64_t cap, int64_t *count_host,
                                     void *stream) {
    API_BEGIN
    VJ_CHECK(count_host != nullptr && cap >= 0 && (cap == 0 || qx != nullptr), VJ_ERR_INVALID_ARG,
             "need count_host, cap >= 0 and qx when cap > 0");
    check_shape(Q, nq, X, nx, d);
    VJ_CHECK(std::isfinite(eps), VJ_ERR_INVALID_ARG, "eps must be finite");
    VJ_CHECK(metric == VJ_L2 || metric == VJ_IP, VJ_ERR_INVALID_ARG, "unknown metric");
    VJ_CHECK(prec == VJ_PREC_FP32 || prec == VJ_PREC_BF16, VJ_ERR_UNSUPPORTED,
             "brute force supports FP32 (split bf16) and BF16 tiles");
    *count_host = bruteforce_join_noalloc(Q, nq, X, nx, d, eps, metric, prec, qx, dist, cap,
                                          (hipStream_t)stream);
    API_END
}

int64_t vj_pairs_count(const vj_pairs *r) { return r ? r->impl.count : -1; }

vj_status vj_pairs_export(const vj_pairs *r, int32_t *qx, float *dist, int sorted, void *stream) {
    API_BEGIN
    VJ_CHECK(r != nullptr, VJ_ERR_INVALID_ARG, "null result");
    VJ_CHECK(qx != nullptr || r->impl.count == 0, VJ_ERR_INVALID_ARG, "null qx");
    hipStream_t s = (hipStream_t)stream;
    export_pairs(r->impl, qx, dist, sorted != 0, s);
    VJ_HIP(hipStreamSynchronize(s));
    API_END
}

vj_status vj_pairs_stats(const vj_pairs *r, int32_t *stats, void *stream) {
    API_BEGIN
    VJ_CHECK(r != nullptr && stats != nullptr, VJ_ERR_INVALID_ARG, "null pointer");
    VJ_CHECK(r->impl.n_queries > 0 && r->impl.stats.p, VJ_ERR_INVALID_ARG, "result has no per-query counters");
    hipStream_t s = (hipStream_t)stream;
    VJ_HIP(hipMemcpyAsync(stats, r->impl.stats.p, (size_t)r->impl.n_queries * 8 * sizeof(int32_t),
                          hipMemcpyDeviceToDevice, s));
    VJ_HIP(hipStreamSynchronize(s));
    API_END
}

vj_status vj_pairs_timing(const vj_pairs *r, float *kernel_ms, float *spill_ms,
                          int64_t *n_spilled) {
    API_BEGIN
    VJ_CHECK(r != nullptr, VJ_ERR_INVALID_ARG, "null result");
    if (kernel_ms) *kernel_ms = r->impl.kernel_ms;
    if (spill_ms) *spill_ms = r->impl.spill_ms;
    if (n_spilled) *n_spilled = r->impl.n_spilled;
    API_END
}

vj_status vj_pairs_rechecked(const vj_pairs *r, int64_t *n) {
    API_BEGIN
    VJ_CHECK(r != nullptr && n != nullptr, VJ_ERR_INVALID_ARG, "null argument");
    *n = r->impl.n_candidates;
    API_END
}

vj_status vj_pairs_tiers(const vj_pairs *r, float *ms, int32_t *launches, int64_t *queries) {
    API_BEGIN
    VJ_CHECK(r != nullptr, VJ_ERR_INVALID_ARG, "null result");
    for (int t = 0; t < 4; ++t) {
        if (ms) ms[t] = r->impl.tier_ms[t];
        if (launches) launches[t] = r->impl.tier_launches[t];
        if (queries) queries[t] = r->impl.tier_queries[t];
    }
    API_END
}

void vj_pairs_free(vj_pairs *r) { delete r; }

// ------------------------------------------------------- batches, tuning --

vj_status vj_join_batches(vj_index *idx, const int32_t *query_ids, const int64_t *batch_start_host,
                          const int64_t *batch_count_host, const float *eps_host,
                          int32_t n_batches, vj_metric metric, const vj_join_params *pp,
                          void *stream, vj_pairs **out, float *batch_ms_host) {
    API_BEGIN
    check_batches(idx, query_ids, batch_start_host, batch_count_host, eps_host, n_batches, out);
    std::vector<vj_pairs *> res((size_t)n_batches, nullptr);
    struct Guard {
        std::vector<vj_pairs *> &v;
        bool done = false;
        ~Guard() { if (!done) for (auto *r : v) delete r; }
    } guard{res};
    hipStream_t s = (hipStream_t)stream;
    std::vector<int32_t> iota_h;
    DevBuf ids_dev;
    for (int32_t b = 0; b < n_batches; ++b) {
        const auto t0 = std::chrono::steady_clock::now();
        const int64_t st = batch_start_host[b], ct = batch_count_host[b];
        const int32_t *ids = nullptr;
        if (query_ids) {
            ids = query_ids + st;
        } else if (ct > 0) {
            // the identity list of this range
            iota_h.resize((size_t)ct);
            for (int64_t i = 0; i < ct; ++i) iota_h[(size_t)i] = (int32_t)(st + i);
            ids_dev.reserve((size_t)ct * sizeof(int32_t));
            VJ_HIP(hipMemcpyAsync(ids_dev.p, iota_h.data(), ct * sizeof(int32_t), hipMemcpyHostToDevice, s));
            ids = ids_dev.as<int32_t>();
        }
        const vj_status rc = vj_join(idx, ids, ct, eps_host[b], metric, pp, stream, &res[(size_t)b]);
        VJ_CHECK(rc == VJ_OK, rc, std::string("batch ") + std::to_string(b) + ": " + vj_last_error());
        if (batch_ms_host)
            batch_ms_host[b] = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    for (int32_t b = 0; b < n_batches; ++b) out[b] = res[(size_t)b];
    guard.done = true;
    API_END
}

vj_status vj_join_batches_device(vj_index *idx, const int32_t *query_ids,
                                 const int64_t *batch_start_host, const int64_t *batch_count_host,
                                 const float *eps_host, int32_t n_batches, vj_metric metric,
                                 const vj_join_params *pp, vj_submit submit, void *stream,
                                 vj_pairs **out, float *batch_ms_host) {
    API_BEGIN
    check_batches(idx, query_ids, batch_start_host, batch_count_host, eps_host, n_batches, out);
    Index &ix = idx->impl;
    VJ_CHECK(metric == ix.metric, VJ_ERR_METRIC_MISMATCH, "join metric differs from the index metric");
    vj_join_params p;
    vj_default_join_params(&p);
    if (pp) p = *pp;
    VJ_CHECK(p.hybrid_beam >= 0, VJ_ERR_INVALID_ARG, "hybrid_beam must be >= 0");
    VJ_CHECK(p.coop_tables == 0 || p.coop_tables == 1, VJ_ERR_INVALID_ARG, "coop_tables is 0 or 1");
    VJ_CHECK(!ix.separate, VJ_ERR_INVALID_ARG,
             "the device batch runner needs a merged index (use vj_join_batches)");
    for (int32_t b = 0; b < n_batches; ++b)
        VJ_CHECK(batch_count_host[b] < ((int64_t)1 << 31), VJ_ERR_UNSUPPORTED, "batch count must be < 2^31");
    std::vector<std::unique_ptr<vj_pairs>> res((size_t)n_batches);
    VJ_CHECK(submit == VJ_SUBMIT_DIRECT || submit == VJ_SUBMIT_GRAPH, VJ_ERR_INVALID_ARG,
             "submit is VJ_SUBMIT_DIRECT or VJ_SUBMIT_GRAPH");
    run_batches_device(ix, query_ids, batch_start_host, batch_count_host, eps_host, n_batches, p,
                       submit == VJ_SUBMIT_GRAPH, (hipStream_t)stream, res, batch_ms_host);
    for (int32_t b = 0; b < n_batches; ++b) out[b] = res[(size_t)b].release();
    API_END
}

vj_status vj_autotune_join(vj_index *idx, const int32_t *query_ids, int64_t n, float eps,
                           vj_metric metric, vj_join_params *pp, float *best_ms_host, void *stream) {
    API_BEGIN
    VJ_CHECK(idx != nullptr && pp != nullptr && (query_ids != nullptr || n == idx->impl.nq) && n >= 1,
             VJ_ERR_INVALID_ARG, "bad arguments");
    const Index &ix = idx->impl;
    vj_join_params base = *pp;
    // candidates: the one-wave or the workgroup tier first; fp32 or (when the
    // data is exactly u8) u8 rows -- all of them give the same decisions
    std::vector<vj_join_params> cand;
    for (int tier : {0, 1}) {
        for (int tables : {0, 1}) {
            if (tier == 0 && tables == 1) continue;
            for (int prec : {(int)VJ_PREC_FP32, (int)VJ_PREC_U8}) {
                if (prec == VJ_PREC_U8 && !ix.integer_u8) continue;
                if (base.precision != VJ_PREC_FP32 && base.precision != VJ_PREC_U8 &&
                    base.precision != VJ_PREC_AUTO) prec = base.precision;
                vj_join_params c = base;
                c.start_tier = tier;
                c.coop_tables = tables;
                c.precision = prec;
                cand.push_back(c);
            }
        }
    }
    float best = INFINITY;
    vj_join_params pick = base;
    for (const auto &c : cand) {
        float t = INFINITY;
        for (int rep = 0; rep < 3; ++rep) {  // first run warms the workspace
            vj_pairs *r = nullptr;
            const vj_status rc = vj_join(idx, query_ids, n, eps, metric, &c, stream, &r);
            VJ_CHECK(rc == VJ_OK, rc, vj_last_error());
            const float ms = r->impl.kernel_ms + r->impl.spill_ms;
            delete r;
            if (rep > 0) t = std::min(t, ms);
        }
        if (t < best) {
            best = t;
            pick = c;
        }
    }
    *pp = pick;
    if (best_ms_host) *best_ms_host = best;
    API_END
}

// ------------------------------------------------------------ predictor --

vj_status vj_join_features(vj_index *idx, const int32_t *query_ids, int64_t n, float eps,
                           vj_metric metric, float *features, void *stream) {
    API_BEGIN
    VJ_CHECK(idx != nullptr && (features != nullptr || n == 0), VJ_ERR_INVALID_ARG, "null pointer");
    Index &ix = idx->impl;
    VJ_CHECK(n >= 0 && (query_ids != nullptr || n == ix.nq || n == 0), VJ_ERR_INVALID_ARG,
             "query_ids may be NULL only with n == nq");
    VJ_CHECK(std::isfinite(eps), VJ_ERR_INVALID_ARG, "eps must be finite");
    VJ_CHECK(metric == ix.metric, VJ_ERR_METRIC_MISMATCH, "metric differs from the index metric");
    VJ_CHECK(!ix.separate, VJ_ERR_INVALID_ARG, "features need the merged index (the probe of q)");
    hipStream_t s = (hipStream_t)stream;
    if (n == 0) {
        vj::set_error("");
        return VJ_OK;
    }
    std::vector<int32_t> ids_h((size_t)n);
    if (query_ids) {
        VJ_HIP(hipMemcpyAsync(ids_h.data(), query_ids, n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        VJ_HIP(hipStreamSynchronize(s));
        for (int32_t q : ids_h) VJ_CHECK(q >= 0 && q < ix.nq, VJ_ERR_INVALID_ARG, "query id out of range");
    } else {
        for (int64_t i = 0; i < n; ++i) ids_h[(size_t)i] = (int32_t)i;
    }
    DevBuf ql((size_t)n * sizeof(int32_t));
    VJ_HIP(hipMemcpyAsync(ql.p, ids_h.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, s));
    compute_features(ix, ql.as<int32_t>(), n, eps, ix.d + kFeatures, features, s);
    VJ_HIP(hipStreamSynchronize(s));
    API_END
}

vj_status vj_predictor_create(int32_t din, int32_t h1, int32_t h2, int32_t k, uint64_t seed,
                              void *stream, vj_predictor **out) {
    API_BEGIN
    VJ_CHECK(out != nullptr, VJ_ERR_INVALID_ARG, "null pointer");
    VJ_CHECK(din >= 1 && h1 >= 1 && h2 >= 1 && k >= 1 && k <= 64, VJ_ERR_INVALID_ARG,
             "layer widths must be >= 1 (k <= 64)");
    auto h = std::make_unique<vj_predictor>();
    predictor_init(h->impl, din, h1, h2, k, seed, (hipStream_t)stream);
    *out = h.release();
    API_END
}

void vj_predictor_free(vj_predictor *p) { delete p; }

vj_status vj_predictor_set_params(vj_predictor *pr, const float *W1, const float *b1,
                                  const float *W2, const float *b2, const float *W3,
                                  const float *b3, const float *mu, const float *inv_sigma,
                                  void *stream) {
    API_BEGIN
    VJ_CHECK(pr != nullptr, VJ_ERR_INVALID_ARG, "null predictor");
    Predictor &p = pr->impl;
    hipStream_t s = (hipStream_t)stream;
    const float *src[8] = {W1, b1, W2, b2, W3, b3, mu, inv_sigma};
    DevBuf *dst[8] = {&p.W1, &p.b1, &p.W2, &p.b2, &p.W3, &p.b3, &p.mu, &p.inv_sigma};
    for (int i = 0; i < 8; ++i)
        if (src[i]) VJ_HIP(hipMemcpyAsync(dst[i]->p, src[i], dst[i]->bytes, hipMemcpyDeviceToDevice, s));
    VJ_HIP(hipStreamSynchronize(s));
    API_END
}

vj_status vj_predictor_get_params(const vj_predictor *pr, float *W1, float *b1, float *W2,
                                  float *b2, float *W3, float *b3, float *mu, float *inv_sigma,
                                  void *stream) {
    API_BEGIN
    VJ_CHECK(pr != nullptr, VJ_ERR_INVALID_ARG, "null predictor");
    const Predictor &p = pr->impl;
    hipStream_t s = (hipStream_t)stream;
    float *dst[8] = {W1, b1, W2, b2, W3, b3, mu, inv_sigma};
    const DevBuf *src[8] = {&p.W1, &p.b1, &p.W2, &p.b2, &p.W3, &p.b3, &p.mu, &p.inv_sigma};
    for (int i = 0; i < 8; ++i)
        if (dst[i]) VJ_HIP(hipMemcpyAsync(dst[i], src[i]->p, src[i]->bytes, hipMemcpyDeviceToDevice, s));
    VJ_HIP(hipStreamSynchronize(s));
    API_END
}

vj_status vj_predictor_fit_normalization(vj_predictor *pr, const float *X, int64_t n, void *stream) {
    API_BEGIN
    VJ_CHECK(pr != nullptr && X != nullptr && n >= 1, VJ_ERR_INVALID_ARG, "bad arguments");
    predictor_fit_normalization(pr->impl, X, n, (hipStream_t)stream);
    API_END
}

vj_status vj_predictor_forward(const vj_predictor *pr, const float *X, int64_t n, float *logits,
                               void *stream) {
    API_BEGIN
    VJ_CHECK(pr != nullptr && n >= 0 && (n == 0 || (X && logits)), VJ_ERR_INVALID_ARG, "bad arguments");
    VJ_CHECK(n < ((int64_t)1 << 31), VJ_ERR_UNSUPPORTED, "n must be < 2^31");
    predictor_forward(pr->impl, X, n, logits, (hipStream_t)stream);
    API_END
}

vj_status vj_predictor_loss_grad(const vj_predictor *pr, const float *X, const float *Y,
                                 const float *mask, int64_t n, double *loss, float *gW1,
                                 float *gb1, float *gW2, float *gb2, float *gW3, float *gb3,
                                 void *stream) {
    API_BEGIN
    VJ_CHECK(pr != nullptr && n >= 0 && (n == 0 || (X && Y)), VJ_ERR_INVALID_ARG, "bad arguments");
    VJ_CHECK(n < ((int64_t)1 << 31), VJ_ERR_UNSUPPORTED, "n must be < 2^31");
    const double l = predictor_loss_grad(pr->impl, X, Y, mask, n, gW1, gb1, gW2, gb2, gW3, gb3,
                                         (hipStream_t)stream);
    if (loss) *loss = l;
    API_END
}

vj_status vj_predictor_train(vj_predictor *pr, const float *X, const float *Y, int64_t n,
                             int32_t epochs, int32_t batch, float lr, uint64_t seed,
                             float *loss_per_epoch_host, void *stream) {
    API_BEGIN
    VJ_CHECK(pr != nullptr && X != nullptr && Y != nullptr && n >= 1, VJ_ERR_INVALID_ARG, "bad arguments");
    VJ_CHECK(epochs >= 0 && batch >= 1 && std::isfinite(lr) && lr > 0.f, VJ_ERR_INVALID_ARG,
             "epochs >= 0, batch >= 1, lr > 0");
    predictor_train(pr->impl, X, Y, n, epochs, batch, lr, seed, loss_per_epoch_host,
                    (hipStream_t)stream);
    API_END
}

vj_status vj_predictor_info(const vj_predictor *pr, int32_t *din, int32_t *h1, int32_t *h2,
                            int32_t *k) {
    API_BEGIN
    VJ_CHECK(pr != nullptr, VJ_ERR_INVALID_ARG, "null predictor");
    const Predictor &p = pr->impl;
    if (din) *din = p.din;
    if (h1) *h1 = p.h1;
    if (h2) *h2 = p.h2;
    if (k) *k = p.k;
    API_END
}

vj_status vj_predictor_save(const vj_predictor *pr, const char *path) {
    API_BEGIN
    VJ_CHECK(pr != nullptr && path != nullptr, VJ_ERR_INVALID_ARG, "null pointer");
    VJ_HIP(hipDeviceSynchronize());
    predictor_save(pr->impl, path);
    API_END
}

vj_status vj_predictor_load(const char *path, void *stream, vj_predictor **out) {
    API_BEGIN
    VJ_CHECK(path != nullptr && out != nullptr, VJ_ERR_INVALID_ARG, "null pointer");
    hipStream_t s = (hipStream_t)stream;
    auto h = std::make_unique<vj_predictor>();
    predictor_load(h->impl, path, s);
    VJ_HIP(hipStreamSynchronize(s));
    *out = h.release();
    API_END
}

vj_status vj_predictor_adam_step(vj_predictor *pr, const float *grad, float lr, void *stream) {
    API_BEGIN
    VJ_CHECK(pr != nullptr && grad != nullptr, VJ_ERR_INVALID_ARG, "null pointer");
    VJ_CHECK(std::isfinite(lr) && lr > 0.f, VJ_ERR_INVALID_ARG, "lr > 0");
    hipStream_t s = (hipStream_t)stream;
    predictor_adam(pr->impl, grad, lr, s);
    VJ_HIP(hipStreamSynchronize(s));
    API_END
}

vj_status vj_predictor_get_adam_state(const vj_predictor *pr, float *m, float *v,
                                      int64_t *steps, void *stream) {
    API_BEGIN
    VJ_CHECK(pr != nullptr, VJ_ERR_INVALID_ARG, "null predictor");
    const Predictor &p = pr->impl;
    hipStream_t s = (hipStream_t)stream;
    const size_t bytes = p.n_params() * sizeof(float);
    if (m) VJ_HIP(hipMemcpyAsync(m, p.m.p, bytes, hipMemcpyDeviceToDevice, s));
    if (v) VJ_HIP(hipMemcpyAsync(v, p.v.p, bytes, hipMemcpyDeviceToDevice, s));
    if (steps) *steps = p.steps;
    VJ_HIP(hipStreamSynchronize(s));
    API_END
}

vj_status vj_index_attach_predictor(vj_index *idx, const vj_predictor *pr, float recall_target,
                                    const int32_t *budgets_host) {
    API_BEGIN
    VJ_CHECK(idx != nullptr, VJ_ERR_INVALID_ARG, "null index");
    Index &ix = idx->impl;
    if (pr == nullptr) {
        ix.pred = nullptr;
        vj::set_error("");
        return VJ_OK;
    }
    VJ_CHECK(budgets_host != nullptr, VJ_ERR_INVALID_ARG, "budgets needed");
    VJ_CHECK(std::isfinite(recall_target) && recall_target > 0.f && recall_target <= 1.f,
             VJ_ERR_INVALID_ARG, "recall_target in (0, 1]");
    const Predictor &p = pr->impl;
    VJ_CHECK(p.din == ix.d + kFeatures, VJ_ERR_INVALID_ARG, "predictor input width is not d + 8");
    for (int j = 0; j < p.k; ++j) {
        VJ_CHECK(budgets_host[j] >= 0, VJ_ERR_INVALID_ARG, "budgets must be >= 0");
        VJ_CHECK(j == 0 || budgets_host[j] > budgets_host[j - 1], VJ_ERR_INVALID_ARG,
                 "budgets must be ascending");
    }
    ix.pred_budgets.alloc((size_t)p.k * sizeof(int32_t));
    VJ_HIP(hipMemcpy(ix.pred_budgets.p, budgets_host, p.k * sizeof(int32_t), hipMemcpyHostToDevice));
    ix.pred = &p;
    ix.pred_target = recall_target;
    API_END
}

}  // extern "C"

namespace vj {
bool launch_join(const JoinLaunch &L, hipStream_t s) {
    switch (L.prec) {
    case VJ_PREC_FP32: return launch_join_f32(L, s);
    case VJ_PREC_U8: return launch_join_u8(L, s);
    case VJ_PREC_FP8: return launch_join_f8(L, s);
    case VJ_PREC_BF16: return launch_join_bf16(L, s);
    default: return false;
    }
}
}  // namespace vj
