// Internal declarations of libvj (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <memory>
#include <string>
#include <vector>

#include "../../include/vj.h"

namespace vj {

// ---------------------------------------------------------------- errors --
void set_error(const std::string &msg);
const char *last_error();

struct Error {
    vj_status st;
    std::string msg;
};

#define VJ_HIP(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            throw ::vj::Error{e_ == hipErrorOutOfMemory ? VJ_ERR_OOM : VJ_ERR_HIP,     \
                              std::string(#call) + ": " + hipGetErrorString(e_)};      \
    } while (0)

#define VJ_CHECK(cond, status, msg)                                                   \
    do {                                                                               \
        if (!(cond)) throw ::vj::Error{status, msg};                                  \
    } while (0)

// Device memory with reuse of large blocks: a block of kBlockCacheMin bytes
// or more is not returned to the runtime when freed but kept per device (the
// device is synchronised first, as hipFree would) and handed to a later
// request of between half its size and its size; at most kBlockCacheMax
// bytes are kept per device, and a failed hipMalloc empties the cache and
// retries.  Such blocks are allocated rounded up to an eighth of their
// power of two (at most 12.5 % more), so that a later request a little
// larger (an insertion's buffers grow with the index) still finds them.
// Large hipMalloc / hipFree pairs cost up to a second each when a build or
// an insertion allocates gigabytes of temporaries again and again.  *cap:
// the bytes allocated, which dev_free takes.
constexpr size_t kBlockCacheMin = (size_t)16 << 20;
constexpr size_t kBlockCacheMax = (size_t)32 << 30;
void *dev_alloc(size_t n, int *dev, size_t *cap);
void dev_free(void *p, size_t n, int dev);
// return every kept block of the current device to the runtime; bytes freed
size_t trim_block_cache();

// Device buffer that frees itself.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    size_t cap = 0;   // bytes allocated (>= bytes)
    bool own = true;  // false: a view into another buffer (not freed here)
    int dev = -1;     // device of the block
    DevBuf() = default;
    explicit DevBuf(size_t n) { alloc(n); }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : p(o.p), bytes(o.bytes), cap(o.cap), own(o.own), dev(o.dev) {
        o.p = nullptr;
        o.bytes = o.cap = 0;
        o.own = true;
        o.dev = -1;
    }
    DevBuf &operator=(DevBuf &&o) noexcept {
        if (this != &o) {
            release();
            p = o.p; bytes = o.bytes; cap = o.cap; own = o.own; dev = o.dev;
            o.p = nullptr; o.bytes = o.cap = 0; o.own = true; o.dev = -1;
        }
        return *this;
    }
    ~DevBuf() { release(); }
    static DevBuf view(void *ptr, size_t n) {
        DevBuf v;
        v.p = ptr;
        v.bytes = n;
        v.own = false;
        return v;
    }
    void alloc(size_t n) {
        release();
        if (n == 0) n = 16;
        p = dev_alloc(n, &dev, &cap);
        bytes = n;
    }
    // grow (contents not kept)
    void reserve(size_t n) { if (n > bytes || !own) alloc(n); }
    void release() {
        if (p && own) dev_free(p, cap, dev);
        p = nullptr;
        bytes = cap = 0;
        own = true;
        dev = -1;
    }
    template <typename T> T *as() const { return static_cast<T *>(p); }
};

// Element tag of fp8 (OCP e4m3) rows: one byte per value, scaled per row.
struct f8e4m3 {
    uint8_t bits;
};

// value of an OCP e4m3 code (normal: exponent field + 120 into the fp32
// exponent; subnormal: m 2^-9)
__device__ __forceinline__ float f8_value(uint32_t b) {
    const uint32_t em = b & 0x7fu;
    const float f = em >= 8u ? __uint_as_float((em << 20) + 0x3C000000u) : (float)em * 0.001953125f;
    return (b & 0x80u) ? -f : f;
}

// Padded row widths the kernels are compiled for (elements).
int padded_dim(int d);

// ----------------------------------------------------------------- index --
// State of one replay slot of the device batch runner (grow only): its
// arguments, counters, descriptors, lists, global tables and output.
struct BatchSlot {
    DevBuf args, counters, desc, rec, lists, gh, gil, gild, gh3, gil3, gild3, out_q, out_x, out_d;
    hipStream_t stream = nullptr;  // default priority, non-blocking
    hipGraphExec_t exec = nullptr; // steps captured for the launch shape in `key`
    std::vector<uint64_t> key;
    BatchSlot() = default;
    BatchSlot(const BatchSlot &) = delete;
    BatchSlot &operator=(const BatchSlot &) = delete;
    ~BatchSlot() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (stream) (void)hipStreamDestroy(stream);
    }
};

// Buffers of vj_join kept between calls on one index (grow only).
struct JoinWorkspace {
    DevBuf qlist, qpos, counters, args, ovf, slots, out_q, out_x, out_d;
    DevBuf sort_keys, sort_tmp;     // densest-first order: d1 buckets, bucket counts
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipStream_t capture = nullptr;  // private stream the batch graphs are captured on
    BatchSlot bslot[2];             // the device batch runner's two replay slots
    hipEvent_t bev[1 + 2] = {};     // its events: the fork, one join per slot
    void *pinned = nullptr;  // 4 KiB of pinned host memory: counters read back, arguments sent
    JoinWorkspace() = default;
    JoinWorkspace(const JoinWorkspace &) = delete;
    JoinWorkspace &operator=(const JoinWorkspace &) = delete;
    ~JoinWorkspace() {
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
        if (capture) (void)hipStreamDestroy(capture);
        for (auto e : bev) if (e) (void)hipEventDestroy(e);
        if (pinned) (void)hipHostFree(pinned);
    }
};

struct Index {
    int64_t nq = 0, nx = 0, N = 0;
    int32_t d = 0, dp = 0, R = 0, entry = 0;
    vj_metric metric = VJ_L2;
    int device = 0;
    bool integer_u8 = false;  // every value an integer in [0, 255]
    bool bf16_exact = false;  // every value exact in bf16 (valid once vec_bf16 exists)
    DevBuf vec;      // float [N][dp], zero padded
    DevBuf vec_u8;   // uint8 [N][dp] (integer_u8 only)
    DevBuf vec_bf16; // bf16 [N][dp] (optional)
    DevBuf vec_f8;   // fp8 e4m3 codes [N][dp] (optional): x~ = scale * decode(code)
    DevBuf f8meta;   // float2 [N]: (power-of-two row scale, bound on |x - x~| rounded up)
    DevBuf adj;      // int32 [N][R], -1 padded
    DevBuf elen;     // float [N][R] L2 edge lengths, +inf padded
    DevBuf parent;   // int32 [nq] MST parent node id (-1: entry)
    DevBuf depth;    // int32 [nq] depth in the MST (root children: 0)
    bool has_mst = false;
    // separate indexes (cfg.merged = false): adj rows 0..nx-1 are the data
    // graph G_X (entry: its entry), rows nx.. the query graph G_Q (node ids),
    // read only by the MST
    bool separate = false;
    // NN-Map of the queries (Section 6): witness, its distance, OOD bit
    DevBuf nn_w, nn_d, nn_ood;
    bool has_nnmap = false;
    // HNSW-style upper layers over the data nodes (layer 1 first): row
    // offsets, node counts and entries of each layer; adjacency [rows][lay_R]
    // in data ids; lay_pos [layers][nx] the row of node v in each layer (-1:
    // absent); lay_seed [nq] the seeds of the last descent
    int32_t lay_n = 0, lay_R = 0;
    std::vector<int64_t> lay_off, lay_cnt;
    std::vector<int32_t> lay_entry;
    DevBuf lay_adj, lay_pos, lay_ids, lay_offd, lay_seed;
    int64_t repairs = 0;  // connectivity-repair edges added by the build
    // work of the last build or insertion: the kNN sweep's tiles (first pass,
    // second pass, all pairs; row blocks x column tiles, 0 on the wide-row
    // sweep), its repair edges and the steps answered from the kNN lists
    int64_t knn_tiles[3] = {0, 0, 0};
    int64_t last_repairs = 0, last_listed = 0;
    // group order of the kNN sweep, kept so that an insertion labels only
    // its new nodes: group centres (fp32 [piv_n][dp]), the nearest centre of
    // nodes [0, piv_cnt) and each group's radius (fp32 [piv_n]: no member of
    // group g is farther than piv_rad[g] from its centre)
    DevBuf piv_rows, piv_of, piv_rad;
    // kNN lists kept for the connectivity repair of later insertions (rows
    // [0, knn_rows), room for knn_cap): node v's knn_kc nearest among the
    // nodes [0, knn_from[v]) that existed when its list was made (int32
    // ids, fp32 squared distances in the repair's arithmetic, sorted by
    // (d2, id)), and knn_cert[v], a squared distance below which no other
    // of those nodes lies (-inf: no list)
    DevBuf knn_id, knn_d2, knn_cert, knn_from;
    int32_t knn_kc = 0;
    int64_t knn_rows = 0, knn_cap = 0;
    int32_t piv_n = 0;
    int64_t piv_cnt = 0;
    // join state shared by calls on this index (calls on one index must not overlap)
    DevBuf cache;    // int32 [nq] soft work sharing: closest visited data node
    DevBuf inb;      // int32 [nq] generation stamp: query is part of the current call
    DevBuf seg;      // int64 [nq] offset of the query's pairs in the call's output
    DevBuf segn;     // int32 [nq] number of pairs of the query
    DevBuf done;     // int32 [nq] persistent soft / hard joins: publication stamp (gen)
    DevBuf ws_gh, ws_gil, ws_gild;  // global tables of the join (kept between calls)
    JoinWorkspace jw;
    // attached difficulty predictor (VJ_HYB_LEARNED); not owned
    const struct Predictor *pred = nullptr;
    float pred_target = 0.f;
    DevBuf pred_budgets;  // int32 [k] out-range pop budget of each head, ascending
    int32_t gen = 0;
};

// ----------------------------------------------------------------- pairs --
struct Pairs {
    int64_t count = 0;
    int64_t n_queries = 0;   // rows of stats (0 for brute force)
    int64_t n_candidates = 0; // brute force: pairs re-checked in fp64
    float kernel_ms = 0.f;    // join: LDS-variant launches, timed with events on the stream
    float spill_ms = 0.f;     // join: spill-variant launches
    int64_t n_spilled = 0;    // join: queries re-run on the spill variant
    float tier_ms[4] = {0.f, 0.f, 0.f, 0.f};  // join: device time per storage tier
    int32_t tier_launches[4] = {0, 0, 0, 0};
    int64_t tier_queries[4] = {0, 0, 0, 0};
    DevBuf q, x, dist;       // int32, int32, float [count]
    DevBuf stats;            // int32 [n_queries][8]
    // blocks that q / x / dist / stats are views into, shared by the results
    // of one batch run
    std::vector<std::shared_ptr<DevBuf>> keep;
};

// --------------------------------------------------------------- kernels --
// Join parameters, resident in device memory for the duration of a call.
struct JoinArgs {
    const void *rows;         // rows the distances read: float or uint8 [N][dp]
    const float *rows32;      // fp32 rows (query slices)
    const int32_t *adj;       // [N][R]
    const float *elen;        // [N][R]
    int64_t nx, nq;
    int32_t R, dp, entry, metric;
    float eps, eps2;          // L2 compares the squared distance with eps2
    float bf_u;               // bf16 rows: bound on |x - bf16(x)| / |bf16(x)| (0: exact copy)
    const float2 *f8meta;     // fp8 rows: per row (scale, bound on |x - x~|)
    unsigned long long *nrecheck;  // bf16 rows: candidates re-decided from fp32 rows
    int32_t ws, hyb, beam, conv;
    int32_t merged;           // 1 merged index; 0 separate indexes (adj rows < nx: data graph)
    const int32_t *nn_w;      // NN-Map: [nq] witness (nearest data node) of each query
    const double *nn_d;       // [nq] its distance (join metric, fp64)
    const uint8_t *nn_ood;    // [nq] OOD bit
    int32_t gbeam;            // separate indexes: greedy queue bound (cfg.greedy_beam_size)
    const int32_t *qseed;     // separate indexes: [nq] per-query seed in place of the entry (null: entry)
    float ood_ratio;
    int32_t gen;              // stamp of this call in inb[]
    const int32_t *parent;    // [nq] MST parent node id (-1: entry)
    const int32_t *inb;       // [nq] == gen: query is part of this call
    int32_t *cache;           // [nq] soft: closest visited data node
    int64_t *seg;             // [nq] hard: offset of the query's pairs
    int32_t *segn;            // [nq] hard: number of them
    const int32_t *budget;    // [n] by caller position (VJ_HYB_BUDGET)
    int32_t *out_q, *out_x;
    float *out_d;
    int64_t cap;
    unsigned long long *out_count;
    int32_t *stats;           // [n][8] by caller position
    int32_t *err;             // bit flags: 8 query id out of range, 16 probe past the table, 32 list entry not a data id, 64 tiers exhausted (batch steps), 128 a wave waited past its bound, 256 a parent wait passed its bound
    // persistent launches of soft / hard work sharing: done[qi] == gen once
    // query qi's cache (soft) or pairs (hard) are published, gen | kDeferred
    // when it was deferred to a later launch; null: parents ran in an
    // earlier launch (no waiting)
    int32_t *done;
};

// One launch over a contiguous piece of the processing list.
struct JoinLaunch {
    const JoinArgs *args;     // device pointer
    const int32_t *qlist;     // query index per processing slot
    const int32_t *qpos;      // caller position per processing slot
    int first, count, dp, prec;  // slots [first, first + count) of qlist
    int tier;                    // 0 one wave + LDS, 1 workgroup + LDS, 2 workgroup + global
    bool coop_small;             // tier 1: the small LDS tables
    bool hyb;
    int32_t *gh;              // global tables: [regions][1 << hash_log2] visited sets
    int hash_log2;
    int32_t *gil;             // [regions][il_cap] in-range lists
    float *gild;
    int il_cap;
    int32_t *promo_next;      // tier 1: counter of the global regions taken in the launch
    int promo_cap;            // tier 1: regions of gh / gil / gild it may take (0: none)
    int32_t *ovf, *ovf_count; // slots (indices into qlist) that must be re-run
    const int32_t *count_dev; // tiers 1-2: the slot count on the device, at most `count` (null: count)
    const int32_t *slots;     // tier 2: entry k is slot slots[k] of qlist (null: slot k)
    int grid;                 // tier 2: workgroups looping over the slots (0: one per slot)
    int32_t *claim;           // tier 1: persistent launch of L.grid workgroups that claim the
                              // slots in order from this counter (null: one workgroup per slot)
};

constexpr int32_t kDeferred = 1 << 30;  // done[] flag of a query deferred to a later launch

bool launch_join(const JoinLaunch &L, hipStream_t s);
bool launch_join_f32(const JoinLaunch &L, hipStream_t s);
bool launch_join_u8(const JoinLaunch &L, hipStream_t s);
bool launch_join_bf16(const JoinLaunch &L, hipStream_t s);
bool launch_join_f8(const JoinLaunch &L, hipStream_t s);
int num_cus();

// edge lengths of every adjacency entry (L2)
void launch_edge_lengths(const float *vec, int dp, const int32_t *adj, int64_t N, int R,
                         float *elen, hipStream_t s);
// the same for the rows rows[0..M) only
void launch_edge_lengths_rows(const float *vec, int dp, const int32_t *adj, int64_t N, int R,
                              const int32_t *rows, int64_t M, float *elen, hipStream_t s);
// copy rows into a zero-padded layout
void launch_pad_rows(const float *src, int64_t rows, int d, float *dst, int dp,
                     hipStream_t s);
// u8 / bf16 copies; flag[0] |= 1 if some value is not an integer in [0,255]
void launch_quantize(const float *vec, int64_t rows, int dp, uint8_t *u8, uint16_t *bf16,
                     int32_t *flag, hipStream_t s);
// fp8 e4m3 copy: per row a power-of-two scale s >= max|x| / 448, codes of
// x / s rounded to nearest even (saturating), meta = (s, |x - s decode|
// computed in fp64 and rounded up)
void launch_quantize_f8(const float *vec, int64_t rows, int dp, uint8_t *codes, float2 *meta,
                        hipStream_t s);

// pairs export
void export_pairs(const Pairs &r, int32_t *qx, float *dist, bool sorted, hipStream_t s);

// index files: the padded rows, graph, edge lengths and MST; at load
// `finish` rebuilds the exact low-precision copies and the join state
void index_save(const Index &ix, const char *path);
void index_load(Index &ix, const char *path, void (*finish)(Index &, hipStream_t), hipStream_t s);

}  // namespace vj
