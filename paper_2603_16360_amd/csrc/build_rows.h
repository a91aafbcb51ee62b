// Row-wise graph-build kernels templated on the padded row width DP:
// exact re-rank of the kNN candidates, the forward RNG prune and the prune
// of forward + reverse candidates (Appendix C edge rule; ties by smaller
// id).  Instantiated once per width by build_inst.hip.
#pragma once

#include "mfma_tile.h"
#include "vj_internal.h"

namespace vj {
namespace brow {

constexpr int kKnnCap = 384;   // per-row candidate buffer of the top-K sweep
constexpr int kCandMax = 1024; // candidates a reverse-edge prune considers

inline unsigned g1b(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }
// --------------------------------------------------- row distance helper --
// squared L2 distances from row `u` to up to 8 rows at once: lane group g
// (8 lanes) handles ids[g]; returns the group's total in every lane of it.
template <int DP>
__device__ __forceinline__ float dist8(const float *vec, int32_t u, int32_t v, int lane) {
    constexpr int CH = DP / 4;             // float4 chunks per row
    constexpr int PER = (CH + 7) / 8;       // chunks per lane
    const int p = lane & 7;
    const float4 *a = reinterpret_cast<const float4 *>(vec + (size_t)u * DP);
    const float4 *b = reinterpret_cast<const float4 *>(vec + (size_t)v * DP);
    float acc = 0.f;
#pragma unroll
    for (int t = 0; t < PER; ++t) {
        const int c = p + 8 * t;
        if (c < CH) {
            const float4 x = a[c], y = b[c];
            float q;
            q = x.x - y.x; acc = fmaf(q, q, acc);
            q = x.y - y.y; acc = fmaf(q, q, acc);
            q = x.z - y.z; acc = fmaf(q, q, acc);
            q = x.w - y.w; acc = fmaf(q, q, acc);
        }
    }
    acc += __shfl_xor(acc, 4);
    acc += __shfl_xor(acc, 2);
    acc += __shfl_xor(acc, 1);
    return acc;
}

// Exact re-rank of the K buffered neighbours of rows [rb, rb + M) (buffers
// indexed from rb): direct fp32 squared distances, sorted by (distance, id);
// the first Kc are written out.
template <int DP>
__global__ void __launch_bounds__(256)
k_rerank(const float *vec, int64_t N, const int32_t *bid, int K, int Kc, int32_t *out_id,
         float *out_d2, int64_t rb, int64_t M) {
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= M) return;
    const int64_t u = rb + i;
    float key[2];
    int id[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) { key[j] = INFINITY; id[j] = 0x7fffffff; }
    for (int base = 0; base < K; base += 8) {
        const int e = base + (lane >> 3);
        const int32_t v = e < K ? bid[i * kKnnCap + e] : -1;
        const bool ok = e < K && v >= 0 && v < N && v != u;
        const float d2 = dist8<DP>(vec, (int32_t)u, ok ? v : (int32_t)u, lane);
        // element e goes to register e / 64 of lane e % 64
        for (int g = 0; g < 8; ++g) {
            const int ee = base + g;
            const float dd = __shfl(d2, g * 8);
            const int vv = __shfl(v, g * 8);
            const bool okk = __shfl((int)ok, g * 8) != 0;
            if (ee < 128 && (ee & 63) == lane) {
                const float kk = okk ? dd : INFINITY;
                const int ii = okk ? vv : 0x7fffffff;
                if (ee < 64) { key[0] = kk; id[0] = ii; }
                else { key[1] = kk; id[1] = ii; }
            }
        }
    }
    mt::wave_sort<2>(key, id, lane);
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int e = j * 64 + lane;
        if (e < Kc) {
            const bool ok = key[j] < INFINITY;
            out_id[i * Kc + e] = ok ? id[j] : -1;
            out_d2[i * Kc + e] = key[j];
        }
    }
}

// RNG prune of one wave's candidate list (sorted by (d2, id), m entries, in
// LDS), continuing from the nk0 ids already in kept[]: keep v unless a kept w
// has d2(w, v) < d2(u, v); at most R kept.  Returns the new kept count.
template <int DP>
__device__ __forceinline__ int rng_prune(const float *vec, const int32_t *cid, const float *cd2,
                                         int m, int R, int32_t *kept, int lane, int nk0 = 0) {
    int nk = nk0;
    for (int i = 0; i < m && nk < R; ++i) {
        const int32_t v = cid[i];
        const float dv = cd2[i];
        if (v < 0) continue;
        bool blocked = false;
        for (int b0 = 0; b0 < nk && !blocked; b0 += 8) {
            const int b = b0 + (lane >> 3);
            const int32_t wv = b < nk ? kept[b] : v;
            const float d2 = dist8<DP>(vec, wv, v, lane);
            blocked = __ballot(b < nk && d2 < dv) != 0;
        }
        if (!blocked) {
            if (lane == 0) kept[nk] = v;
            ++nk;
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
            __builtin_amdgcn_wave_barrier();
        }
    }
    return nk;
}

// forward prune of the re-ranked kNN lists of rows [rb, rb + M) (every
// buffer indexed from rb; indeg by node id)
template <int DP>
__global__ void __launch_bounds__(256)
k_prune_fwd(const float *vec, int64_t M, const int32_t *kid, const float *kd2, int Kc, int R,
            int32_t *fwd, float *fwd_d2, int32_t *fdeg, int32_t *indeg, int64_t rb) {
    __shared__ int32_t s_kept[4][64];
    __shared__ int32_t s_cid[4][256];
    __shared__ float s_cd[4][256];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t i = (int64_t)blockIdx.x * 4 + w;
    if (i >= M) return;
    const int64_t u = rb + i;
    for (int e = lane; e < Kc; e += 64) { s_cid[w][e] = kid[i * Kc + e]; s_cd[w][e] = kd2[i * Kc + e]; }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
    __builtin_amdgcn_wave_barrier();
    const int nk = rng_prune<DP>(vec, s_cid[w], s_cd[w], Kc, R, s_kept[w], lane);
    for (int e = lane; e < R; e += 64) {
        const int32_t v = e < nk ? s_kept[w][e] : -1;
        fwd[i * R + e] = v;
        float dv = INFINITY;
        for (int t = 0; t < Kc; ++t)
            if (s_cid[w][t] == v) { dv = s_cd[w][t]; break; }
        fwd_d2[i * R + e] = e < nk ? dv : INFINITY;
        if (e < nk) atomicAdd(&indeg[v], 1);
    }
    if (lane == 0) fdeg[i] = nk;
}


// final rows: fwd(v) + rev(v), sorted by (d2, id), deduplicated; kept whole
// if <= R, else RNG-pruned to R over the whole sorted list.  The candidates
// are streamed through a sorted buffer of 1024 (16 per lane); when more than
// 1024 pass a pass's filter, only the first 768 of the buffer are exact ranks,
// so the prune takes those and the next pass streams the candidates after
// the last of them again, until R are kept or the list is exhausted.
// The rows are rows[0..M) (all rows 0..M-1 when rows is null); fwd, fwd_d2
// and fdeg are indexed by the position in that list, roff and adj by node.
template <int DP>
__global__ void __launch_bounds__(256)
k_prune_rev(const float *vec, int64_t M, int R, const int32_t *fwd, const float *fwd_d2,
            const int32_t *fdeg, const int64_t *roff, const int32_t *rid, const float *rd2,
            int32_t *adj, const int32_t *rows) {
    __shared__ int32_t s_kept[4][64];
    __shared__ int32_t s_cid[4][kCandMax];
    __shared__ float s_cd[4][kCandMax];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t li = (int64_t)blockIdx.x * 4 + w;
    if (li >= M) return;
    const int64_t v = rows ? (int64_t)rows[li] : li;
    const int nf = fdeg[li];
    const int64_t r0 = roff[v], nr = roff[v + 1] - r0;
    const int64_t total = nf + nr;
    // exclusive lower bound (in (d2, id) order) of the candidates a pass takes
    float lo_k = -INFINITY;
    int lo_i = -1;
    int nk = 0;
    for (int pass = 0;; ++pass) {
        float key[16];
        int id[16];
#pragma unroll
        for (int j = 0; j < 16; ++j) { key[j] = INFINITY; id[j] = 0x7fffffff; }
        // stream the candidates after the bound, 256 new ones at a time into
        // ranks 768..1023 of the sorted buffer; ranks 0..767 always hold the
        // 768 smallest streamed so far.  `lost`: a candidate at ranks
        // 768..1023 was overwritten, so only ranks 0..767 are exact.
        bool lost = false;
        for (int64_t base = 0; base < total; base += 256) {
            lost |= __ballot(id[12] != 0x7fffffff || id[13] != 0x7fffffff ||
                             id[14] != 0x7fffffff || id[15] != 0x7fffffff) != 0;
#pragma unroll
            for (int j = 12; j < 16; ++j) {
                const int64_t e = base + (j - 12) * 64 + lane;
                float k = INFINITY;
                int i = 0x7fffffff;
                if (e < total) {
                    if (e < nf) { i = fwd[li * R + e]; k = fwd_d2[li * R + e]; }
                    else { i = rid[r0 + (e - nf)]; k = rd2[r0 + (e - nf)]; }
                    if (!mt::kless(lo_k, lo_i, k, i)) { k = INFINITY; i = 0x7fffffff; }
                }
                key[j] = k;
                id[j] = i;
            }
            mt::wave_sort<16>(key, id, lane);
        }
        // nothing lost: the buffer holds every remaining candidate, in order
        const bool last = !lost;
        const int limit = last ? kCandMax : 768;
        // dedup (equal ids are adjacent: same id, same squared distance)
        int m = 0;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int up = __shfl_up(id[j], 1);
            const int prv = j > 0 ? __shfl(id[j > 0 ? j - 1 : 0], 63) : -2;
            const int prev = lane == 0 ? prv : up;
            const bool keep = (j * 64 + lane) < limit && key[j] < INFINITY && id[j] != 0x7fffffff &&
                              id[j] != prev;
            const uint64_t mk = __ballot(keep);
            if (keep) {
                const int at = m + __popcll(mk & ((1ull << lane) - 1ull));
                s_cid[w][at] = id[j];
                s_cd[w][at] = key[j];
            }
            m += __popcll(mk);
        }
        // the last exact rank of this pass bounds the next one (entry 767:
        // register 11 of lane 63)
        lo_k = __shfl(key[11], 63);
        lo_i = __shfl(id[11], 63);
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
        __builtin_amdgcn_wave_barrier();
        if (pass == 0 && last && m <= R) {
            // the whole list fits: keep every candidate
            for (int e = lane; e < m; e += 64) s_kept[w][e] = s_cid[w][e];
            nk = m;
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
            __builtin_amdgcn_wave_barrier();
            break;
        }
        nk = rng_prune<DP>(vec, s_cid[w], s_cd[w], m, R, s_kept[w], lane, nk);
        if (last || nk >= R) break;
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
        __builtin_amdgcn_wave_barrier();
    }
    for (int e = lane; e < R; e += 64) adj[v * R + e] = e < nk ? s_kept[w][e] : -1;
}

// the current rows of the listed nodes below n_old (from adj), the forward
// lists of the others (from fwd_new, indexed from n_old), with fp32 squared
// lengths, as the forward part of an insertion's final prune
template <int DP>
__global__ void __launch_bounds__(256)
k_gather_rows(const float *vec, int R, const int32_t *adj, const int32_t *fwd_new,
              const int32_t *fdeg_new, int64_t n_old, const int32_t *rows, int64_t M,
              int32_t *fwd, float *fwd_d2, int32_t *fdeg) {
    const int lane = threadIdx.x & 63;
    const int64_t li = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (li >= M) return;
    const int64_t v = rows[li];
    const int32_t *src = v < n_old ? adj + v * R : fwd_new + (v - n_old) * R;
    int deg = 0;
    if (v < n_old) {
        for (int j = 0; j < R; ++j) deg += src[j] >= 0;
    } else {
        deg = fdeg_new[v - n_old];
    }
    for (int b = 0; b < R; b += 8) {
        const int e = b + (lane >> 3);
        const int32_t x = e < deg ? src[e] : -1;
        const float d2 = dist8<DP>(vec, (int32_t)v, x >= 0 ? x : (int32_t)v, lane);
        if ((lane & 7) == 0 && e < R) {
            fwd[li * R + e] = x;
            fwd_d2[li * R + e] = x >= 0 ? d2 : INFINITY;
        }
    }
    if (lane == 0) fdeg[li] = deg;
}

template <int DP>
void launch_rows(const float *vec, int64_t N, int R, int K, int Kc, const int32_t *bid,
                 int32_t *kid, float *kd2, int32_t *fwd, float *fwd_d2, int32_t *fdeg,
                 int32_t *indeg, int64_t rb, int64_t M, hipStream_t s) {
    hipLaunchKernelGGL(k_rerank<DP>, dim3(g1b(M, 4)), dim3(256), 0, s, vec, N, bid, K, Kc, kid,
                       kd2, rb, M);
    hipLaunchKernelGGL(k_prune_fwd<DP>, dim3(g1b(M, 4)), dim3(256), 0, s, vec, M, kid, kd2, Kc, R,
                       fwd, fwd_d2, fdeg, indeg, rb);
}

template <int DP>
void launch_rev(const float *vec, int64_t M, int R, const int32_t *fwd, const float *fwd_d2,
                const int32_t *fdeg, const int64_t *roff, const int32_t *rid, const float *rd2,
                int32_t *adj, const int32_t *rows, hipStream_t s) {
    hipLaunchKernelGGL(k_prune_rev<DP>, dim3(g1b(M, 4)), dim3(256), 0, s, vec, M, R, fwd, fwd_d2,
                       fdeg, roff, rid, rd2, adj, rows);
}

template <int DP>
void launch_gather(const float *vec, int R, const int32_t *adj, const int32_t *fwd_new,
                   const int32_t *fdeg_new, int64_t n_old, const int32_t *rows, int64_t M,
                   int32_t *fwd, float *fwd_d2, int32_t *fdeg, hipStream_t s) {
    hipLaunchKernelGGL(k_gather_rows<DP>, dim3(g1b(M, 4)), dim3(256), 0, s, vec, R, adj, fwd_new,
                       fdeg_new, n_old, rows, M, fwd, fwd_d2, fdeg);
}

}  // namespace brow
}  // namespace vj
