// Merged-graph construction on the GPU (Section 4.3: one graph over Q and X;
// Appendix C: the RNG edge rule).  The paper treats the graph index as a
// black box; this build makes it deterministic, ties broken by smaller id:
//   1. exact K nearest neighbours of every node (MFMA tiles + a running
//      top-K per row), re-ranked by direct fp32 distances;
//   2. RNG prune of each list: scan by (distance, id), keep v unless an
//      already-kept w is closer to v than the owner is; at most R kept;
//   3. reverse edges: the candidates of v are its pruned list plus every u
//      whose pruned list holds v; all of them if they fit in R, otherwise
//      the RNG prune of them;
//   4. entry = node nearest to the fp64 centroid;
//   5. connectivity repair from the entry: the smallest unreachable node
//      gets an edge from its nearest reachable node with a free slot (else
//      it replaces that node's longest edge), until all are reachable.
#include <algorithm>
#include <cfloat>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <vector>

#include "build.h"
#include "build_rows.h"
#include "lds_ring.h"
#include "mfma_tile.h"
#include "tiles.h"
#include "util.h"

namespace vj {
namespace {

using mt::floatx4;
using brow::kKnnCap;
using brow::g1b;

// ------------------------------------------------------------------ kNN --
// A workgroup of 4 waves owns 64 rows (16 per wave) and sweeps all N rows as
// columns, 128 per step.  Each step's column tile is staged once in LDS (in
// chunks of 128 dimensions, rows padded by 16 bytes) and read by all four
// waves; each wave's rows come from global memory (cached).  Each row keeps
// a buffer [K best | pending] in global memory; an element enters the buffer
// when its key (|x|^2 - 2<u,x>, same order as |u-x|^2) is <= the row's
// current K-th key.  After a step, rows with > K + 128 entries are sorted
// and cut back to K.  The rows are [rb, rb + M) of the N (buffers indexed
// from rb), the columns all N.
constexpr int kKc = 128;          // dimensions per staged chunk
constexpr int kLdsRow = kKc + 8;  // bf16 per staged row

template <int NSPLIT>
__global__ void __launch_bounds__(256)
k_knn(const uint16_t *Ah, const uint16_t *Al, int64_t N, int Kp, const float *n2, int K,
      float *bkey, int32_t *bid, int64_t rb, int64_t M) {
    __shared__ float s_tau[4][16];
    __shared__ int s_cnt[4][16];
    __shared__ __attribute__((aligned(16))) uint16_t sb_hi[128 * kLdsRow];
    __shared__ __attribute__((aligned(16))) uint16_t sb_lo[NSPLIT == 3 ? 128 * kLdsRow : 8];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t r0 = rb + (int64_t)blockIdx.x * 64 + w * 16;
    const int64_t rend = rb + M;
    if (lane < 16) { s_tau[w][lane] = INFINITY; s_cnt[w][lane] = 0; }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
    __builtin_amdgcn_wave_barrier();
    auto merge_row = [&](int r) {
        const int64_t row = r0 + r;
        const int c = min(s_cnt[w][r], kKnnCap);
        float key[8];
        int id[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int e = j * 64 + lane;
            const bool ok = e < c && row < rend;
            key[j] = ok ? bkey[(row - rb) * kKnnCap + e] : INFINITY;
            id[j] = ok ? bid[(row - rb) * kKnnCap + e] : 0x7fffffff;
        }
        mt::wave_sort<8>(key, id, lane);
        const int keep = min(c, K);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int e = j * 64 + lane;
            if (e < K && row < rend) {
                bkey[(row - rb) * kKnnCap + e] = e < keep ? key[j] : INFINITY;
                bid[(row - rb) * kKnnCap + e] = e < keep ? id[j] : -1;
            }
        }
        // K-th key (element K-1) is register (K-1)/64 of lane (K-1)%64
        float kth = INFINITY;
#pragma unroll
        for (int j = 0; j < 8; ++j)
            if (j == (K - 1) / 64) kth = __shfl(key[j], (K - 1) & 63);
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
        if (lane == 0) {
            s_cnt[w][r] = keep;
            s_tau[w][r] = keep >= K ? kth : INFINITY;
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
        __builtin_amdgcn_wave_barrier();
    };

    const int r16 = lane & 15, kq = (lane >> 4) * 8;
    for (int64_t c0 = 0; c0 < N; c0 += 128) {
        floatx4 acc[8];
#pragma unroll
        for (int ct = 0; ct < 8; ++ct) acc[ct] = floatx4{0.f, 0.f, 0.f, 0.f};
        for (int kc0 = 0; kc0 < Kp; kc0 += kKc) {
            const int kw = min(kKc, Kp - kc0);  // a multiple of 32
            const int cpr = kw / 8;             // 16-byte chunks per staged row
            __syncthreads();                    // the previous chunk is consumed
            // one 64-bit base per tile, 32-bit offsets inside it (128 rows);
            // e / cpr as a multiply: with inv = ceil(2^16 / cpr) the quotient
            // is exact for e < 2^16 / 16 and cpr <= 16
            const uint16_t *th = Ah + c0 * Kp + kc0;
            const uint16_t *tl = NSPLIT == 3 ? Al + c0 * Kp + kc0 : nullptr;
            const int nrow = (int)std::min<int64_t>(128, N - c0);
            const uint32_t inv = (65536u + (uint32_t)cpr - 1u) / (uint32_t)cpr;
            for (int e = threadIdx.x; e < 128 * cpr; e += 256) {
                const int rr = (int)(((uint32_t)e * inv) >> 16), ch = e - rr * cpr;
                uint4 vh = make_uint4(0, 0, 0, 0), vl = make_uint4(0, 0, 0, 0);
                if (rr < nrow) {
                    const int off = rr * Kp + ch * 8;
                    vh = *reinterpret_cast<const uint4 *>(th + off);
                    if (NSPLIT == 3) vl = *reinterpret_cast<const uint4 *>(tl + off);
                }
                *reinterpret_cast<uint4 *>(sb_hi + rr * kLdsRow + ch * 8) = vh;
                if (NSPLIT == 3) *reinterpret_cast<uint4 *>(sb_lo + rr * kLdsRow + ch * 8) = vl;
            }
            __syncthreads();
            for (int k0 = 0; k0 < kw; k0 += 32) {
                const mt::bf16x8 a = mt::load8(Ah, r0 + r16, N, Kp, kc0 + k0 + kq);
                mt::bf16x8 b[8];
#pragma unroll
                for (int ct = 0; ct < 8; ++ct)
                    b[ct] = *reinterpret_cast<const mt::bf16x8 *>(sb_hi + (ct * 16 + r16) * kLdsRow + k0 + kq);
#pragma unroll
                for (int ct = 0; ct < 8; ++ct)
                    acc[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[ct], acc[ct], 0, 0, 0);
                if (NSPLIT == 3) {
                    const mt::bf16x8 al = mt::load8(Al, r0 + r16, N, Kp, kc0 + k0 + kq);
#pragma unroll
                    for (int ct = 0; ct < 8; ++ct) {
                        const mt::bf16x8 bl = *reinterpret_cast<const mt::bf16x8 *>(
                            sb_lo + (ct * 16 + r16) * kLdsRow + k0 + kq);
                        acc[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bl, acc[ct], 0, 0, 0);
                        acc[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, b[ct], acc[ct], 0, 0, 0);
                    }
                }
            }
        }
        // the filter in 32-bit indices (N < 2^31) with each row's threshold
        // read once per tile: the same keys and decisions as the row-wise loop
        {
            const int n32 = (int)N, re32 = (int)rend, rb32 = (int)rb;
            const int row0 = (int)r0 + (lane >> 4) * 4;
            float tau[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) tau[i] = s_tau[w][(lane >> 4) * 4 + i];
#pragma unroll
            for (int ct = 0; ct < 8; ++ct) {
                const int col = (int)c0 + ct * 16 + (lane & 15);
                const float nc = col < n32 ? n2[col] : 0.f;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int row = row0 + i;
                    const float key = nc - 2.f * acc[ct][i];
                    if (key <= tau[i] && row < re32 && col < n32 && col != row) {
                        const int at = atomicAdd(&s_cnt[w][(lane >> 4) * 4 + i], 1);
                        if (at < kKnnCap) {
                            bkey[(int64_t)(row - rb32) * kKnnCap + at] = key;
                            bid[(int64_t)(row - rb32) * kKnnCap + at] = col;
                        }
                    }
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
        __builtin_amdgcn_wave_barrier();
        // rows whose buffers passed K + 128 entries: one read per lane, then
        // the rows of the ballot (each merge touches its own row only)
        const int cl = lane < 16 ? s_cnt[w][lane] : 0;
        uint64_t full = __ballot(lane < 16 && cl > K + 128);
        while (full) {
            const int r = __ffsll((unsigned long long)full) - 1;
            full &= full - 1;
            merge_row(r);
        }
    }
    for (int r = 0; r < 16; ++r) merge_row(r);
}

// kNN sweep with the rows' fragments held in registers (Kp <= 256).
// A workgroup of 4 waves owns 4 * RT * 16 rows (RT row tiles of 16 per wave)
// of the call's rows, taken in a given processing order (rowperm), and
// sweeps the column tiles of its split (blockIdx.y) 32 columns at a time.
// The columns come as a copy in group order (node ids bid_of; each group
// padded to whole tiles with id -1 and +inf norms).  A block sweeps the
// tiles of its runs (run_off / run_tile / run_pos / vtot): in the first
// pass the tiles of its own groups, so its thresholds tighten early and few
// later columns pass, in the second only the groups a bound keeps.
// Column tiles stream through a ring of NB LDS stages filled by direct
// global-to-LDS loads (global_load_lds_dwordx4), NB - 1 tiles ahead of the
// tile being multiplied, so the loads' latency hides behind NB - 2 tiles of
// MFMA work; one barrier per tile.  A staged row is CPR + 1 chunks of 16
// bytes (one pad chunk), which spreads a fragment read's 16 rows over
// distinct banks.  Every wave issues the same number of load instructions
// per tile (slots past the tile load a real chunk into the pad area), so a
// fixed vmcnt marks the tile as landed.  The tile's norms and node ids are
// staged beside it (each wave its own copy).
// Per element the epilogue is one fma (key = |x|^2 - 2<u,x>, the order of
// |u-x|^2 for a fixed row u) and one compare against the row's threshold;
// a wave takes the append path only for a 16 x 16 tile where some element
// passes.  Thresholds are the K-th key of the last merge (FLT_MAX until a
// row holds K entries), so every element of the final top-K passes when it
// is seen, whatever the order.  Rows past the call's M get threshold -inf.
// progress of long builds on stderr when the environment sets VJ_LOG (the
// stream is synchronised first, so the time is that of the finished step)
constexpr int64_t kKnnChunk = 16384;  // row blocks per kNN sweep launch
double build_clock() {
    using C = std::chrono::steady_clock;
    static const C::time_point t0 = C::now();
    return std::chrono::duration<double>(C::now() - t0).count();
}
void build_log(hipStream_t s, const char *fmt, ...) {
    static const bool on = std::getenv("VJ_LOG") != nullptr;
    if (!on) return;
    VJ_HIP(hipStreamSynchronize(s));
    char msg[256];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(msg, sizeof msg, fmt, ap);
    va_end(ap);
    std::fprintf(stderr, "[vj %.1fs] %s\n", build_clock(), msg);
    std::fflush(stderr);
}

// order-preserving map of a float key to uint32 (-0 and +0 both map as +0)
__device__ __forceinline__ uint32_t key_bits(float k) {
    const uint32_t b = __float_as_uint(k + 0.0f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// count of elements in the wave (E per lane) for which pred holds
template <int E, typename P>
__device__ __forceinline__ int wave_count(P pred) {
    int c = 0;
#pragma unroll
    for (int j = 0; j < E; ++j) c += __popcll(__ballot(pred(j)));
    return c;
}

// keep the K smallest (key, id) entries of row buffer [off, off + cnt) in
// its first K slots (unordered; the re-rank orders them) and return the
// K-th smallest key (FLT_MAX while fewer than K are held).  A bitwise
// search on order-preserving key bits finds the K-th key T; entries equal
// to T are kept by smallest id (a second bitwise search on the ids).  One
// wave; E * 64 >= kKnnCap.
__device__ __noinline__ float knn_merge_row(float *bkey, int32_t *bid, int64_t off, int cnt,
                                            int K, int lane) {
    constexpr int E = (kKnnCap + 63) / 64;
    const int c = min(cnt, kKnnCap);
    float key[E];
    int id[E];
    uint32_t u[E];
#pragma unroll
    for (int j = 0; j < E; ++j) {
        const int e = j * 64 + lane;
        const bool ok = e < c;
        key[j] = ok ? bkey[off + e] : INFINITY;
        id[j] = ok ? bid[off + e] : 0x7fffffff;
        u[j] = ok ? key_bits(key[j]) : 0xffffffffu;
    }
    if (c <= K) {  // everything is kept
#pragma unroll
        for (int j = 0; j < E; ++j) {
            const int e = j * 64 + lane;
            if (e >= c && e < K) {
                bkey[off + e] = INFINITY;
                bid[off + e] = -1;
            }
        }
        return FLT_MAX;
    }
    // T = the smallest t with #(u <= t) >= K
    uint32_t T = 0;
    for (int bit = 31; bit >= 0; --bit) {
        const uint32_t cand = T | ((1u << bit) - 1u);
        if (wave_count<E>([&](int j) { return u[j] <= cand; }) < K) T |= 1u << bit;
    }
    const int nless = wave_count<E>([&](int j) { return u[j] < T; });
    const int need = K - nless;  // entries equal to T that are kept, >= 1
    // I = the smallest i with #(u == T && id <= i) >= need (ids >= 0)
    int32_t I = 0x7fffffff;
    if (wave_count<E>([&](int j) { return u[j] == T; }) > need) {
        uint32_t t = 0;
        for (int bit = 30; bit >= 0; --bit) {
            const uint32_t cand = t | ((1u << bit) - 1u);
            if (wave_count<E>([&](int j) { return u[j] == T && (uint32_t)id[j] <= cand; }) < need)
                t |= 1u << bit;
        }
        I = (int32_t)t;
    }
    // compact the kept entries into slots [0, K)
    int base = 0;
    float kth = 0.f;
#pragma unroll
    for (int j = 0; j < E; ++j) {
        const bool keep = u[j] < T || (u[j] == T && id[j] <= I);
        const uint64_t m = __ballot(keep);
        const int rank = base + __popcll(m & ((1ull << lane) - 1ull));
        if (keep) {
            bkey[off + rank] = key[j];
            bid[off + rank] = id[j];
        }
        if (u[j] == T) kth = key[j];
        base += __popcll(m);
    }
    // every lane returns T's key (some lane holds an entry equal to T)
    bool h = false;
#pragma unroll
    for (int j = 0; j < E; ++j) h |= u[j] == T;
    const uint64_t hasT = __ballot(h);
    return __shfl(kth, __ffsll((unsigned long long)hasT) - 1);
}

template <int NSPLIT, int KP>
__global__ void __launch_bounds__(256, 2)
k_knn_reg(const uint16_t *Ah, const uint16_t *Al, const int32_t *rowperm, int32_t M,
          const uint16_t *Bh, const uint16_t *Bl, const float *bn2, const int32_t *bid_of,
          const int64_t *__restrict__ run_off, const int32_t *__restrict__ run_tile,
          const int32_t *__restrict__ run_pos, const int32_t *__restrict__ vtot,
          int32_t split_base, const float *tau_in, const int32_t *cnt_in, int K, float *bkey,
          int32_t *bid, int32_t rb, int32_t blk0, const int32_t *order) {
    using S = ring::Shape<NSPLIT, KP>;
    constexpr int RT = S::RT, CT = S::CT, KS = S::KS, BN = S::BN, CPR = S::CPR, SPR = S::SPR;
    constexpr int IPW = S::IPW, TERMS = S::TERMS, PART = S::PART, STAGE = S::STAGE, NB = S::NB;
    constexpr int LPT = S::LPT;
    __shared__ __attribute__((aligned(1024))) char sring[NB * STAGE];
    __shared__ float s_tau[4][RT * 16];
    __shared__ int32_t s_node[4][RT * 16];
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int r16 = lane & 15, kq = (lane >> 4) * 8, rq = (lane >> 4) * 4, grp = lane >> 4;
    // row block (launches may be chunked; order: the blocks in launch order)
    const int32_t blk = order ? order[blk0 + (int32_t)blockIdx.x] : blk0 + (int32_t)blockIdx.x;
    const int32_t prow0 = blk * S::ROWS + w * RT * 16;  // wave's first row (order)
    const int64_t boff = (int64_t)(split_base + blockIdx.y) * M;  // this split's buffer rows
    // the block's tiles are runs [run_off[blk], run_off[blk + 1]): run k
    // covers positions [run_pos[k], next run's start or vtot[blk]) from tile
    // run_tile[k] on; split y of gridDim.y sweeps positions [jb, je)
    const int64_t k0 = run_off[blk], k1 = run_off[blk + 1];
    const int32_t V = vtot[blk];
    const int32_t tps = (V + (int32_t)gridDim.y - 1) / (int32_t)gridDim.y;
    const int32_t jb = min(V, (int32_t)blockIdx.y * tps), je = min(V, jb + tps);
    const int ntile = je - jb;
    // the run holding position jb (the last one starting at or before it)
    int64_t rk = k0;
    if (ntile > 0) {
        int64_t lo = k0, hi = k1 - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            if (run_pos[mid] <= jb) lo = mid; else hi = mid - 1;
        }
        rk = lo;
    }
    int32_t rdelta = ntile > 0 ? run_tile[rk] - run_pos[rk] : 0;  // tile - position in run rk
    int32_t rend = ntile > 0 ? (rk + 1 < k1 ? run_pos[rk + 1] : V) : 0;
    int32_t pnext = jb;  // the next position issued (positions are issued in order)
    const int32_t first_col = ntile > 0 ? (jb + rdelta) * BN : 0;
    // a row is cut back to K once it holds more than merge_at entries: the
    // threshold then tightens early, which keeps the appends few
    const int merge_at = min(K + 96, kKnnCap - BN);
    // entries held by the wave's row r: lane r of cnt (a later pass goes on
    // with the lists an earlier one left: cnt_in entries, threshold tau_in)
    int cnt = 0;
    if (lane < RT * 16) {
        const int32_t node = prow0 + lane < M ? rowperm[prow0 + lane] : -1;
        s_node[w][lane] = node;
        s_tau[w][lane] = node < 0 ? -INFINITY : tau_in ? tau_in[prow0 + lane] : FLT_MAX;
        if (cnt_in && node >= 0) cnt = cnt_in[prow0 + lane];
    }

    // the wave's rows: fragment (rt, ks) holds row rt*16 + (lane & 15),
    // dimensions ks*32 + (lane >> 4)*8 .. +7
    mt::bf16x8 a[RT][KS], al[NSPLIT == 3 ? RT : 1][NSPLIT == 3 ? KS : 1];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
        const int32_t pr = prow0 + rt * 16 + r16;
        const int32_t node = pr < M ? rowperm[pr] : -1;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            a[rt][ks] = mt::load8(Ah, node < 0 ? 0 : node, node < 0 ? 0 : node + 1, KP, ks * 32 + kq);
            if (NSPLIT == 3)
                al[rt][ks] = mt::load8(Al, node < 0 ? 0 : node, node < 0 ? 0 : node + 1, KP, ks * 32 + kq);
        }
    }

    // loads of the tile at column c0 into stage st: slot s of a part is
    // row s / SPR, chunk s % SPR; pad chunks and slots past the tile load
    // the tile's first chunk.  A lane's slots are the same in every tile, so
    // their byte offsets from the tile's first row are fixed.
    const uint32_t ring0 = ring::lds_byte_addr(sring);
    uint32_t soff[IPW];
#pragma unroll
    for (int j = 0; j < IPW; ++j) {
        const int sl = (w * IPW + j) * 64 + lane;
        const int rr = sl / SPR, ch = sl - rr * SPR;
        const bool real = rr < BN && ch < CPR;
        soff[j] = real ? (uint32_t)((rr * KP + ch * 8) * 2) : 0u;
    }
    const uint32_t soff4 = (uint32_t)((lane < BN ? lane : 0) * 4);
    auto issue = [&](int32_t c0, int st) {
        const uint32_t sbase = ring0 + (uint32_t)(st * STAGE);
        const char *th = reinterpret_cast<const char *>(Bh + (int64_t)c0 * KP);
        const char *tl = NSPLIT == 3 ? reinterpret_cast<const char *>(Bl + (int64_t)c0 * KP) : nullptr;
#pragma unroll
        for (int j = 0; j < IPW; ++j) {
            const uint32_t dst = sbase + (uint32_t)((w * IPW + j) * 1024);
            ring::lds_dma16(th, soff[j], dst);
            if (NSPLIT == 3) ring::lds_dma16(tl, soff[j], dst + PART);
        }
        ring::lds_dma4(bn2 + c0, soff4, sbase + TERMS * PART + w * 256);
        ring::lds_dma4(bid_of + c0, soff4, sbase + TERMS * PART + 1024 + w * 256);
    };
    // column of the next position (in order; past the split's last one the
    // first tile's column, loaded into a stage no tile reads)
    auto next_col = [&]() -> int32_t {
        while (pnext >= rend) {
            ++rk;
            rdelta = run_tile[rk] - run_pos[rk];
            rend = rk + 1 < k1 ? run_pos[rk + 1] : V;
        }
        return (pnext++ + rdelta) * BN;
    };

    float tau[RT][4];
    auto load_tau = [&]() {
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int i = 0; i < 4; ++i) tau[rt][i] = s_tau[w][rt * 16 + rq + i];
    };
    auto merge = [&](int r) {
        const int c = __builtin_amdgcn_readlane(cnt, r);
        const int32_t node = s_node[w][r];
        const float kth = knn_merge_row(bkey, bid, (boff + (node - rb)) * kKnnCap, c, K, lane);
        cnt = lane == r ? min(c, K) : cnt;
        if (lane == 0) s_tau[w][r] = fminf(s_tau[w][r], kth);
    };

    // prologue: tiles 0 .. NB-2 in flight (every wave issues LPT loads per
    // tile slot, a slot past the last tile re-loads tile 0's stage 0 data
    // into the last stage, which no tile reads before it is re-issued)
#pragma unroll
    for (int p = 0; p < NB - 1; ++p)
        issue(p < ntile ? next_col() : first_col, p < ntile ? p : NB - 1);
    for (int it = 0; it < ntile; ++it) {
        const int st = it % NB;
        // tile it has landed when at most (NB - 2) tiles' loads are in
        // flight: loads complete in issue order, and the appends' stores
        // issued since only add to the count, so they can only make this
        // wait longer
        ring::wait_barrier<(NB - 2) * LPT>();
        if (it == 0) load_tau();
        {
            const int nx = it + NB - 1;  // into the stage read at it - 1
            issue(nx < ntile ? next_col() : first_col, nx < ntile ? nx % NB : (it + NB - 1) % NB);
        }
        const char *sp = sring + st * STAGE;
        floatx4 acc[RT][CT];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) acc[rt][ct] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            mt::bf16x8 b[CT], bl[NSPLIT == 3 ? CT : 1];
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) {
                const int off = ((ct * 16 + r16) * SPR + ks * 4 + (lane >> 4)) * 16;
                b[ct] = *reinterpret_cast<const mt::bf16x8 *>(sp + off);
                if (NSPLIT == 3) bl[ct] = *reinterpret_cast<const mt::bf16x8 *>(sp + PART + off);
            }
#pragma unroll
            for (int ct = 0; ct < CT; ++ct)
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) {
                    acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[rt][ks], b[ct], acc[rt][ct], 0, 0, 0);
                    if (NSPLIT == 3) {
                        acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[rt][ks], bl[ct], acc[rt][ct], 0, 0, 0);
                        acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[rt][ks], b[ct], acc[rt][ct], 0, 0, 0);
                    }
                }
        }
        // epilogue: the keys (in place of the products) and one pass test
        // for the whole step; only a step with a passing element looks at
        // its 16 x 16 tiles and appends (rare once the rows hold K)
        const float *snc = reinterpret_cast<const float *>(sp + TERMS * PART + w * 256);
        const int32_t *sid = reinterpret_cast<const int32_t *>(sp + TERMS * PART + 1024 + w * 256);
        float nc[CT];
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) nc[ct] = snc[ct * 16 + r16];  // +inf past the last node
#pragma unroll
        for (int ct = 0; ct < CT; ++ct)
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int i = 0; i < 4; ++i) acc[rt][ct][i] = fmaf(-2.f, acc[rt][ct][i], nc[ct]);
        // a row passes somewhere iff the smallest of its keys does (fminf is
        // exact): one compare per row and lane, its wave mask (the compare's
        // own SGPR result) or-ed into one, no per-element masks kept
        uint64_t pass_mask = 0;
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                float m = acc[rt][0][i];
#pragma unroll
                for (int ct = 1; ct < CT; ++ct) m = fminf(m, acc[rt][ct][i]);
                pass_mask |= __ballot(m <= tau[rt][i]);
            }
        bool appended = false;
        if (pass_mask) {
            appended = true;
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) {
                const int32_t col = sid[ct * 16 + r16];  // node id of the lane's column
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) {
                    bool hit = false;
#pragma unroll
                    for (int i = 0; i < 4; ++i) hit |= acc[rt][ct][i] <= tau[rt][i];
                    if (!__ballot(hit)) continue;
                    // per row (rt*16 + 4g + i of lane group g) the passing
                    // lanes' slots: the row's count (lane r of cnt) plus the
                    // lane's rank among its group's passing lanes
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int32_t node = s_node[w][rt * 16 + rq + i];
                        const bool ok = acc[rt][ct][i] <= tau[rt][i] && col >= 0 && col != node;
                        const uint64_t m = __ballot(ok);
                        if (!m) continue;
                        int at = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                           __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
#pragma unroll
                        for (int g = 0; g < 4; ++g) {
                            const int r = rt * 16 + 4 * g + i;
                            const int below = __popcll(m & ((1ull << (16 * g)) - 1ull));
                            const int here = __popcll((m >> (16 * g)) & 0xffffull);
                            const int base = __builtin_amdgcn_readlane(cnt, r);
                            cnt = lane == r ? base + here : cnt;
                            at += grp == g ? base - below : 0;
                        }
                        if (ok && at < kKnnCap) {
                            const int64_t o = (boff + (node - rb)) * kKnnCap + at;
                            bkey[o] = acc[rt][ct][i];
                            bid[o] = col;
                        }
                    }
                }
            }
        }
        if (appended) {
            // rows that could not take another full tile: cut to K
            uint64_t full = __ballot(lane < RT * 16 && cnt > merge_at);
            if (full) {
                // the appends' stores complete before the merges read them
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
                __builtin_amdgcn_wave_barrier();
                while (full) {
                    const int r = __ffsll((unsigned long long)full) - 1;
                    full &= full - 1;
                    merge(r);
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
                __builtin_amdgcn_wave_barrier();
                load_tau();
            }
        }
    }
    // every load in flight lands before the workgroup ends
    ring::wait_barrier<0>();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
    __builtin_amdgcn_wave_barrier();
    for (int r = 0; r < RT * 16; ++r)
        if (s_node[w][r] >= 0) merge(r);
}

// one round of the split merge: group g of row i merges lists b + j * step
// (j < G, list index < S; b = g * G * step; list s of row i at
// (s * M + i) * kKnnCap, its first K entries) into list b's first K
// entries, by (key, id); one wave per (row, group), G * K <= 512
__global__ void __launch_bounds__(256)
k_knn_merge_splits(float *bkey, int32_t *bid, int64_t M, int S, int K, int G, int step) {
    const int lane = threadIdx.x & 63;
    const int ng = (S + G * step - 1) / (G * step);
    const int64_t wv = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t i = wv / ng;
    if (i >= M) return;
    const int b = (int)(wv - i * ng) * G * step;
    float key[8];
    int id[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int e = j * 64 + lane;
        const int jl = e / K, k = e - jl * K;
        const int sp = b + jl * step;
        const bool ok = jl < G && sp < S;
        const int64_t o = ((int64_t)sp * M + i) * kKnnCap + k;
        key[j] = ok ? bkey[o] : INFINITY;
        id[j] = ok ? bid[o] : 0x7fffffff;
        if (ok && id[j] < 0) { key[j] = INFINITY; id[j] = 0x7fffffff; }
    }
    mt::wave_sort<8>(key, id, lane);
    const int64_t ob = ((int64_t)b * M + i) * kKnnCap;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int e = j * 64 + lane;
        if (e < K) {
            const bool ok = key[j] < INFINITY;
            bkey[ob + e] = key[j];
            bid[ob + e] = ok ? id[j] : -1;
        }
    }
}

// starting thresholds of a later pass: the K-th key of each row's list 0,
// i.e. the largest of its K kept entries (kept unordered or sorted),
// FLT_MAX while it holds fewer than K, and the number of entries held (the
// first cnt slots; the rest hold id -1); by processing position (rowperm[pos]
// is row rb + i of list 0)
__global__ void k_list_tau(const float *bkey, const int32_t *bid, const int32_t *rowperm,
                           int64_t M, int64_t rb, int K, float *tau, int32_t *cnt) {
    const int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (pos >= M) return;
    const int64_t o = ((int64_t)rowperm[pos] - rb) * kKnnCap;
    float t = -FLT_MAX;
    int c = 0;
    for (int e = 0; e < K; ++e) {
        const bool ok = bid[o + e] >= 0;
        t = ok ? fmaxf(t, bkey[o + e]) : FLT_MAX;
        c += ok;
    }
    tau[pos] = t;
    cnt[pos] = c;
}

// distance bound of each row's list (rows by processing position; cert
// indexed by row - rb): every node outside the K kept entries has a key >=
// the K-th key t, so its squared distance is >= t + |r|^2 less the key's
// error bound (ea, eb, maxn as in k_visit_groups) and the rounding of that
// sum; +inf while the row holds fewer than K (every node is in the list)
__global__ void k_list_cert(const float *bkey, const int32_t *bid, const int32_t *rowperm,
                            int64_t M, int64_t rb, int K, const float *n2, float ea, float eb,
                            float maxn, float *cert) {
    const int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (pos >= M) return;
    const int32_t node = rowperm[pos];
    const int64_t o = ((int64_t)node - rb) * kKnnCap;
    float t = -FLT_MAX;
    for (int e = 0; e < K; ++e) t = bid[o + e] >= 0 ? fmaxf(t, bkey[o + e]) : FLT_MAX;
    const float nr2 = n2[node], nr = sqrtf(nr2);
    const float E = 2.f * (ea * nr * maxn + eb * (maxn * maxn + nr * maxn + nr2)) +
                    4.f * FLT_EPSILON * (fabsf(t) + nr2);
    cert[node - rb] = t >= FLT_MAX ? INFINITY : fmaxf(0.f, (t + nr2 - E) * (1.f - 1e-4f));
}

// an insertion's changing rows: every old node that receives an offer and
// every new node (flag), then their ids at the flags' scan positions
__global__ void k_changed_flags(const int32_t *indeg, int64_t n_old, int64_t N, int32_t *flag) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < N) flag[v] = v >= n_old || indeg[v] > 0;
}
__global__ void k_scatter_flagged(const int32_t *flag, const int64_t *pos, int64_t N,
                                  int32_t *rows) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < N && flag[v]) rows[pos[v]] = (int32_t)v;
}

// reverse offers of the forward lists of rows [rb, rb + M) (fwd indexed from rb)
__global__ void k_scatter_rev(int64_t M, int R, const int32_t *fwd, const float *fwd_d2,
                              const int64_t *roff, int32_t *rpos, int32_t *rid, float *rd2,
                              int64_t rb) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= M * R) return;
    const int32_t v = fwd[e];
    if (v < 0) return;
    const int64_t u = rb + e / R;
    const int at = atomicAdd(&rpos[v], 1);
    rid[roff[v] + at] = (int32_t)u;
    rd2[roff[v] + at] = fwd_d2[e];
}

// ------------------------------------------------------- entry point --
__global__ void k_centroid(const float *vec, int64_t N, int dp, double *sum) {
    const int c = blockIdx.y * blockDim.x + threadIdx.x;
    if (c >= dp) return;
    double acc = 0.0;
    for (int64_t r = blockIdx.x; r < N; r += gridDim.x) acc += (double)vec[r * dp + c];
    atomicAdd(&sum[c], acc);
}

__global__ void k_centroid_dist(const float *vec, int64_t N, int dp, const double *sum,
                                double *dist, unsigned long long *best) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long key = ~0ull;  // non-negative doubles order as their bits
    if (r < N) {
        double acc = 0.0;
        for (int c = 0; c < dp; ++c) {
            const double t = (double)vec[r * dp + c] - sum[c] / (double)N;
            acc += t * t;
        }
        dist[r] = acc;
        key = (unsigned long long)__double_as_longlong(acc);
    }
    // one atomic per wave
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(key, off);
        key = o < key ? o : key;
    }
    if ((threadIdx.x & 63) == 0 && key != ~0ull) atomicMin(best, key);
}

__global__ void k_argmin_id(const double *dist, int64_t N, const unsigned long long *best,
                            int *id) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= N) return;
    if ((unsigned long long)__double_as_longlong(dist[r]) == *best) atomicMin(id, (int)r);
}

// ------------------------------------------------------ connectivity --
// one BFS level: every edge of the front; a node seen first here goes to the
// next front (one counter atomic per wave).  A plain read skips the nodes
// already seen (seen only goes from 0 to 1 within a BFS, so a stale 0 only
// leads to the exchange, which decides), and the exchange claims each new
// node for exactly one edge.
__global__ void k_bfs_step(const int32_t *adj, int R, const int32_t *front, int nf, int *seen,
                           int32_t *next, int *nnext) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int32_t v = -1;
    if (t < (int64_t)nf * R) v = adj[(int64_t)front[t / R] * R + t % R];
    const bool fresh = v >= 0 && __atomic_load_n(&seen[v], __ATOMIC_RELAXED) == 0 &&
                       atomicExch(&seen[v], 1) == 0;
    const unsigned long long m = __ballot(fresh);
    if (m == 0) return;
    const int lane = threadIdx.x & 63;
    int base = 0;
    if (lane == 0) base = atomicAdd(nnext, __popcll(m));
    base = __shfl(base, 0);
    if (fresh) next[base + __popcll(m & ((1ull << lane) - 1))] = v;
}

// smallest unseen node in [from, N), grid-stride: a thread's first unseen
// index is its smallest, the workgroup's minimum goes out with one atomic
__global__ void __launch_bounds__(256)
k_first_unseen(const int *seen, int64_t from, int64_t N, int *first) {
    __shared__ int s_min[4];
    int best = 0x7fffffff;
    for (int64_t r = from + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < N;
         r += (int64_t)gridDim.x * blockDim.x)
        if (!seen[r]) { best = (int)r; break; }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) best = min(best, __shfl_xor(best, off));
    if ((threadIdx.x & 63) == 0) s_min[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        best = min(min(s_min[0], s_min[1]), min(s_min[2], s_min[3]));
        if (best != 0x7fffffff) atomicMin(first, best);
    }
}

// the repair loop's device-side state (one copy, read back once per step)
struct RepairCtl {
    int first;                     // smallest unseen node (INT_MAX: none)
    int nnext;                     // BFS: size of the next front
    unsigned long long best_any;   // (d2 bits << 32 | id) of the nearest reached node
    unsigned long long best_free;  // the same among nodes with a free slot
    int certified;                 // best_free is known: no scan
    int pad;
    int64_t scan_from;             // else the nodes [scan_from, N) to scan
};

__global__ void k_repair_reset(RepairCtl *c) {
    c->first = 0x7fffffff;
    c->nnext = 0;
    c->best_any = ~0ull;
    c->best_free = ~0ull;
    c->certified = 0;
    c->scan_from = 0;
}

// the nearest free reached node to w = c->first from w's own sorted list
// (kc entries by (d2, id), d2 in the scan's arithmetic) among the nodes
// [0, from[w]) that existed when the list was made: every one of those
// outside the list is at squared distance >= cert[w] (the kNN sweep's K-th
// key turned into a distance bound; -inf: w has no list), so a first reached
// free entry closer than that is the answer among them.  Nodes added since
// (from[w] < N) are left to a scan of [from[w], N).  Rows [0, n) have
// lists; one wave.
__global__ void k_repair_from_list(const int32_t *kid, const float *kd2, int kc, const float *cert,
                                   const int32_t *from, int64_t n, int64_t N, const int *seen,
                                   const int32_t *adj, int R, RepairCtl *c) {
    const int32_t w = c->first;
    if (w == 0x7fffffff || w >= n) return;
    const int lane = threadIdx.x;
    const int64_t row = w;
    const float bound = cert[row];
    if (!(bound > -INFINITY)) return;
    for (int e0 = 0; e0 < kc; e0 += 64) {
        const int e = e0 + lane;
        const int32_t v = e < kc ? kid[row * kc + e] : -1;
        const bool hit = v >= 0 && seen[v] && adj[(int64_t)v * R + R - 1] < 0;
        const unsigned long long m = __ballot(hit);
        if (m) {
            const int f = __ffsll((unsigned long long)m) - 1;
            if (lane == f) {
                const float d = kd2[row * kc + e];
                if (d < bound) {
                    c->best_free = ((unsigned long long)__float_as_uint(d) << 32) | (uint32_t)v;
                    if (from[row] >= N) c->certified = 1;
                    else c->scan_from = from[row];
                }
            }
            return;
        }
    }
}

// BFS seed: start is seen, the front is {start}
__global__ void k_bfs_seed(int *seen, int32_t *front, int32_t start, RepairCtl *c) {
    seen[start] = 1;
    front[0] = start;
    c->nnext = 0;
}

__global__ void k_zero_nnext(RepairCtl *c) { c->nnext = 0; }

// nearest reached node to w: overall and among nodes with a free slot;
// results packed as (float bits << 32 | id) so atomicMin gives (d2, id) order.
// 8 lanes per node (16-byte loads), 8 nodes per wave, one atomic per wave.
__device__ __forceinline__ unsigned long long min_u64(unsigned long long a, unsigned long long b) {
    return a < b ? a : b;
}

// one lane's share of |a - b|^2 over float4 chunks p8, p8 + 8, ... (8 lanes
// per node; the caller sums the 8 lanes with xor shuffles 4, 2, 1): every
// repair kernel uses this order, so equal inputs give equal bits
__device__ __forceinline__ float d2_part(const float4 *a, const float4 *b, int nc4, int p8) {
    float acc = 0.f;
    for (int c = p8; c < nc4; c += 8) {
        const float4 x = a[c], y = b[c];
        float t = x.x - y.x; acc = fmaf(t, t, acc);
        t = x.y - y.y; acc = fmaf(t, t, acc);
        t = x.z - y.z; acc = fmaf(t, t, acc);
        t = x.w - y.w; acc = fmaf(t, t, acc);
    }
    return acc;
}
__device__ __forceinline__ float sum8(float acc) {
#pragma unroll
    for (int off = 4; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    return acc;
}

__global__ void __launch_bounds__(256)
k_nearest_reached(const float *vec, int64_t N, int dp, const int *wp, const int *seen,
                  const int32_t *adj, int R, const int *skip, const int64_t *from,
                  unsigned long long *best_any, unsigned long long *best_free) {
    // 8 lanes per node, 32 nodes per workgroup step, grid-stride over the
    // nodes [*from, N); one atomic per workgroup (the minimum of unique
    // (d2, id) keys does not depend on the order).  w (*wp) INT_MAX or *skip
    // (the answer is known): nothing to do.
    __shared__ unsigned long long s_a[4], s_f[4];
    const int32_t w = *wp;
    if (w == 0x7fffffff || *skip) return;
    const int lane = threadIdx.x & 63;
    const int g = lane >> 3, p8 = lane & 7;
    const float4 *b = reinterpret_cast<const float4 *>(vec + (int64_t)w * dp);
    unsigned long long ka = ~0ull, kf = ~0ull;
    const int64_t stride = (int64_t)gridDim.x * 32;
    const int64_t p0 = *from;
    for (int64_t base = p0 + (int64_t)blockIdx.x * 32; base < N; base += stride) {
        const int64_t p = base + (threadIdx.x >> 6) * 8 + g;
        const bool ok = p < N && seen[p];
        float acc = 0.f;
        if (ok) acc = d2_part(reinterpret_cast<const float4 *>(vec + p * dp), b, dp / 4, p8);
        acc = sum8(acc);
        if (ok) {
            const unsigned long long key = ((unsigned long long)__float_as_uint(acc) << 32) | (uint32_t)p;
            ka = min_u64(ka, key);
            if (adj[p * R + R - 1] < 0) kf = min_u64(kf, key);
        }
    }
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        ka = min_u64(ka, __shfl_xor(ka, off));
        kf = min_u64(kf, __shfl_xor(kf, off));
    }
    if (lane == 0) {
        s_a[threadIdx.x >> 6] = ka;
        s_f[threadIdx.x >> 6] = kf;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < 4; ++i) {
            ka = min_u64(ka, s_a[i]);
            kf = min_u64(kf, s_f[i]);
        }
        if (ka != ~0ull) atomicMin(best_any, ka);
        if (kf != ~0ull) atomicMin(best_free, kf);
    }
}

// put w into row p (free slot, else the last = longest slot), then re-sort
// the row by (d2, id); one wave
__global__ void k_attach(const float *vec, int dp, int32_t *adj, int R, int32_t p, int32_t w) {
    __shared__ float s_d[64];
    __shared__ int32_t s_i[64];
    const int lane = threadIdx.x;
    int32_t *row = adj + (int64_t)p * R;
    int deg = 0;
    for (int j = 0; j < R; ++j) deg += row[j] >= 0;
    const int slot = deg < R ? deg : R - 1;
    int32_t v = lane < R ? row[lane] : -1;
    if (lane == slot) v = w;
    float acc = INFINITY;
    if (v >= 0) {
        acc = 0.f;
        for (int c = 0; c < dp; ++c) {
            const float t = vec[(int64_t)p * dp + c] - vec[(int64_t)v * dp + c];
            acc = fmaf(t, t, acc);
        }
    }
    float key[1] = {acc};
    int id[1] = {v >= 0 ? v : 0x7fffffff};
    mt::wave_sort<1>(key, id, lane);
    if (lane < R) row[lane] = key[0] < INFINITY ? id[0] : -1;
    (void)s_d;
    (void)s_i;
}


}  // namespace

// row-width instantiations of the row kernels (build_inst.hip)
#define VJ_BUILD_WIDTHS(X) X(32) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) X(1024)
#define VJ_DECL(dp)                                                                         \
    void build_rows_##dp(const float *, int64_t, int, int, int, const int32_t *, int32_t *,  \
                         float *, int32_t *, float *, int32_t *, int32_t *, int64_t,         \
                         int64_t, hipStream_t);                                              \
    void build_rev_##dp(const float *, int64_t, int, const int32_t *, const float *,         \
                        const int32_t *, const int64_t *, const int32_t *, const float *,    \
                        int32_t *, const int32_t *, hipStream_t);                            \
    void build_gather_##dp(const float *, int, const int32_t *, const int32_t *,             \
                           const int32_t *, int64_t, const int32_t *, int64_t, int32_t *,    \
                           float *, int32_t *, hipStream_t);
VJ_BUILD_WIDTHS(VJ_DECL)
#undef VJ_DECL

namespace {

void launch_rows(int dp, const float *vec, int64_t N, int R, int K, int Kc, const int32_t *bid,
                 int32_t *kid, float *kd2, int32_t *fwd, float *fwd_d2, int32_t *fdeg,
                 int32_t *indeg, int64_t rb, int64_t M, hipStream_t s) {
    switch (dp) {
#define VJ_CASE(w) case w: build_rows_##w(vec, N, R, K, Kc, bid, kid, kd2, fwd, fwd_d2, fdeg, indeg, rb, M, s); return;
        VJ_BUILD_WIDTHS(VJ_CASE)
#undef VJ_CASE
    default: VJ_CHECK(false, VJ_ERR_UNSUPPORTED, "row width");
    }
}

void launch_rev(int dp, const float *vec, int64_t M, int R, const int32_t *fwd,
                const float *fwd_d2, const int32_t *fdeg, const int64_t *roff,
                const int32_t *rid, const float *rd2, int32_t *adj, const int32_t *rows,
                hipStream_t s) {
    switch (dp) {
#define VJ_CASE(w) case w: build_rev_##w(vec, M, R, fwd, fwd_d2, fdeg, roff, rid, rd2, adj, rows, s); return;
        VJ_BUILD_WIDTHS(VJ_CASE)
#undef VJ_CASE
    default: VJ_CHECK(false, VJ_ERR_UNSUPPORTED, "row width");
    }
}

void launch_gather(int dp, const float *vec, int R, const int32_t *adj, const int32_t *fwd_new,
                   const int32_t *fdeg_new, int64_t n_old, const int32_t *rows, int64_t M,
                   int32_t *fwd, float *fwd_d2, int32_t *fdeg, hipStream_t s) {
    switch (dp) {
#define VJ_CASE(w) case w: build_gather_##w(vec, R, adj, fwd_new, fdeg_new, n_old, rows, M, fwd, fwd_d2, fdeg, s); return;
        VJ_BUILD_WIDTHS(VJ_CASE)
#undef VJ_CASE
    default: VJ_CHECK(false, VJ_ERR_UNSUPPORTED, "row width");
    }
}

// ---- group order of the kNN sweep
// The nodes are grouped by their nearest of P centres (P <= kMaxGroups;
// centres: every (N / P)-th node, moved to its group's mean lloyd_steps(N)
// times),
// rows and columns are sorted by group, and each group starts a tile.  The
// sweep of a row block runs in two passes: its own groups first, whose
// lists give every row a threshold tau (its K-th key), then only the groups
// that a row of the block could still take a member from.  Group g has
// centre m_g and radius rad_g (no member farther from m_g); by the triangle
// inequality every member c has |r - c| >= |r - m_g| - rad_g, so when that
// bound, less the tile key's error bound, puts every member's key above tau
// for every row of the block, no member of g would enter a list: skipping g
// leaves the lists exactly as the full sweep leaves them.
constexpr int64_t kGroupRows = 512;  // nodes per group (on average, at most kMaxGroups)
constexpr int kMaxGroups = 4096;
// mean steps of the centres before the last labelling: one, two from 4M
// nodes on (where the tighter groups save more sweep than a step costs)
inline int lloyd_steps(int64_t N) { return N >= 4000000 ? 2 : 1; }

// Distances of rows to centres, eight lanes per row: lane p8 of a row's
// group holds float4 slices p8, p8 + 8, ... (NCHL = dp / 32 of them) of two
// rows in registers; a chunk of 32 centres is staged in LDS.  Each lane
// sums its slices for all 32 centres, then three exchange steps (xor 4, 2,
// 1) leave lane p8 with the totals of centres 4 p8 .. 4 p8 + 3.
template <int NCHL>
struct RowPair {
    float4 a[NCHL], b[NCHL];
    __device__ void load(const float *xa, const float *xb, int p8) {
#pragma unroll
        for (int j = 0; j < NCHL; ++j) {
            a[j] = reinterpret_cast<const float4 *>(xa)[j * 8 + p8];
            b[j] = reinterpret_cast<const float4 *>(xb)[j * 8 + p8];
        }
    }
    // totals of centres 4 p8 + i (i < 4) for both rows
    __device__ void dist(const float *sp, int p8, float (&da)[4], float (&db)[4]) const {
        constexpr int dp = NCHL * 32;
        float pa[32], pb[32];
#pragma unroll
        for (int k = 0; k < 32; ++k) { pa[k] = 0.f; pb[k] = 0.f; }
#pragma unroll
        for (int k = 0; k < 32; ++k)
#pragma unroll
            for (int j = 0; j < NCHL; ++j) {
                const float4 c = reinterpret_cast<const float4 *>(sp + k * dp)[j * 8 + p8];
                float t = a[j].x - c.x; pa[k] = fmaf(t, t, pa[k]);
                t = a[j].y - c.y; pa[k] = fmaf(t, t, pa[k]);
                t = a[j].z - c.z; pa[k] = fmaf(t, t, pa[k]);
                t = a[j].w - c.w; pa[k] = fmaf(t, t, pa[k]);
                t = b[j].x - c.x; pb[k] = fmaf(t, t, pb[k]);
                t = b[j].y - c.y; pb[k] = fmaf(t, t, pb[k]);
                t = b[j].z - c.z; pb[k] = fmaf(t, t, pb[k]);
                t = b[j].w - c.w; pb[k] = fmaf(t, t, pb[k]);
            }
        reduce_scatter(pa, p8);
        reduce_scatter(pb, p8);
#pragma unroll
        for (int i = 0; i < 4; ++i) { da[i] = pa[i]; db[i] = pb[i]; }
    }
    // step with mask m keeps the half of v[0 .. 2h) selected by lane bit m
    // and adds the partner's copy of it
    __device__ static void reduce_scatter(float (&v)[32], int p8) {
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            const int m = 4 >> s, h = 16 >> s;
            const bool up = (p8 & m) != 0;
#pragma unroll
            for (int i = 0; i < h; ++i) {
                const float send = up ? v[i] : v[i + h];
                const float keep = up ? v[i + h] : v[i];
                v[i] = keep + __shfl_xor(send, m);
            }
        }
    }
};

// stage centres p0 .. p0 + np - 1 (np <= 32) into sp; past np, +inf rows
__device__ __forceinline__ void stage_centres(const float *cen, int p0, int np, int dp, float *sp) {
    for (int e = threadIdx.x; e < 32 * dp; e += blockDim.x)
        sp[e] = e < np * dp ? cen[(int64_t)p0 * dp + e] : INFINITY;
}

// nearest of P centres (fp32 L2; the smaller index on ties) for every node,
// 64 nodes per workgroup (dp = 32 NCHL <= 256).  With one slice of centres
// (gridDim.y = 1) the label goes to assign and, with rad, the group's
// radius grows to the node's distance (non-negative floats order as their
// bits).  With several, slice y covers centre words [y wps, (y + 1) wps) and
// each node's best goes to best[v] as (d2 bits << 32 | index) by atomicMin,
// for k_assign_finish.
template <int NCHL>
__global__ void __launch_bounds__(256, 3)
k_assign_pivot(const float *vec, int64_t N, const float *piv, int P, int wps, int32_t *assign,
               float *rad, unsigned long long *best) {
    constexpr int dp = NCHL * 32;
    __shared__ __attribute__((aligned(16))) float sp[32 * dp];
    const int p8 = threadIdx.x & 7, grp = threadIdx.x >> 3;
    const int64_t va = (int64_t)blockIdx.x * 64 + grp, vb = va + 32;
    RowPair<NCHL> rp;
    rp.load(vec + (va < N ? va : 0) * dp, vec + (vb < N ? vb : 0) * dp, p8);
    float ba = INFINITY, bb = INFINITY;
    int ia = 0, ib = 0;
    const int pe = min(P, (int)(blockIdx.y + 1) * wps * 32);
    for (int p0 = blockIdx.y * wps * 32; p0 < pe; p0 += 32) {
        __syncthreads();
        stage_centres(piv, p0, min(32, pe - p0), dp, sp);
        __syncthreads();
        float da[4], db[4];
        rp.dist(sp, p8, da, db);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int g = p0 + 4 * p8 + i;  // staged +inf rows never win
            if (da[i] < ba) { ba = da[i]; ia = g; }
            if (db[i] < bb) { bb = db[i]; ib = g; }
        }
    }
    // the smallest (d2, index) over the row's eight lanes
#pragma unroll
    for (int m = 4; m > 0; m >>= 1) {
        const float oa = __shfl_xor(ba, m), ob = __shfl_xor(bb, m);
        const int ja = __shfl_xor(ia, m), jb = __shfl_xor(ib, m);
        if (oa < ba || (oa == ba && ja < ia)) { ba = oa; ia = ja; }
        if (ob < bb || (ob == bb && jb < ib)) { bb = ob; ib = jb; }
    }
    if (p8 != 0) return;
    if (best) {
        if (va < N && ba < INFINITY)
            atomicMin(best + va, ((unsigned long long)__float_as_uint(ba) << 32) | (uint32_t)ia);
        if (vb < N && bb < INFINITY)
            atomicMin(best + vb, ((unsigned long long)__float_as_uint(bb) << 32) | (uint32_t)ib);
        return;
    }
    if (va < N) {
        assign[va] = ia;
        if (rad) atomicMax(reinterpret_cast<unsigned int *>(rad) + ia, __float_as_uint(sqrtf(ba)));
    }
    if (vb < N) {
        assign[vb] = ib;
        if (rad) atomicMax(reinterpret_cast<unsigned int *>(rad) + ib, __float_as_uint(sqrtf(bb)));
    }
}

// labels (and radii) from the slices' packed minima
__global__ void k_assign_finish(const unsigned long long *best, int64_t N, int32_t *assign,
                                float *rad) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= N) return;
    const unsigned long long k = best[v];
    const int32_t g = (int32_t)(uint32_t)k;
    assign[v] = g;
    if (rad)
        atomicMax(reinterpret_cast<unsigned int *>(rad) + g,
                  __float_as_uint(sqrtf(__uint_as_float((uint32_t)(k >> 32)))));
}

// centre of each non-empty group: the mean of its members (sweep positions
// [gstart, gend) of perm); an empty group keeps its centre.  Lanes split
// the float4 columns and the members; the parts meet in LDS.
__global__ void __launch_bounds__(256)
k_center_means(const float *vec, int dp, const int32_t *perm, const int32_t *gstart,
               const int32_t *gend, float *cen) {
    __shared__ float4 part[256];
    const int g = blockIdx.x;
    const int j0 = gstart[g], j1 = gend[g];
    if (j0 < 0 || j1 <= j0) return;
    const int nc4 = dp / 4, lanes = 256 / nc4;
    const int c = threadIdx.x % nc4, m = threadIdx.x / nc4;
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    if (m < lanes)
        for (int j = j0 + m; j < j1; j += lanes) {
            const float4 x = reinterpret_cast<const float4 *>(vec + (int64_t)perm[j] * dp)[c];
            acc.x += x.x; acc.y += x.y; acc.z += x.z; acc.w += x.w;
        }
    part[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x < nc4) {
        float4 t = make_float4(0.f, 0.f, 0.f, 0.f);
        for (int k = 0; k < lanes; ++k) {
            const float4 y = part[k * nc4 + threadIdx.x];
            t.x += y.x; t.y += y.y; t.z += y.z; t.w += y.w;
        }
        const float inv = 1.f / (float)(j1 - j0);
        reinterpret_cast<float4 *>(cen + (int64_t)g * dp)[threadIdx.x] =
            make_float4(t.x * inv, t.y * inv, t.z * inv, t.w * inv);
    }
}

// sweep-order copy of the tile rows: slot j of the copy is node slot[j], a
// zero row with |x|^2 = +inf and id -1 where slot[j] < 0 (group padding)
__global__ void k_sweep_copy(const uint16_t *hi, const uint16_t *lo, const float *n2, int Kp,
                             const int32_t *slot, int64_t Np, uint16_t *bh, uint16_t *bl,
                             float *bn2, int32_t *bid_of) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int cpr = Kp / 8;
    if (e >= Np * cpr) return;
    const int64_t j = e / cpr, c = e - j * cpr;
    const int32_t v = slot[j];
    const uint4 z = make_uint4(0, 0, 0, 0);
    reinterpret_cast<uint4 *>(bh + j * Kp)[c] = v >= 0 ? reinterpret_cast<const uint4 *>(hi + (int64_t)v * Kp)[c] : z;
    if (bl) reinterpret_cast<uint4 *>(bl + j * Kp)[c] = v >= 0 ? reinterpret_cast<const uint4 *>(lo + (int64_t)v * Kp)[c] : z;
    if (c == 0) {
        bn2[j] = v >= 0 ? n2[v] : INFINITY;
        bid_of[j] = v;
    }
}

// first and last sweep position of each group (keys: the sorted group ids)
__global__ void k_group_start(const int32_t *keys, int64_t N, int32_t *gstart, int32_t *gend) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    if (j == 0 || keys[j] != keys[j - 1]) gstart[keys[j]] = (int32_t)j;
    if (j == N - 1 || keys[j] != keys[j + 1]) gend[keys[j]] = (int32_t)(j + 1);
}

// the copy slot of sorted position j: its group's first tile, plus its rank
// in the group
__global__ void k_slot_map(const int32_t *keys, const int32_t *perm, int64_t N,
                           const int32_t *gstart, const int32_t *gt_s, int bn, int32_t *slot) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    const int32_t g = keys[j];
    slot[(int64_t)gt_s[g] * bn + (j - gstart[g])] = perm[j];
}

// keys and values of the call's rows [rb, rb + M): their group, their id
__global__ void k_row_keys(const int32_t *assign, int64_t rb, int64_t M, int32_t *keys,
                           int32_t *vals) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M) return;
    keys[i] = assign[rb + i];
    vals[i] = (int32_t)(rb + i);
}

// sort keys that put larger counts first
__global__ void k_desc_keys(const int32_t *v, int32_t vmax, int64_t n, int32_t *keys) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) keys[i] = vmax - v[i];
}

// first pass: one run per row block, the tiles of the groups from its first
// row's to its last row's (rkeys: the rows' sorted group ids)
__global__ void k_pass1_runs(const int32_t *rkeys, int64_t M, int rows, const int32_t *gt_s,
                             const int32_t *gt_e, int64_t nb, int64_t *run_off,
                             int32_t *run_tile, int32_t *run_pos, int32_t *vtot) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const int32_t t0 = gt_s[rkeys[b * rows]];
    const int32_t t1 = gt_e[rkeys[min(M, (b + 1) * rows) - 1]];
    run_off[b] = b;
    if (b == nb - 1) run_off[nb] = nb;
    run_tile[b] = t0;
    run_pos[b] = 0;
    vtot[b] = t1 - t0;
}

// the groups the second pass of row block b visits (bit g of words
// need[b][0 .. W)): not one of the block's own groups, not empty, and not
// ruled out for every row of the block by the bound above.  Row r takes a
// key <= tau_r only from a member c with |r - c|^2 <= tau_r + |r|^2 + E_r,
// E_r covering the tile key's error (ea: dot products, relative to
// |r| |c|; eb: norms and the final adds) and the fp32 norm of r; the
// distances here carry a relative margin of 1e-4 (fp32 sums of at most 256
// squares are far closer).  Rows as in k_assign_pivot, 64 per pass over the
// centres (rows / 64 passes); workgroup (b, y) takes centre words
// [y wps, (y + 1) wps) and adds its count to nneed[b] (zeroed before).
template <int NCHL>
__global__ void __launch_bounds__(256, 3)
k_visit_groups(const float *vec, const int32_t *rowperm, int64_t M, int rows, const int32_t *rkeys,
               const float *cen, const float *rad, const int32_t *gt_s, const int32_t *gt_e,
               int P, int wps, const float *tau, const float *n2, float ea, float eb, float maxn,
               uint32_t *need, int32_t *nneed) {
    constexpr int dp = NCHL * 32;
    __shared__ __attribute__((aligned(16))) float sp[32 * dp];
    __shared__ float srad[32];
    __shared__ uint32_t sneed[kMaxGroups / 32];
    __shared__ int scount[4];
    const int64_t b = blockIdx.x;
    const int i = threadIdx.x, p8 = i & 7, grp = i >> 3;
    const int W = (P + 31) / 32;
    const int w0 = blockIdx.y * wps, w1 = min(W, w0 + wps);
    for (int k = w0 + i; k < w1; k += blockDim.x) sneed[k] = 0u;
    // a row's bound: -1 past M (takes nothing), +inf while it holds < K
    auto bound = [&](int64_t pos, int32_t node) {
        const float t = tau[pos], nr2 = n2[node], nr = sqrtf(nr2);
        const float E = 2.f * (ea * nr * maxn + eb * (maxn * maxn + nr * maxn + nr2));
        return t >= FLT_MAX ? INFINITY : (t + nr2 + E) * (1.f + 1e-4f) + FLT_MIN;
    };
    const int64_t rend = min(M, (b + 1) * (int64_t)rows);
    for (int64_t r0 = b * rows; r0 < rend; r0 += 64) {
        const int64_t pa = r0 + grp, pb = pa + 32;
        const int32_t na = pa < rend ? rowperm[pa] : 0, nb = pb < rend ? rowperm[pb] : 0;
        const float ha = pa < rend ? bound(pa, na) : -1.f, hb = pb < rend ? bound(pb, nb) : -1.f;
        RowPair<NCHL> rp;
        rp.load(vec + (int64_t)na * dp, vec + (int64_t)nb * dp, p8);
        for (int p0 = w0 * 32; p0 < min(P, w1 * 32); p0 += 32) {
            const int np = min(32, P - p0);
            __syncthreads();
            stage_centres(cen, p0, np, dp, sp);
            if (i < 32) srad[i] = i < np ? rad[p0 + i] : 0.f;
            __syncthreads();
            float da[4], db[4];
            rp.dist(sp, p8, da, db);
            uint32_t m = 0u;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int k = 4 * p8 + q;
                const float rk = srad[k] * (1.f + 1e-4f);
                const float la = sqrtf(da[q]) * (1.f - 1e-4f) - rk;
                const float lb = sqrtf(db[q]) * (1.f - 1e-4f) - rk;
                const bool fa = ha < 0.f || (la > 0.f && la * la > ha);
                const bool fb = hb < 0.f || (lb > 0.f && lb * lb > hb);
                if (k < np && (!fa || !fb)) m |= 1u << k;
            }
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) m |= __shfl_xor(m, off);
            if ((i & 63) == 0 && m) atomicOr(&sneed[p0 / 32], m);
        }
    }
    __syncthreads();
    const int32_t gf = rkeys[b * rows], gl = rkeys[rend - 1];
    int cnt = 0;
    for (int k = w0 + i; k < w1; k += blockDim.x) {
        uint32_t word = sneed[k];
        for (int bit = 0; bit < 32; ++bit) {
            const int g = k * 32 + bit;
            if (g >= P || (g >= gf && g <= gl) || gt_e[g] == gt_s[g]) word &= ~(1u << bit);
        }
        need[b * W + k] = word;
        cnt += __popc(word);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off);
    if ((i & 63) == 0) scount[i >> 6] = cnt;
    __syncthreads();
    if (i == 0) atomicAdd(nneed + b, scount[0] + scount[1] + scount[2] + scount[3]);
}

// squared fp32 distances between all pairs of the P centres (out [P][P])
__global__ void k_centre_d2(const float *c, int P, int dp, float *out) {
    const int i = blockIdx.x;
    const int j = blockIdx.y * blockDim.x + threadIdx.x;
    if (j >= P) return;
    const float *a = c + (int64_t)i * dp, *b = c + (int64_t)j * dp;
    float acc = 0.f;
    for (int k = 0; k < dp; ++k) {
        const float t = a[k] - b[k];
        acc = fmaf(t, t, acc);
    }
    out[(int64_t)i * P + j] = acc;
}

// renumber the P centres along a nearest-neighbour chain: centre 0 first,
// then always the nearest centre not yet taken (the smaller index on
// ties).  Groups with nearby numbers then lie near each other, so a block
// whose few rows come from several consecutive groups (an insertion batch)
// needs fewer other groups.  The order changes no list, only the work.
void order_centres(DevBuf &cen, int P, int dp, hipStream_t s) {
    if (P <= 2) return;
    DevBuf d2((size_t)P * P * sizeof(float));
    hipLaunchKernelGGL(k_centre_d2, dim3((unsigned)P, (unsigned)g1b(P, 256)), dim3(256), 0, s,
                       cen.as<float>(), P, dp, d2.as<float>());
    std::vector<float> h((size_t)P * P);
    VJ_HIP(hipMemcpyAsync(h.data(), d2.p, h.size() * sizeof(float), hipMemcpyDeviceToHost, s));
    VJ_HIP(hipStreamSynchronize(s));
    std::vector<int32_t> order((size_t)P);
    std::vector<char> taken((size_t)P, 0);
    int cur = 0;
    taken[0] = 1;
    order[0] = 0;
    for (int k = 1; k < P; ++k) {
        const float *row = h.data() + (size_t)cur * P;
        int best = -1;
        float bd = INFINITY;
        for (int j = 0; j < P; ++j)
            if (!taken[(size_t)j] && (best < 0 || row[j] < bd)) {
                best = j;
                bd = row[j];
            }
        taken[(size_t)best] = 1;
        order[(size_t)k] = best;
        cur = best;
    }
    DevBuf ids((size_t)P * sizeof(int32_t)), out((size_t)P * dp * sizeof(float));
    VJ_HIP(hipMemcpyAsync(ids.p, order.data(), (size_t)P * sizeof(int32_t), hipMemcpyHostToDevice, s));
    gather_rows_f32(cen.as<float>(), dp, ids.as<int32_t>(), P, out.as<float>(), s);
    VJ_HIP(hipStreamSynchronize(s));  // ids and the old rows are freed on return
    cen = std::move(out);
}

// the two kernels above for dp = 32 NCHL (dp <= 256, a multiple of 32)
#define VJ_NCHL_SWITCH(dp, CALL)                                                        \
    switch ((dp) / 32) {                                                                \
    case 1: CALL(1); break;                                                             \
    case 2: CALL(2); break;                                                             \
    case 3: CALL(3); break;                                                             \
    case 4: CALL(4); break;                                                             \
    case 6: CALL(6); break;                                                             \
    case 8: CALL(8); break;                                                             \
    default: VJ_CHECK(false, VJ_ERR_UNSUPPORTED, "row width of the group order");     \
    }
// slices of the centre words so that a launch of nb row workgroups has
// about 2,048 workgroups (few rows: an insertion batch)
inline int centre_slices(int64_t nb, int W) {
    return (int)std::min<int64_t>(W, std::max<int64_t>(1, (2048 + nb - 1) / nb));
}
void assign_groups(const float *vec, int dp, int64_t n, const float *cen, int P, int32_t *assign,
                   float *rad, hipStream_t s) {
    VJ_CHECK(dp % 32 == 0 && dp <= 256, VJ_ERR_UNSUPPORTED, "row width of the group order");
    const int64_t nb = g1b(n, 64);
    const int W = (P + 31) / 32, cs = centre_slices(nb, W), wps = (W + cs - 1) / cs;
    const int ny = (W + wps - 1) / wps;
    DevBuf best;
    if (ny > 1) {
        best.alloc((size_t)n * sizeof(unsigned long long));
        VJ_HIP(hipMemsetAsync(best.p, 0xff, best.bytes, s));
    }
    unsigned long long *bp = ny > 1 ? best.as<unsigned long long>() : nullptr;
#define VJ_CALL(c)                                                                                 \
    hipLaunchKernelGGL(k_assign_pivot<c>, dim3((unsigned)nb, (unsigned)ny), dim3(256), 0, s, vec, n, \
                       cen, P, wps, assign, rad, bp)
    VJ_NCHL_SWITCH(dp, VJ_CALL)
#undef VJ_CALL
    if (ny > 1) {
        hipLaunchKernelGGL(k_assign_finish, dim3(g1b(n, 256)), dim3(256), 0, s, bp, n, assign, rad);
        VJ_HIP(hipStreamSynchronize(s));  // best is freed on return
    }
}
void visit_groups(const float *vec, int dp, const int32_t *rowperm, int64_t M, int rows,
                  const int32_t *rkeys, const float *cen, const float *rad, const int32_t *gt_s,
                  const int32_t *gt_e, int P, const float *tau, const float *n2, float ea,
                  float eb, float maxn, uint32_t *need, int32_t *nneed, hipStream_t s) {
    const int64_t nb = (M + rows - 1) / rows;
    const int W = (P + 31) / 32, cs = centre_slices(nb, W), wps = (W + cs - 1) / cs;
    const int ny = (W + wps - 1) / wps;
    fill_i32(nneed, nb, 0, s);
#define VJ_CALL(c)                                                                                 \
    hipLaunchKernelGGL(k_visit_groups<c>, dim3((unsigned)nb, (unsigned)ny), dim3(256), 0, s, vec,   \
                       rowperm, M, rows, rkeys, cen, rad, gt_s, gt_e, P, wps, tau, n2, ea, eb, maxn, \
                       need, nneed)
    VJ_NCHL_SWITCH(dp, VJ_CALL)
#undef VJ_CALL
}
#undef VJ_NCHL_SWITCH

// runs of the second pass: one per visited group of row block b, in group
// order, at run_off[b] on; positions counted from 0; vtot[b] the total.
// 128 threads, thread k for word k (W <= 128).
__global__ void __launch_bounds__(128)
k_visit_runs(const uint32_t *need, int W, const int32_t *gt_s, const int32_t *gt_e,
             const int64_t *run_off, int32_t *run_tile, int32_t *run_pos, int32_t *vtot) {
    __shared__ int s_n[2], s_l[2];
    const int64_t b = blockIdx.x;
    const int k = threadIdx.x, lane = k & 63;
    const uint32_t word = k < W ? need[b * W + k] : 0u;
    int n = __popc(word), len = 0;
    for (uint32_t m = word; m; m &= m - 1) {
        const int g = k * 32 + __builtin_ctz(m);
        len += gt_e[g] - gt_s[g];
    }
    // inclusive scans within the wave, then the first wave's totals
    int ni = n, li = len;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int a = __shfl_up(ni, off), c = __shfl_up(li, off);
        if (lane >= off) { ni += a; li += c; }
    }
    if (lane == 63) { s_n[k >> 6] = ni; s_l[k >> 6] = li; }
    __syncthreads();
    const int nb0 = k >= 64 ? s_n[0] : 0, lb0 = k >= 64 ? s_l[0] : 0;
    int64_t at = run_off[b] + nb0 + ni - n;
    int32_t p = lb0 + li - len;
    for (uint32_t m = word; m; m &= m - 1) {
        const int g = k * 32 + __builtin_ctz(m);
        run_tile[at] = gt_s[g];
        run_pos[at] = p;
        p += gt_e[g] - gt_s[g];
        ++at;
    }
    if (k == 127) vtot[b] = lb0 + li;
}

// the register-row kNN sweep for one (NSPLIT, Kp); false if that shape has
// no instantiation.  Rows and columns are in group order (above); a pass
// over runs of tiles is split over columns (gridDim.y) when there are few
// row blocks (an insertion batch), the splits' lists merged afterwards.
template <int NSPLIT, int KP>
bool launch_knn_reg_t(Index &ix, const TileRows &t, const float *vec, int dp, int64_t N, int K,
                      int64_t rb, int64_t M, DevBuf &bkey, DevBuf &bidb, float *cert,
                      hipStream_t s) {
    using S = ring::Shape<NSPLIT, KP>;
    if constexpr (!S::OK || !S::WHOLE) {
        return false;
    } else {
        constexpr int BN = S::BN;
        if (dp > 256) return false;
        DevBuf skeys((size_t)N * sizeof(int32_t)), iota((size_t)N * sizeof(int32_t)),
            perm((size_t)N * sizeof(int32_t)), tmp;
        int P = ix.piv_n;
        int key_bits = 1;
        DevBuf gstart, gend;
        // nodes sorted by group (skeys, perm), each group's sweep positions
        auto group_sort = [&]() {
            iota_i32(iota.as<int32_t>(), N, s);
            sort_pairs_i32(ix.piv_of.as<int32_t>(), skeys.as<int32_t>(), iota.as<int32_t>(),
                           perm.as<int32_t>(), N, key_bits, tmp, s);
            fill_i32(gstart.as<int32_t>(), P, -1, s);
            fill_i32(gend.as<int32_t>(), P, 0, s);
            hipLaunchKernelGGL(k_group_start, dim3(g1b(N, 256)), dim3(256), 0, s,
                               skeys.as<int32_t>(), N, gstart.as<int32_t>(), gend.as<int32_t>());
        };
        // 1. groups: a build chooses the centres and labels every node; an
        //    insertion (rows [rb, N) appended to a graph whose nodes [0, rb)
        //    are labelled) labels its new nodes, the radii grow with them
        if (ix.piv_n == 0 || rb == 0 || ix.piv_cnt != rb) {
            P = (int)std::min<int64_t>(kMaxGroups, std::max<int64_t>(1, N / kGroupRows));
            while ((1 << key_bits) < P) ++key_bits;
            gstart.alloc((size_t)P * sizeof(int32_t));
            gend.alloc((size_t)P * sizeof(int32_t));
            std::vector<int32_t> ph((size_t)P);
            for (int k = 0; k < P; ++k) ph[(size_t)k] = (int32_t)((int64_t)k * (N / P));
            DevBuf pids((size_t)P * sizeof(int32_t));
            ix.piv_rows.alloc((size_t)P * dp * sizeof(float));
            ix.piv_of.alloc((size_t)N * sizeof(int32_t));
            ix.piv_rad.alloc((size_t)P * sizeof(float));
            VJ_HIP(hipMemcpyAsync(pids.p, ph.data(), (size_t)P * sizeof(int32_t),
                                  hipMemcpyHostToDevice, s));
            gather_rows_f32(vec, dp, pids.as<int32_t>(), P, ix.piv_rows.as<float>(), s);
            for (int l = 0; l < lloyd_steps(N); ++l) {
                assign_groups(vec, dp, N, ix.piv_rows.as<float>(), P, ix.piv_of.as<int32_t>(),
                              nullptr, s);
                group_sort();
                hipLaunchKernelGGL(k_center_means, dim3(P), dim3(256), 0, s, vec, dp,
                                   perm.as<int32_t>(), gstart.as<int32_t>(), gend.as<int32_t>(),
                                   ix.piv_rows.as<float>());
            }
            order_centres(ix.piv_rows, P, dp, s);
            VJ_HIP(hipMemsetAsync(ix.piv_rad.p, 0, ix.piv_rad.bytes, s));
            assign_groups(vec, dp, N, ix.piv_rows.as<float>(), P, ix.piv_of.as<int32_t>(),
                          ix.piv_rad.as<float>(), s);
            VJ_HIP(hipStreamSynchronize(s));  // pids is freed on return
            ix.piv_n = P;
        } else {
            while ((1 << key_bits) < P) ++key_bits;
            gstart.alloc((size_t)P * sizeof(int32_t));
            gend.alloc((size_t)P * sizeof(int32_t));
            DevBuf grown((size_t)N * sizeof(int32_t));
            VJ_HIP(hipMemcpyAsync(grown.p, ix.piv_of.p, (size_t)rb * sizeof(int32_t),
                                  hipMemcpyDeviceToDevice, s));
            assign_groups(vec + rb * dp, dp, N - rb, ix.piv_rows.as<float>(), P,
                          grown.as<int32_t>() + rb, ix.piv_rad.as<float>(), s);
            ix.piv_of = std::move(grown);
        }
        ix.piv_cnt = N;
        build_log(s, "kNN sweep: %d groups", P);
        // 2. columns in group order, each group from a tile start (its last
        //    tile padded with zero rows of id -1 and |x|^2 = +inf)
        group_sort();
        std::vector<int32_t> gs((size_t)P), ge((size_t)P), ts((size_t)P), te((size_t)P);
        VJ_HIP(hipMemcpyAsync(gs.data(), gstart.p, (size_t)P * sizeof(int32_t),
                              hipMemcpyDeviceToHost, s));
        VJ_HIP(hipMemcpyAsync(ge.data(), gend.p, (size_t)P * sizeof(int32_t),
                              hipMemcpyDeviceToHost, s));
        VJ_HIP(hipStreamSynchronize(s));
        int64_t T = 0;
        for (int g = 0; g < P; ++g) {
            const int64_t n = gs[(size_t)g] < 0 ? 0 : ge[(size_t)g] - gs[(size_t)g];
            ts[(size_t)g] = (int32_t)T;
            T += (n + BN - 1) / BN;
            te[(size_t)g] = (int32_t)T;
        }
        const int64_t Np = T * BN;
        VJ_CHECK(Np < ((int64_t)1 << 31), VJ_ERR_UNSUPPORTED, "kNN sweep columns");
        DevBuf gt_s((size_t)P * sizeof(int32_t)), gt_e((size_t)P * sizeof(int32_t)),
            slot((size_t)Np * sizeof(int32_t));
        VJ_HIP(hipMemcpyAsync(gt_s.p, ts.data(), (size_t)P * sizeof(int32_t),
                              hipMemcpyHostToDevice, s));
        VJ_HIP(hipMemcpyAsync(gt_e.p, te.data(), (size_t)P * sizeof(int32_t),
                              hipMemcpyHostToDevice, s));
        fill_i32(slot.as<int32_t>(), Np, -1, s);
        hipLaunchKernelGGL(k_slot_map, dim3(g1b(N, 256)), dim3(256), 0, s, skeys.as<int32_t>(),
                           perm.as<int32_t>(), N, gstart.as<int32_t>(), gt_s.as<int32_t>(), BN,
                           slot.as<int32_t>());
        DevBuf bh((size_t)Np * KP * sizeof(uint16_t)),
            bl(NSPLIT == 3 ? (size_t)Np * KP * sizeof(uint16_t) : 16), bn2((size_t)Np * sizeof(float)),
            bid_of((size_t)Np * sizeof(int32_t));
        hipLaunchKernelGGL(k_sweep_copy, dim3(g1b(Np * (KP / 8), 256)), dim3(256), 0, s,
                           t.hi.as<uint16_t>(), NSPLIT == 3 ? t.lo.as<uint16_t>() : nullptr,
                           t.norm2.as<float>(), KP, slot.as<int32_t>(), Np, bh.as<uint16_t>(),
                           NSPLIT == 3 ? bl.as<uint16_t>() : nullptr, bn2.as<float>(),
                           bid_of.as<int32_t>());
        slot.release();
        skeys.release();
        perm.release();
        iota.release();
        // 3. the call's rows in group order
        const int64_t nb = (M + S::ROWS - 1) / S::ROWS;
        DevBuf rkeys((size_t)M * sizeof(int32_t)), rkeys2((size_t)M * sizeof(int32_t)),
            rvals((size_t)M * sizeof(int32_t)), rowperm((size_t)M * sizeof(int32_t));
        hipLaunchKernelGGL(k_row_keys, dim3(g1b(M, 256)), dim3(256), 0, s, ix.piv_of.as<int32_t>(),
                           rb, M, rkeys.as<int32_t>(), rvals.as<int32_t>());
        sort_pairs_i32(rkeys.as<int32_t>(), rkeys2.as<int32_t>(), rvals.as<int32_t>(),
                       rowperm.as<int32_t>(), M, key_bits, tmp, s);
        rkeys.release();
        rvals.release();
        // launches of at most kKnnChunk row blocks (progress between them
        // when logging; no launch runs for minutes on the largest builds)
        auto sweep = [&](const DevBuf &roff, const DevBuf &rtile, const DevBuf &rpos,
                         const DevBuf &vt, int splits, int32_t split_base, const float *tau_in,
                         const int32_t *cnt_in, const int32_t *order) {
            for (int64_t b0 = 0; b0 < nb; b0 += kKnnChunk) {
                const int64_t nbc = std::min<int64_t>(kKnnChunk, nb - b0);
                hipLaunchKernelGGL((k_knn_reg<NSPLIT, KP>), dim3((unsigned)nbc, (unsigned)splits),
                                   dim3(256), 0, s, t.hi.as<uint16_t>(),
                                   NSPLIT == 3 ? t.lo.as<uint16_t>() : nullptr,
                                   rowperm.as<int32_t>(), (int32_t)M, bh.as<uint16_t>(),
                                   NSPLIT == 3 ? bl.as<uint16_t>() : nullptr, bn2.as<float>(),
                                   bid_of.as<int32_t>(), roff.as<int64_t>(), rtile.as<int32_t>(),
                                   rpos.as<int32_t>(), vt.as<int32_t>(), split_base, tau_in,
                                   cnt_in, K, bkey.as<float>(), bidb.as<int32_t>(), (int32_t)rb,
                                   (int32_t)b0, order);
                if (nb > kKnnChunk)
                    build_log(s, "kNN sweep: row blocks %lld of %lld", (long long)(b0 + nbc),
                              (long long)nb);
            }
        };
        // column splits of a pass whose blocks sweep vsum tiles in all
        auto nsplits = [&](int64_t vsum) {
            const int64_t mean = (vsum + nb - 1) / nb;
            int sp = 1;
            while (nb * sp < 1024 && mean / (sp * 2) >= 8 && sp < 256) sp *= 2;
            return sp;
        };
        int64_t vmax = 0;  // the most tiles of one block in the last pass counted
        auto total = [&](const DevBuf &vt) {
            std::vector<int32_t> h((size_t)nb);
            VJ_HIP(hipMemcpyAsync(h.data(), vt.p, (size_t)nb * sizeof(int32_t),
                                  hipMemcpyDeviceToHost, s));
            VJ_HIP(hipStreamSynchronize(s));
            int64_t v = 0;
            vmax = 0;
            for (int32_t x : h) {
                v += x;
                vmax = std::max<int64_t>(vmax, x);
            }
            return v;
        };
        // lists 0 .. S-1 of every row into list 0 (sorted), in rounds
        auto merge_lists = [&](int S) {
            const int G = std::max(2, 512 / K);
            for (int64_t step = 1; step < S; step *= G) {
                const int64_t ng = (S + G * step - 1) / (G * step);
                hipLaunchKernelGGL(k_knn_merge_splits, dim3(g1b(M * ng, 4)), dim3(256), 0, s,
                                   bkey.as<float>(), bidb.as<int32_t>(), M, S, K, G, (int)step);
            }
        };
        // 4. first pass: each block's own groups
        DevBuf roff1((size_t)(nb + 1) * sizeof(int64_t)), rtile1((size_t)nb * sizeof(int32_t)),
            rpos1((size_t)nb * sizeof(int32_t)), vt1((size_t)nb * sizeof(int32_t));
        hipLaunchKernelGGL(k_pass1_runs, dim3(g1b(nb, 256)), dim3(256), 0, s, rkeys2.as<int32_t>(),
                           M, S::ROWS, gt_s.as<int32_t>(), gt_e.as<int32_t>(), nb,
                           roff1.as<int64_t>(), rtile1.as<int32_t>(), rpos1.as<int32_t>(),
                           vt1.as<int32_t>());
        const int64_t v1 = total(vt1);
        const int s1 = nsplits(v1);
        bkey.alloc((size_t)s1 * M * kKnnCap * sizeof(float));
        bidb.alloc((size_t)s1 * M * kKnnCap * sizeof(int32_t));
        sweep(roff1, rtile1, rpos1, vt1, s1, 0, nullptr, nullptr, nullptr);
        merge_lists(s1);
        // 5. thresholds, then the groups each block still needs
        DevBuf tau((size_t)M * sizeof(float)), cnt((size_t)M * sizeof(int32_t));
        hipLaunchKernelGGL(k_list_tau, dim3(g1b(M, 256)), dim3(256), 0, s, bkey.as<float>(),
                           bidb.as<int32_t>(), rowperm.as<int32_t>(), M, rb, K, tau.as<float>(),
                           cnt.as<int32_t>());
        const int W = (P + 31) / 32;
        double e_dot = 0.0, e_fin = 0.0;
        tile_error_bounds(t, t, NSPLIT, e_dot, e_fin);
        DevBuf need((size_t)nb * W * sizeof(uint32_t)), nneed((size_t)nb * sizeof(int32_t)),
            roff2((size_t)(nb + 1) * sizeof(int64_t)), vt2((size_t)nb * sizeof(int32_t));
        visit_groups(vec, dp, rowperm.as<int32_t>(), M, S::ROWS, rkeys2.as<int32_t>(),
                     ix.piv_rows.as<float>(), ix.piv_rad.as<float>(), gt_s.as<int32_t>(),
                     gt_e.as<int32_t>(), P, tau.as<float>(), t.norm2.as<float>(), (float)e_dot,
                     (float)e_fin, t.maxnorm, need.as<uint32_t>(), nneed.as<int32_t>(), s);
        exclusive_scan_i32_i64(nneed.as<int32_t>(), roff2.as<int64_t>(), nb, tmp, s);
        int64_t nruns = 0;
        VJ_HIP(hipMemcpyAsync(&nruns, roff2.as<int64_t>() + nb, sizeof(int64_t),
                              hipMemcpyDeviceToHost, s));
        VJ_HIP(hipStreamSynchronize(s));
        DevBuf rtile2((size_t)std::max<int64_t>(nruns, 1) * sizeof(int32_t)),
            rpos2((size_t)std::max<int64_t>(nruns, 1) * sizeof(int32_t));
        hipLaunchKernelGGL(k_visit_runs, dim3((unsigned)nb), dim3(128), 0, s, need.as<uint32_t>(),
                           W, gt_s.as<int32_t>(), gt_e.as<int32_t>(), roff2.as<int64_t>(),
                           rtile2.as<int32_t>(), rpos2.as<int32_t>(), vt2.as<int32_t>());
        const int64_t v2 = total(vt2);
        ix.knn_tiles[0] = v1;
        ix.knn_tiles[1] = v2;
        ix.knn_tiles[2] = nb * T;
        build_log(s, "kNN sweep: first pass %lld tiles, second pass %lld of %lld (%.3f; %lld blocks, "
                  "at most %lld of %lld tiles in one)", (long long)v1, (long long)v2,
                  (long long)(nb * T), (double)v2 / (double)(nb * T), (long long)nb,
                  (long long)vmax, (long long)T);
        // 6. second pass: with one split the lists go on in list 0 (from
        //    their counts and thresholds); with more, the splits start empty
        //    lists 1 .. s2 from the thresholds (a true top-K entry is at or
        //    below them, so it passes in its split and survives that split's
        //    merges) and all are merged again
        if (v2 > 0) {
            const int s2 = nsplits(v2);
            if (s2 == 1) {
                // the blocks by falling tile count: a block whose rows got no
                // threshold from their own groups sweeps nearly every tile,
                // and runs beside the others instead of after them
                DevBuf keys((size_t)nb * sizeof(int32_t)), keys2((size_t)nb * sizeof(int32_t)),
                    iota2((size_t)nb * sizeof(int32_t)), order((size_t)nb * sizeof(int32_t));
                int bits = 1;
                while (((int64_t)1 << bits) <= vmax) ++bits;
                hipLaunchKernelGGL(k_desc_keys, dim3(g1b(nb, 256)), dim3(256), 0, s,
                                   vt2.as<int32_t>(), (int32_t)vmax, nb, keys.as<int32_t>());
                iota_i32(iota2.as<int32_t>(), nb, s);
                sort_pairs_i32(keys.as<int32_t>(), keys2.as<int32_t>(), iota2.as<int32_t>(),
                               order.as<int32_t>(), nb, bits, tmp, s);
                sweep(roff2, rtile2, rpos2, vt2, 1, 0, tau.as<float>(), cnt.as<int32_t>(),
                      order.as<int32_t>());
                VJ_HIP(hipStreamSynchronize(s));  // the order buffers are freed at the block's end
            } else {
                if ((size_t)(1 + s2) > (size_t)s1) {
                    // room for 1 + s2 lists, list 0 kept
                    DevBuf k2((size_t)(1 + s2) * M * kKnnCap * sizeof(float)),
                        i2((size_t)(1 + s2) * M * kKnnCap * sizeof(int32_t));
                    VJ_HIP(hipMemcpyAsync(k2.p, bkey.p, (size_t)M * kKnnCap * sizeof(float),
                                          hipMemcpyDeviceToDevice, s));
                    VJ_HIP(hipMemcpyAsync(i2.p, bidb.p, (size_t)M * kKnnCap * sizeof(int32_t),
                                          hipMemcpyDeviceToDevice, s));
                    bkey = std::move(k2);
                    bidb = std::move(i2);
                }
                sweep(roff2, rtile2, rpos2, vt2, s2, 1, tau.as<float>(), nullptr, nullptr);
                merge_lists(1 + s2);
            }
        }
        if (cert)
            hipLaunchKernelGGL(k_list_cert, dim3(g1b(M, 256)), dim3(256), 0, s, bkey.as<float>(),
                               bidb.as<int32_t>(), rowperm.as<int32_t>(), M, rb, K,
                               t.norm2.as<float>(), (float)e_dot, (float)e_fin, t.maxnorm, cert);
        VJ_HIP(hipGetLastError());
        VJ_HIP(hipStreamSynchronize(s));  // the temporaries above are freed on return
        return true;
    }
}

bool launch_knn_reg(Index &ix, int nsplit, int Kp, const TileRows &t, const float *vec, int dp,
                    int64_t N, int K, int64_t rb, int64_t M, DevBuf &bkey, DevBuf &bidb,
                    float *cert, hipStream_t s) {
    if (K > 128 || M <= 0) return false;
#define VJ_KNN_CASE(kp)                                                                         \
    case kp:                                                                                    \
        return nsplit == 3 ? launch_knn_reg_t<3, kp>(ix, t, vec, dp, N, K, rb, M, bkey, bidb, cert, s) \
                           : launch_knn_reg_t<1, kp>(ix, t, vec, dp, N, K, rb, M, bkey, bidb, cert, s);
    switch (Kp) {
        VJ_KNN_CASE(32) VJ_KNN_CASE(64) VJ_KNN_CASE(96) VJ_KNN_CASE(128) VJ_KNN_CASE(192)
        VJ_KNN_CASE(256)
    default: return false;
    }
#undef VJ_KNN_CASE
}

// exact top-K candidate lists (ids in bid [M][kKnnCap], K of them) of rows
// [rb, rb + M) of ix.vec among all ix.N rows, on MFMA tiles; true if the
// lists' distance bounds went to cert (M floats; the register-row sweep)
bool knn_candidates(Index &ix, int64_t rb, int64_t M, int K, DevBuf &bidb, float *cert,
                    hipStream_t s) {
    const int64_t N = ix.N;
    const int dp = ix.dp;
    const float *vec = ix.vec.as<float>();
    TileRows t;
    const int Kp = ((dp + 31) / 32) * 32;
    prepare_rows(vec, N, dp, Kp, true, t, s);
    double e_dot, e_fin;
    tile_error_bounds(t, t, 1, e_dot, e_fin);
    const int nsplit = (e_dot == 0.0) ? 1 : 3;
    DevBuf bkey;
    if (launch_knn_reg(ix, nsplit, Kp, t, vec, dp, N, K, rb, M, bkey, bidb, cert, s)) {
        VJ_HIP(hipGetLastError());
        VJ_HIP(hipStreamSynchronize(s));
        return true;
    }
    ix.knn_tiles[0] = ix.knn_tiles[1] = ix.knn_tiles[2] = 0;
    bkey.alloc((size_t)M * kKnnCap * sizeof(float));
    bidb.alloc((size_t)M * kKnnCap * sizeof(int32_t));
    if (nsplit == 3)
        hipLaunchKernelGGL(k_knn<3>, dim3(g1b(M, 64)), dim3(256), 0, s, t.hi.as<uint16_t>(),
                           t.lo.as<uint16_t>(), N, Kp, t.norm2.as<float>(), K, bkey.as<float>(),
                           bidb.as<int32_t>(), rb, M);
    else
        hipLaunchKernelGGL(k_knn<1>, dim3(g1b(M, 64)), dim3(256), 0, s, t.hi.as<uint16_t>(),
                           nullptr, N, Kp, t.norm2.as<float>(), K, bkey.as<float>(),
                           bidb.as<int32_t>(), rb, M);
    VJ_HIP(hipGetLastError());
    VJ_HIP(hipStreamSynchronize(s));
    return false;
}

// connectivity repair from the entry: the smallest unreachable node gets an
// edge from its nearest reached node with a free slot (else that node's
// longest edge is replaced), until every node is reached.  The rows changed
// are appended to `touched` (if given).
// sorted kNN lists of rows [rb, rb + n) and their distance bounds (see
// k_repair_from_list); kid null: none
struct RepairLists {
    const int32_t *kid = nullptr, *from = nullptr;
    const float *kd2 = nullptr, *cert = nullptr;
    int kc = 0;
    int64_t n = 0;  // rows [0, n)
};

void repair_connectivity(Index &ix, hipStream_t s, std::vector<int32_t> *touched,
                         const RepairLists &L) {
    const int64_t N = ix.N;
    const int R = ix.R, dp = ix.dp;
    const float *vec = ix.vec.as<float>();
    DevBuf seen((size_t)N * sizeof(int)), fa((size_t)N * sizeof(int32_t)),
        fb((size_t)N * sizeof(int32_t)), ctlb(sizeof(RepairCtl));
    int *seenp = seen.as<int>();
    RepairCtl *ctl = ctlb.as<RepairCtl>();
    // pinned mirror of the control block: one small read-back per step
    RepairCtl *h = nullptr;
    VJ_HIP(hipHostMalloc((void **)&h, sizeof(RepairCtl), hipHostMallocDefault));
    struct Free {
        RepairCtl *p;
        ~Free() { (void)hipHostFree(p); }
    } free_h{h};
    auto readback = [&]() {
        VJ_HIP(hipMemcpyAsync(h, ctl, sizeof(RepairCtl), hipMemcpyDeviceToHost, s));
        VJ_HIP(hipStreamSynchronize(s));
    };
    auto bfs_from = [&](int32_t start, bool reset) {
        if (reset) VJ_HIP(hipMemsetAsync(seen.p, 0, seen.bytes, s));
        hipLaunchKernelGGL(k_bfs_seed, dim3(1), dim3(1), 0, s, seenp, fa.as<int32_t>(), start, ctl);
        int nf = 1;
        int32_t *cur = fa.as<int32_t>(), *nxt = fb.as<int32_t>();
        for (int64_t level = 0; nf > 0 && level <= N; ++level) {
            if (level > 0) hipLaunchKernelGGL(k_zero_nnext, dim3(1), dim3(1), 0, s, ctl);
            hipLaunchKernelGGL(k_bfs_step, dim3(g1b((int64_t)nf * R, 256)), dim3(256), 0, s,
                               ix.adj.as<int32_t>(), R, cur, nf, seenp, nxt, &ctl->nnext);
            readback();
            nf = h->nnext;
            std::swap(cur, nxt);
        }
    };
    bfs_from(ix.entry, true);
    const int64_t max_iter = std::min<int64_t>(N, 200000);
    int64_t ncert = 0, nrange = 0;  // steps answered from the lists; with a scan of newer nodes
    ix.last_repairs = 0;
    // while edges are only added, reachability only grows and the smallest
    // unseen node only moves up: each scan starts after the last one
    int64_t from = 0;
    const unsigned scan_grid = std::min<unsigned>(g1b(N, 256), 1024);
    for (int64_t iter = 0;; ++iter) {
        VJ_CHECK(iter <= max_iter, VJ_ERR_INTERNAL, "connectivity repair did not converge");
        hipLaunchKernelGGL(k_repair_reset, dim3(1), dim3(1), 0, s, ctl);
        hipLaunchKernelGGL(k_first_unseen, dim3(scan_grid), dim3(256), 0, s, seenp, from, N,
                           &ctl->first);
        if (L.kid)
            hipLaunchKernelGGL(k_repair_from_list, dim3(1), dim3(64), 0, s, L.kid, L.kd2, L.kc,
                               L.cert, L.from, L.n, N, seenp, ix.adj.as<int32_t>(), R, ctl);
        hipLaunchKernelGGL(k_nearest_reached, dim3(std::min<unsigned>(g1b(N, 32), 2048)), dim3(256),
                           0, s, vec, N, dp, &ctl->first, seenp, ix.adj.as<int32_t>(), R,
                           &ctl->certified, &ctl->scan_from, &ctl->best_any, &ctl->best_free);
        readback();
        ncert += h->certified;
        nrange += h->scan_from > 0;
        const int32_t first = h->first;
        if (first == 0x7fffffff) break;
        const bool has_free = h->best_free != ~0ull;
        const int32_t p = (int32_t)(uint32_t)(has_free ? h->best_free : h->best_any);
        VJ_CHECK(p >= 0 && p < N, VJ_ERR_INTERNAL, "repair source");
        hipLaunchKernelGGL(k_attach, dim3(1), dim3(64), 0, s, vec, dp, ix.adj.as<int32_t>(), R, p,
                           first);
        ix.repairs += 1;
        ix.last_repairs = iter + 1;
        if ((iter + 1) % 1024 == 0) build_log(s, "connectivity repair: %lld edges", (long long)(iter + 1));
        if (touched) touched->push_back(p);
        // a new edge only adds reachability; an overwritten edge may remove some
        if (has_free) {
            bfs_from(first, false);
            from = first + 1;
        } else {
            bfs_from(ix.entry, true);
            from = 0;
        }
    }
    build_log(s, "connectivity repair: %lld steps answered from the kNN lists, %lld from a list "
              "and the nodes added since", (long long)ncert, (long long)nrange);
    ix.last_listed = ncert + nrange;
}

}  // namespace

void build_graph(Index &ix, int kc, hipStream_t s) {
    const int64_t N = ix.N;
    const int R = ix.R, dp = ix.dp;
    VJ_CHECK(N >= 2, VJ_ERR_INVALID_ARG, "need at least two vectors");
    VJ_CHECK(N < ((int64_t)1 << 31), VJ_ERR_UNSUPPORTED, "node ids are int32: N < 2^31");
    kc = (int)std::min<int64_t>(kc, N - 1);
    const int K = std::min(128, kc + 16);  // top-K of the tile sweep, re-ranked to kc
    const float *vec = ix.vec.as<float>();

    // 1. kNN on MFMA tiles over all nodes, then exact re-rank
    DevBuf bidb, cert((size_t)N * sizeof(float));
    build_log(s, "build over %lld nodes: start", (long long)N);
    const bool have_cert = knn_candidates(ix, 0, N, K, bidb, cert.as<float>(), s);
    build_log(s, "kNN lists done");

    // 2. re-rank + forward prune
    DevBuf kid((size_t)N * kc * sizeof(int32_t)), kd2((size_t)N * kc * sizeof(float));
    DevBuf fwd((size_t)N * R * sizeof(int32_t)), fwd_d2((size_t)N * R * sizeof(float));
    DevBuf fdeg((size_t)N * sizeof(int32_t)), indeg((size_t)N * sizeof(int32_t));
    VJ_HIP(hipMemsetAsync(indeg.p, 0, indeg.bytes, s));
    launch_rows(dp, vec, N, R, K, kc, bidb.as<int32_t>(), kid.as<int32_t>(), kd2.as<float>(),
                fwd.as<int32_t>(), fwd_d2.as<float>(), fdeg.as<int32_t>(), indeg.as<int32_t>(), 0, N, s);
    VJ_HIP(hipGetLastError());
    bidb.release();

    // 3. reverse lists (CSR by target, offsets scanned on the device), then
    //    the final rows
    DevBuf roff((size_t)(N + 1) * sizeof(int64_t)), rpos((size_t)N * sizeof(int32_t)), stmp;
    exclusive_scan_i32_i64(indeg.as<int32_t>(), roff.as<int64_t>(), N, stmp, s);
    int64_t nrev = 0;
    VJ_HIP(hipMemcpyAsync(&nrev, roff.as<int64_t>() + N, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    VJ_HIP(hipStreamSynchronize(s));
    DevBuf rid((size_t)std::max<int64_t>(nrev, 1) * sizeof(int32_t));
    DevBuf rd2((size_t)std::max<int64_t>(nrev, 1) * sizeof(float));
    VJ_HIP(hipMemsetAsync(rpos.p, 0, rpos.bytes, s));
    hipLaunchKernelGGL(k_scatter_rev, dim3(g1b(N * R, 256)), dim3(256), 0, s, N, R,
                       fwd.as<int32_t>(), fwd_d2.as<float>(), roff.as<int64_t>(),
                       rpos.as<int32_t>(), rid.as<int32_t>(), rd2.as<float>(), (int64_t)0);
    ix.adj.alloc((size_t)N * R * sizeof(int32_t));
    launch_rev(dp, vec, N, R, fwd.as<int32_t>(), fwd_d2.as<float>(), fdeg.as<int32_t>(),
               roff.as<int64_t>(), rid.as<int32_t>(), rd2.as<float>(), ix.adj.as<int32_t>(),
               nullptr, s);
    VJ_HIP(hipGetLastError());

    build_log(s, "forward and reverse prunes done");
    // 4. entry = node nearest to the fp64 centroid (ties: smaller id)
    {
        DevBuf sum((size_t)dp * sizeof(double)), dist((size_t)N * sizeof(double)), best(16);
        VJ_HIP(hipMemsetAsync(sum.p, 0, sum.bytes, s));
        VJ_HIP(hipMemsetAsync(best.p, 0xff, 8, s));
        VJ_HIP(hipMemsetAsync(best.as<char>() + 8, 0x7f, 4, s));
        hipLaunchKernelGGL(k_centroid, dim3(std::min<int64_t>(N, 1024), g1b(dp, 128)), dim3(128), 0, s,
                           vec, N, dp, sum.as<double>());
        hipLaunchKernelGGL(k_centroid_dist, dim3(g1b(N, 256)), dim3(256), 0, s, vec, N, dp,
                           sum.as<double>(), dist.as<double>(), best.as<unsigned long long>());
        hipLaunchKernelGGL(k_argmin_id, dim3(g1b(N, 256)), dim3(256), 0, s, dist.as<double>(), N,
                           best.as<unsigned long long>(), reinterpret_cast<int *>(best.as<char>() + 8));
        int e = 0;
        VJ_HIP(hipMemcpyAsync(&e, best.as<char>() + 8, 4, hipMemcpyDeviceToHost, s));
        VJ_HIP(hipStreamSynchronize(s));
        VJ_CHECK(e >= 0 && e < N, VJ_ERR_INTERNAL, "entry point");
        ix.entry = e;
    }

    // 5. connectivity repair from the entry (with the sorted lists and their
    //    distance bounds: a step whose answer is certified there skips the scan)
    //    The lists stay with the index for the repairs of later insertions.
    RepairLists lists;
    ix.knn_id.release();
    ix.knn_d2.release();
    ix.knn_cert.release();
    ix.knn_from.release();
    ix.knn_rows = ix.knn_cap = 0;
    if (have_cert) {
        ix.knn_from.alloc((size_t)N * sizeof(int32_t));
        fill_i32(ix.knn_from.as<int32_t>(), N, (int32_t)N, s);
        ix.knn_id = std::move(kid);
        ix.knn_d2 = std::move(kd2);
        ix.knn_cert = std::move(cert);
        ix.knn_kc = kc;
        ix.knn_rows = ix.knn_cap = N;
        lists.kid = ix.knn_id.as<int32_t>();
        lists.from = ix.knn_from.as<int32_t>();
        lists.kd2 = ix.knn_d2.as<float>();
        lists.cert = ix.knn_cert.as<float>();
        lists.kc = kc;
        lists.n = N;
    }
    repair_connectivity(ix, s, nullptr, lists);
    build_log(s, "connectivity repair done (%lld edges)", (long long)ix.repairs);

    // 6. edge lengths
    ix.elen.alloc((size_t)N * R * sizeof(float));
    launch_edge_lengths(vec, dp, ix.adj.as<int32_t>(), N, R, ix.elen.as<float>(), s);
    VJ_HIP(hipGetLastError());
    VJ_HIP(hipStreamSynchronize(s));
}

void insert_graph(Index &ix, int64_t n_old, int kc, hipStream_t s) {
    const int64_t N = ix.N, M = N - n_old;
    const int R = ix.R, dp = ix.dp;
    VJ_CHECK(M >= 0 && n_old >= 1, VJ_ERR_INTERNAL, "insertion rows");
    if (M == 0) return;
    kc = (int)std::min<int64_t>(kc, N - 1);
    const int K = std::min(128, kc + 16);
    const float *vec = ix.vec.as<float>();
    int32_t *adj = ix.adj.as<int32_t>();

    // 1. candidates of the new rows among all rows, re-rank, forward prune
    DevBuf bidb, cert((size_t)M * sizeof(float));
    const bool have_cert = knn_candidates(ix, n_old, M, K, bidb, cert.as<float>(), s);
    DevBuf kid((size_t)M * kc * sizeof(int32_t)), kd2((size_t)M * kc * sizeof(float));
    DevBuf fwd((size_t)M * R * sizeof(int32_t)), fwd_d2((size_t)M * R * sizeof(float));
    DevBuf fdeg((size_t)M * sizeof(int32_t)), indeg((size_t)N * sizeof(int32_t));
    VJ_HIP(hipMemsetAsync(indeg.p, 0, indeg.bytes, s));
    launch_rows(dp, vec, N, R, K, kc, bidb.as<int32_t>(), kid.as<int32_t>(), kd2.as<float>(),
                fwd.as<int32_t>(), fwd_d2.as<float>(), fdeg.as<int32_t>(), indeg.as<int32_t>(),
                n_old, M, s);
    VJ_HIP(hipGetLastError());
    bidb.release();

    // 2. offers (CSR by target) and the rows that change: every old row that
    //    receives an offer, and every new row (offsets and the row list
    //    scanned on the device; two totals come back)
    DevBuf roff((size_t)(N + 1) * sizeof(int64_t)), rpos((size_t)N * sizeof(int32_t)),
        flag((size_t)N * sizeof(int32_t)), fpos((size_t)(N + 1) * sizeof(int64_t)), stmp;
    exclusive_scan_i32_i64(indeg.as<int32_t>(), roff.as<int64_t>(), N, stmp, s);
    hipLaunchKernelGGL(k_changed_flags, dim3(g1b(N, 256)), dim3(256), 0, s, indeg.as<int32_t>(),
                       n_old, N, flag.as<int32_t>());
    exclusive_scan_i32_i64(flag.as<int32_t>(), fpos.as<int64_t>(), N, stmp, s);
    int64_t tot[2] = {0, 0};
    VJ_HIP(hipMemcpyAsync(&tot[0], roff.as<int64_t>() + N, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    VJ_HIP(hipMemcpyAsync(&tot[1], fpos.as<int64_t>() + N, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    VJ_HIP(hipStreamSynchronize(s));
    const int64_t nrev = tot[0], L = tot[1];
    DevBuf rid((size_t)std::max<int64_t>(nrev, 1) * sizeof(int32_t));
    DevBuf rd2((size_t)std::max<int64_t>(nrev, 1) * sizeof(float));
    DevBuf rows((size_t)std::max<int64_t>(L, 1) * sizeof(int32_t));
    hipLaunchKernelGGL(k_scatter_flagged, dim3(g1b(N, 256)), dim3(256), 0, s, flag.as<int32_t>(),
                       fpos.as<int64_t>(), N, rows.as<int32_t>());
    VJ_HIP(hipMemsetAsync(rpos.p, 0, rpos.bytes, s));
    hipLaunchKernelGGL(k_scatter_rev, dim3(g1b(M * R, 256)), dim3(256), 0, s, M, R,
                       fwd.as<int32_t>(), fwd_d2.as<float>(), roff.as<int64_t>(),
                       rpos.as<int32_t>(), rid.as<int32_t>(), rd2.as<float>(), n_old);

    // 3. candidates of each changing row (current row or forward list, plus
    //    its offers), kept whole if they fit, else RNG-pruned
    DevBuf gf((size_t)L * R * sizeof(int32_t)), gd((size_t)L * R * sizeof(float)),
        gdeg((size_t)L * sizeof(int32_t));
    launch_gather(dp, vec, R, adj, fwd.as<int32_t>(), fdeg.as<int32_t>(), n_old,
                  rows.as<int32_t>(), L, gf.as<int32_t>(), gd.as<float>(), gdeg.as<int32_t>(), s);
    launch_rev(dp, vec, L, R, gf.as<int32_t>(), gd.as<float>(), gdeg.as<int32_t>(),
               roff.as<int64_t>(), rid.as<int32_t>(), rd2.as<float>(), adj, rows.as<int32_t>(), s);
    VJ_HIP(hipGetLastError());
    VJ_HIP(hipStreamSynchronize(s));

    // 4. connectivity repair from the (unchanged) entry, then the lengths of
    //    every row that changed (the listed rows and the repairs' sources)
    std::vector<int32_t> touched;
    //    The new rows' lists join those the index kept for its old rows (from
    //    the build and earlier insertions; an old row without one gets the
    //    bound -inf), in arrays grown by half when full.
    RepairLists lists;
    if (have_cert) {
        const bool keep_old = ix.knn_rows == n_old && ix.knn_kc == kc;
        if (!keep_old || ix.knn_cap < N) {
            const int64_t cap = keep_old ? std::max<int64_t>(N, ix.knn_cap + ix.knn_cap / 2) : N;
            DevBuf nid((size_t)cap * kc * sizeof(int32_t)), nd2((size_t)cap * kc * sizeof(float)),
                ncert((size_t)cap * sizeof(float)), nfrom((size_t)cap * sizeof(int32_t));
            if (keep_old) {
                VJ_HIP(hipMemcpyAsync(nid.p, ix.knn_id.p, (size_t)n_old * kc * sizeof(int32_t),
                                      hipMemcpyDeviceToDevice, s));
                VJ_HIP(hipMemcpyAsync(nd2.p, ix.knn_d2.p, (size_t)n_old * kc * sizeof(float),
                                      hipMemcpyDeviceToDevice, s));
                VJ_HIP(hipMemcpyAsync(ncert.p, ix.knn_cert.p, (size_t)n_old * sizeof(float),
                                      hipMemcpyDeviceToDevice, s));
                VJ_HIP(hipMemcpyAsync(nfrom.p, ix.knn_from.p, (size_t)n_old * sizeof(int32_t),
                                      hipMemcpyDeviceToDevice, s));
            } else {
                fill_i32(ncert.as<int32_t>(), n_old, (int32_t)0xff800000u, s);  // -inf
                fill_i32(nfrom.as<int32_t>(), n_old, 0, s);
            }
            ix.knn_id = std::move(nid);
            ix.knn_d2 = std::move(nd2);
            ix.knn_cert = std::move(ncert);
            ix.knn_from = std::move(nfrom);
            ix.knn_cap = cap;
            ix.knn_kc = kc;
        }
        VJ_HIP(hipMemcpyAsync(ix.knn_id.as<int32_t>() + n_old * kc, kid.p,
                              (size_t)M * kc * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
        VJ_HIP(hipMemcpyAsync(ix.knn_d2.as<float>() + n_old * kc, kd2.p,
                              (size_t)M * kc * sizeof(float), hipMemcpyDeviceToDevice, s));
        VJ_HIP(hipMemcpyAsync(ix.knn_cert.as<float>() + n_old, cert.p, (size_t)M * sizeof(float),
                              hipMemcpyDeviceToDevice, s));
        fill_i32(ix.knn_from.as<int32_t>() + n_old, M, (int32_t)N, s);
        ix.knn_rows = N;
        lists.kid = ix.knn_id.as<int32_t>();
        lists.from = ix.knn_from.as<int32_t>();
        lists.kd2 = ix.knn_d2.as<float>();
        lists.cert = ix.knn_cert.as<float>();
        lists.kc = kc;
        lists.n = N;
    } else {
        ix.knn_rows = 0;  // the old rows' lists no longer line up
    }
    repair_connectivity(ix, s, &touched, lists);
    int64_t nrows = L;
    if (!touched.empty()) {
        nrows = L + (int64_t)touched.size();
        DevBuf grown((size_t)nrows * sizeof(int32_t));
        if (L > 0)
            VJ_HIP(hipMemcpyAsync(grown.p, rows.p, (size_t)L * sizeof(int32_t),
                                  hipMemcpyDeviceToDevice, s));
        VJ_HIP(hipMemcpyAsync(grown.as<int32_t>() + L, touched.data(),
                              touched.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
        VJ_HIP(hipStreamSynchronize(s));  // touched is host memory
        rows = std::move(grown);
    }
    launch_edge_lengths_rows(vec, dp, adj, N, R, rows.as<int32_t>(), nrows, ix.elen.as<float>(), s);
    VJ_HIP(hipGetLastError());
    VJ_HIP(hipStreamSynchronize(s));
}

}  // namespace vj
