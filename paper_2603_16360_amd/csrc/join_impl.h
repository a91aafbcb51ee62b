// Merged-index join kernel: the online path of Algorithm 1 with cfg.merged =
// true (Sections 4.1-4.4).  Included by one translation unit per row type.
//
// Shape: by default one workgroup (four waves) per query (the workgroup
// tier); the small tier runs one wavefront (64 lanes) per query, four per
// workgroup.  A launch covers a contiguous range of a processing list.  Per
// query:
//   seeds    {s} (+ the parent's cached node, soft mode; its in-range
//            nodes, hard mode)                                  Algorithm 3
//   probe    the neighbours of the query node q                 Algorithms 4-5
//   check    d1/d2 OOD test or a per-query budget               Algorithm 6
//   expand   in-range data nodes to closure; in hybrid mode the closest
//            out-range node of a bounded queue is expanded whenever the
//            in-range worklist is empty                         Algorithm 7
//   cache    closest visited data node (soft)                   Algorithm 8
// All per-query state lives in LDS: the visited hash, the in-range worklist
// (which is also the query's pair buffer) and the out-range queue.  A query
// that outgrows them is re-run on a larger tier: from the one-wave tier a
// whole workgroup with 8x the LDS visited slots, then (in the same launch
// while free regions last) a whole workgroup with tables in global memory.
//
// Rows are gathered LPR lanes per row, 16 bytes per lane per load (a row
// group's load covers whole 128-byte lines), and reduced with xor shuffles
// inside the lane group.  Every loop has a static bound; ids read back from
// memory are range-checked before they index anything.
#pragma once

#include <type_traits>

#include "vj_internal.h"

namespace vj {
namespace wj {

// LDS tiers: one wave per query, four per workgroup, for most queries; the
// queries that outgrow it run on all four waves of a workgroup with 8x the
// visited slots.  Both keep every per-query structure in LDS.
constexpr int kWaves = 4;      // waves per workgroup
constexpr int kBeamMax = 256;  // largest out-range queue the LDS variant holds
constexpr int kHeap = kBeamMax + 64;

template <typename T> struct Elem;
template <> struct Elem<float> { static constexpr int CE = 4; };
template <> struct Elem<uint8_t> { static constexpr int CE = 16; };
template <> struct Elem<uint16_t> { static constexpr int CE = 8; };  // bf16 bits
template <> struct Elem<f8e4m3> { static constexpr int CE = 16; };   // e4m3 codes

// bf16 and fp8 rows carry a rounding error that the kernels bound and
// re-check (kLowp); fp8 rows are scaled per row
template <typename T> constexpr bool kIsF8 = std::is_same<T, f8e4m3>::value;
template <typename T> constexpr bool kIsBf16 = std::is_same<T, uint16_t>::value || kIsF8<T>;

// lanes per row: a power of two with at most 8 16-byte chunks per lane
constexpr int pick_lpr(int cpr) {
    int l = 8;
    while (l > 1 && cpr % l) l >>= 1;
    if (cpr / l > 8) {
        l = 16;
        while ((l < 64) && (cpr % l || cpr / l > 8)) l <<= 1;
    }
    return l;
}

__device__ __forceinline__ void to_float(const uint4 &r, float *f, float) {
    f[0] = __uint_as_float(r.x); f[1] = __uint_as_float(r.y);
    f[2] = __uint_as_float(r.z); f[3] = __uint_as_float(r.w);
}
__device__ __forceinline__ void to_float(const uint4 &r, float *f, uint8_t) {
    const uint32_t w[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        f[4 * i + 0] = (float)(w[i] & 0xffu);
        f[4 * i + 1] = (float)((w[i] >> 8) & 0xffu);
        f[4 * i + 2] = (float)((w[i] >> 16) & 0xffu);
        f[4 * i + 3] = (float)(w[i] >> 24);
    }
}

__device__ __forceinline__ void to_float(const uint4 &r, float *f, f8e4m3) {
    const uint32_t w[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int b = 0; b < 4; ++b) f[4 * i + b] = f8_value((w[i] >> (8 * b)) & 0xffu);
    }
}

__device__ __forceinline__ void to_float(const uint4 &r, float *f, uint16_t) {
    const uint32_t w[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        f[2 * i + 0] = __uint_as_float(w[i] << 16);
        f[2 * i + 1] = __uint_as_float(w[i] & 0xffff0000u);
    }
}

// lanes of one wave exchange data through LDS / their own global stores
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

// multiplicative hash scaled to [0, n) (for n = 2^k: its top k bits)
__device__ __forceinline__ uint32_t slot_of(int32_t v, uint32_t n) {
    return (uint32_t)(((uint64_t)((uint32_t)v * 0x9E3779B1u) * n) >> 32);
}

// wave-wide (key, id, index) reduction keeping the min or the max by (key, id)
__device__ __forceinline__ void wave_best(float &k, int &id, int &ix, bool want_max) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const float ok = __shfl_xor(k, off);
        const int oid = __shfl_xor(id, off);
        const int oix = __shfl_xor(ix, off);
        const bool take = want_max ? (ok > k || (ok == k && oid > id))
                                   : (ok < k || (ok == k && oid < id));
        if (take) { k = ok; id = oid; ix = oix; }
    }
}

// Per-wave query state.  Uniform fields are kept identical in every lane.
struct QState {
    int tail, head, hc, nvis, ndist, nexp, hpops;
    bool abort, hyb_active;
    float best_k;
    int best_id;
    float d1sum;
    int c1;
};

// Everything one wave needs to touch: LDS or spill regions, plus the query.
struct WaveMem {
    int32_t *hash;   // visited set (LDS or global)
    int hash_n, hash_limit;  // slots (any size), nodes it may hold
    int32_t *il;     // in-range worklist ids
    float *ild;      // their distance keys
    int il_cap;
    int32_t *stage;  // 64 candidate ids (LDS)
    float *hk;       // out-range queue keys (LDS)
    int32_t *hi;     // out-range queue ids
    int32_t *aux;    // 64 ids re-checked from fp32 rows (LDS, bf16 rows only)
    float *auxf;     // their fp32 values
};

// Insert each active lane's id; returns true where the id was new.  A lane
// probes at most the table size before giving up (error flag + abort).
__device__ __forceinline__ bool visit(const JoinArgs &a, const WaveMem &m, bool &abort, int32_t v,
                                      bool active) {
    bool isnew = false;
    const int n = m.hash_n;
    uint32_t h = slot_of(v, (uint32_t)n);
    int probes = 0;
    for (int it = 0; it <= n; ++it) {
        if (__ballot(active) == 0) break;
        if (active) {
            if (++probes > n) {
                active = false;
                atomicOr(a.err, 16);
            } else {
                const int old = atomicCAS(&m.hash[h], -1, v);
                if (old == -1) { isnew = true; active = false; }
                else if (old == v) active = false;
                else h = h + 1 == (uint32_t)n ? 0u : h + 1;
            }
        }
    }
    if (__ballot(probes > n)) abort = true;
    return isnew;
}

template <int LPR, int VPL, int CE, typename T>
__device__ __forceinline__ float row_partial(const uint4 *buf, const float *qf, bool l2) {
    float acc = 0.f;
#pragma unroll
    for (int w = 0; w < VPL; ++w) {
        float f[CE];
        to_float(buf[w], f, T());
#pragma unroll
        for (int e = 0; e < CE; ++e) {
            if (l2) { const float t = f[e] - qf[w * CE + e]; acc = fmaf(t, t, acc); }
            else acc = fmaf(f[e], qf[w * CE + e], acc);
        }
    }
#pragma unroll
    for (int off = LPR / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    return acc;
}

// as row_partial, plus the squared norm of the row (xn2)
template <int LPR, int VPL, int CE, typename T>
__device__ __forceinline__ float row_partial_n(const uint4 *buf, const float *qf, bool l2,
                                               float &xn2, float scale = 1.f) {
    float acc = 0.f, nn = 0.f;
#pragma unroll
    for (int w = 0; w < VPL; ++w) {
        float f[CE];
        to_float(buf[w], f, T());
        if constexpr (kIsF8<T>) {
#pragma unroll
            for (int e = 0; e < CE; ++e) f[e] *= scale;  // exact: a power of two
        }
#pragma unroll
        for (int e = 0; e < CE; ++e) {
            if (l2) { const float t = f[e] - qf[w * CE + e]; acc = fmaf(t, t, acc); }
            else acc = fmaf(f[e], qf[w * CE + e], acc);
            nn = fmaf(f[e], f[e], nn);
        }
    }
#pragma unroll
    for (int off = LPR / 2; off > 0; off >>= 1) {
        acc += __shfl_xor(acc, off);
        nn += __shfl_xor(nn, off);
    }
    xn2 = nn;
    return acc;
}

// The fp32 kernels' value of candidate `id` (L2: squared distance, IP: dot
// product), from the fp32 rows with exactly their lane layout and order of
// operations, so that a decision taken on it is the fp32 kernels' decision.
// Each group of pick_lpr(DP / 4) lanes evaluates its own id.
template <int DP>
__device__ __forceinline__ float fp32_value(const JoinArgs &a, int32_t q, int32_t id, bool l2,
                                            int lane) {
    constexpr int CPR = DP / 4;
    constexpr int LPR = pick_lpr(CPR);
    constexpr int VPL = CPR / LPR;
    const int p = lane % LPR;
    const uint4 *xrow = reinterpret_cast<const uint4 *>(a.rows32 + (size_t)id * DP);
    const float4 *qrow = reinterpret_cast<const float4 *>(a.rows32 + (size_t)q * DP);
    uint4 buf[VPL];
    float qf[VPL * 4];
#pragma unroll
    for (int w = 0; w < VPL; ++w) {
        buf[w] = xrow[p + w * LPR];
        const float4 t = qrow[p + w * LPR];
        qf[4 * w + 0] = t.x; qf[4 * w + 1] = t.y; qf[4 * w + 2] = t.z; qf[4 * w + 3] = t.w;
    }
    return row_partial<LPR, VPL, 4, float>(buf, qf, l2);
}

// drop the largest (key, id) entries until the queue holds `beam`
__device__ __forceinline__ void heap_trim(const WaveMem &m, int &hc, int beam, int lane) {
    for (int guard = 0; guard < 64 * kWaves && hc > beam; ++guard) {
        float bk = -INFINITY;
        int bid = -1, bx = 0;
        for (int i = lane; i < hc; i += 64) {
            const float kk = m.hk[i];
            const int id = m.hi[i];
            if (kk > bk || (kk == bk && id > bid)) { bk = kk; bid = id; bx = i; }
        }
        wave_best(bk, bid, bx, true);
        bx = uni(bx);
        if (lane == 0) { m.hk[bx] = m.hk[hc - 1]; m.hi[bx] = m.hi[hc - 1]; }
        hc -= 1;
        wave_sync();
    }
}

// One candidate batch (<= 1 id per lane): visited check, compaction, row
// gathers, distances, classification.  probe: distances for every valid
// data candidate (the d1 feature needs them), not only new ones.
template <typename T, int DP>
__device__ __forceinline__ void run_batch(const JoinArgs &a, const WaveMem &m, QState &s,
                                          const float *qf, int32_t v, bool probe, int lane) {
    constexpr int CE = Elem<T>::CE;
    constexpr int CPR = DP / CE;
    constexpr int LPR = pick_lpr(CPR);
    constexpr int VPL = CPR / LPR;
    constexpr int RPP = 64 / LPR;
    constexpr int PG = (12 / VPL) < (64 / RPP) ? (12 / VPL) : (64 / RPP);
    const bool l2 = a.metric == VJ_L2;
    const int p = lane % LPR, rr = lane / LPR;
    const uint64_t ltmask = (1ull << lane) - 1ull;
    const T *vbase = reinterpret_cast<const T *>(a.rows);

    const bool valid = v >= 0 && v < a.nx;
    const bool isnew = visit(a, m, s.abort, v, valid);
    s.nvis += __popcll(__ballot(isnew));
    if (s.nvis > m.hash_limit) s.abort = true;
    if (s.abort) return;
    const bool need = probe ? valid : isnew;
    const uint64_t mneed = __ballot(need);
    const int cnt = __popcll(mneed);
    if (need) m.stage[__popcll(mneed & ltmask)] = isnew ? v : ~v;
    wave_sync();
    s.ndist += cnt;
    for (int base = 0; base < cnt; base += RPP * PG) {
        uint4 buf[PG][VPL];
        int sid[PG];
#pragma unroll
        for (int g = 0; g < PG; ++g) {
            const int c = base + g * RPP + rr;
            sid[g] = c < cnt ? m.stage[c] : 0;
            const int id = sid[g] >= 0 ? sid[g] : ~sid[g];
            const uint4 *row = reinterpret_cast<const uint4 *>(vbase + (size_t)id * DP);
#pragma unroll
            for (int w = 0; w < VPL; ++w)
                buf[g][w] = c < cnt ? row[p + w * LPR] : make_uint4(0, 0, 0, 0);
        }
#pragma unroll
        for (int g = 0; g < PG; ++g) {
            const float acc = row_partial<LPR, VPL, CE, T>(buf[g], qf, l2);
            const int c = base + g * RPP + rr;
            const bool lead = p == 0 && c < cnt;
            const bool nw = sid[g] >= 0;
            const int id = nw ? sid[g] : ~sid[g];
            const float key = l2 ? acc : 1.0f - acc;
            const bool inr = l2 ? (acc < a.eps2) : (key < a.eps);
            if (lead && nw && (key < s.best_k || (key == s.best_k && id < s.best_id))) {
                s.best_k = key;
                s.best_id = id;
            }
            if (probe && lead) {
                s.d1sum += l2 ? sqrtf(key) : sqrtf(fmaxf(0.f, 2.f * key));
                s.c1 += 1;
            }
            const bool ap = lead && nw && inr;
            const uint64_t ma = __ballot(ap);
            const int na = __popcll(ma);
            if (s.tail + na > m.il_cap) {
                s.abort = true;
            } else {
                if (ap) {
                    const int o = s.tail + __popcll(ma & ltmask);
                    m.il[o] = id;
                    m.ild[o] = key;
                }
                s.tail += na;
            }
            if (s.hyb_active) {
                const bool hp = lead && nw && !inr;
                const uint64_t mh = __ballot(hp);
                if (hp) {
                    const int o = s.hc + __popcll(mh & ltmask);
                    m.hk[o] = key;
                    m.hi[o] = id;
                }
                s.hc += __popcll(mh);
                if (s.hc > a.beam) { wave_sync(); heap_trim(m, s.hc, a.beam, lane); }
            }
        }
    }
    wave_sync();
}

template <typename T, int DP>
__device__ __forceinline__ void run_query(const JoinArgs &a, const WaveMem &m, int k,
                                          const int32_t *qlist, const int32_t *qpos,
                                          int32_t *ovf, int32_t *ovf_count, int lane) {
    constexpr int CE = Elem<T>::CE;
    constexpr int CPR = DP / CE;
    constexpr int LPR = pick_lpr(CPR);
    constexpr int VPL = CPR / LPR;
    constexpr int QF = VPL * CE;
    const int R = a.R;
    const int qi = uni(qlist[k]);
    const int pos = uni(qpos[k]);
    int32_t *st = a.stats + (size_t)pos * 8;
    if (qi < 0 || qi >= a.nq) {
        if (lane < 8) st[lane] = 0;
        if (lane == 0) atomicOr(a.err, 8);
        return;
    }
    const int32_t q = (int32_t)(a.nx + qi);
    if (a.hyb == VJ_HYB_BUDGET && a.budget[pos] < 0) {  // routed to brute force
        if (lane < 8) st[lane] = lane == 7 ? 2 : 0;
        if (lane == 0 && a.ws == VJ_WS_SOFT) a.cache[qi] = -1;
        return;
    }

    // the query's slice of dimensions, fp32
    float qf[QF];
    {
        const int p = lane % LPR;
        const float *qrow = a.rows32 + (size_t)q * DP;
#pragma unroll
        for (int w = 0; w < VPL; ++w) {
            const float4 *src = reinterpret_cast<const float4 *>(qrow + (p + w * LPR) * CE);
#pragma unroll
            for (int e = 0; e < CE / 4; ++e) {
                const float4 t = src[e];
                qf[w * CE + 4 * e + 0] = t.x; qf[w * CE + 4 * e + 1] = t.y;
                qf[w * CE + 4 * e + 2] = t.z; qf[w * CE + 4 * e + 3] = t.w;
            }
        }
    }
    for (int i = lane; i < m.hash_n; i += 64) m.hash[i] = -1;
    wave_sync();

    QState s{};
    s.best_k = INFINITY;
    s.best_id = 0x7fffffff;

    // ---- SeedPhase: s, plus the parent's cache (parents ran in an earlier launch)
    int pcache = -1;
    int64_t pseg = 0;
    int pcnt = 0;
    if (a.ws == VJ_WS_SOFT || a.ws == VJ_WS_HARD) {
        const int32_t par = a.parent[qi];
        if (par >= a.nx && par < a.nx + a.nq && a.inb[par - a.nx] == (int32_t)a.gen) {
            const int pq = par - (int32_t)a.nx;
            if (a.ws == VJ_WS_SOFT) {
                pcache = uni(a.cache[pq]);
            } else {
                pseg = a.seg[pq];
                pcnt = uni(a.segn[pq]);
                if (pseg < 0 || pseg + pcnt > a.cap) pcnt = 0;
            }
        }
    }
    {
        int32_t v = -1;
        if (lane == 0) v = a.entry;
        if (lane == 1) v = pcache;
        run_batch<T, DP>(a, m, s, qf, v, false, lane);
        for (int t = 0; !s.abort && t < pcnt && t < a.nx + 64; t += 64) {
            const int32_t u = t + lane < pcnt ? a.out_x[pseg + t + lane] : -1;
            run_batch<T, DP>(a, m, s, qf, u, false, lane);
        }
    }

    // ---- GreedySearchPhase on the merged index: probe N(q), then stop
    const int32_t nbq = lane < R ? a.adj[(size_t)q * R + lane] : -1;
    if (!s.abort) run_batch<T, DP>(a, m, s, qf, nbq, a.hyb == VJ_HYB_ADAPT, lane);

    // ---- CheckHybrid
    bool hyb = false;
    int ood = 0;
    if (!s.abort) {
        if (a.hyb == VJ_HYB_FORCE) {
            hyb = true;
        } else if (a.hyb == VJ_HYB_BUDGET) {
            hyb = a.budget[pos] > 0;
        } else if (a.hyb == VJ_HYB_ADAPT) {
            float s1 = s.d1sum;
            int n1 = s.c1;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) { s1 += __shfl_xor(s1, off); n1 += __shfl_xor(n1, off); }
            float s2 = 0.f;
            int n2 = 0;
            const int NB = 64 / R;
            for (int j0 = 0; j0 < R; j0 += NB) {
                const int b = lane / R, j = lane - b * R;
                const int yj = j0 + b;
                const bool ok = b < NB && yj < R;
                const int32_t y = __shfl(nbq, ok ? yj : 0);
                if (ok && y >= 0 && y < a.nx) {
                    const int32_t z = a.adj[(size_t)y * R + j];
                    if (z >= 0 && z < a.nx) { s2 += a.elen[(size_t)y * R + j]; n2 += 1; }
                }
            }
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) { s2 += __shfl_xor(s2, off); n2 += __shfl_xor(n2, off); }
            if (n1 == 0) hyb = true;
            else if (n2 == 0) hyb = false;
            else hyb = (s1 / (float)n1) / (s2 / (float)n2) > a.ood_ratio;
            ood = hyb ? 1 : 0;
        }
    }
    s.hyb_active = hyb && a.beam > 0;

    // ---- ExpansionPhase: in-range closure, then one out-range pop at a time
    const int NB = 64 / R;
    int unprod = 0, before = 0;
    bool pending = false;
    const int budget = a.hyb == VJ_HYB_BUDGET ? a.budget[pos] : 0;
    for (int round = 0; round <= m.hash_limit + 1 && !s.abort; ++round) {
        for (int it = 0; it <= m.il_cap && !s.abort && s.head < s.tail; ++it) {
            const int nb = min(NB, s.tail - s.head);
            const int b = lane / R, j = lane - b * R;
            int32_t v = -1;
            if (b < nb) {
                const int32_t u = m.il[s.head + b];
                if (u >= 0 && u < a.nx) v = a.adj[(size_t)u * R + j];
                else atomicOr(a.err, 32);
            }
            s.head += nb;
            s.nexp += nb;
            run_batch<T, DP>(a, m, s, qf, v, false, lane);
        }
        if (s.abort) break;
        if (pending) { unprod = (s.tail == before) ? unprod + 1 : 0; pending = false; }
        if (!s.hyb_active || s.hc == 0) break;
        if (a.hyb == VJ_HYB_BUDGET) { if (s.hpops >= budget) break; }
        else if (a.conv > 0 && unprod >= a.conv) break;
        float bk = INFINITY;
        int bid = 0x7fffffff, bx = 0;
        for (int i = lane; i < s.hc; i += 64) {
            const float kk = m.hk[i];
            const int id = m.hi[i];
            if (kk < bk || (kk == bk && id < bid)) { bk = kk; bid = id; bx = i; }
        }
        wave_best(bk, bid, bx, false);
        bid = uni(bid);
        bx = uni(bx);
        if (lane == 0) { m.hk[bx] = m.hk[s.hc - 1]; m.hi[bx] = m.hi[s.hc - 1]; }
        s.hc -= 1;
        wave_sync();
        s.hpops += 1;
        s.nexp += 1;
        before = s.tail;
        pending = true;
        if (bid < 0 || bid >= a.nx) { if (lane == 0) atomicOr(a.err, 32); s.abort = true; break; }
        const int32_t v = lane < R ? a.adj[(size_t)bid * R + lane] : -1;
        run_batch<T, DP>(a, m, s, qf, v, false, lane);
    }

    if (s.abort) {
        // not written: re-run on the next tier
        if (lane == 0) ovf[atomicAdd(ovf_count, 1)] = k;
        if (lane < 8) st[lane] = lane == 7 ? 4 : 0;
        return;
    }

    // ---- emit pairs
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(a.out_count, (unsigned long long)s.tail);
    const uint32_t blo = __shfl((uint32_t)base, 0), bhi = __shfl((uint32_t)(base >> 32), 0);
    base = ((unsigned long long)bhi << 32) | blo;
    const bool fits = base + (unsigned long long)s.tail <= (unsigned long long)a.cap;
    const bool l2 = a.metric == VJ_L2;
    if (fits) {
        for (int i = lane; i < s.tail; i += 64) {
            a.out_q[base + i] = qi;
            a.out_x[base + i] = m.il[i];
            const float kk = m.ild[i];
            a.out_d[base + i] = l2 ? sqrtf(kk) : kk;
        }
    }

    // ---- UpdateCache (read by children in a later launch)
    if (a.ws == VJ_WS_SOFT) {
        float bk = s.best_k;
        int bid = s.best_id, bx = 0;
        wave_best(bk, bid, bx, false);
        if (lane == 0) a.cache[qi] = bid == 0x7fffffff ? -1 : bid;
    } else if (a.ws == VJ_WS_HARD && lane == 0) {
        a.seg[qi] = (int64_t)base;
        a.segn[qi] = fits ? s.tail : 0;
    }

    if (lane == 0) {
        st[0] = s.tail;
        st[1] = s.ndist;
        st[2] = s.nexp;
        st[3] = s.hpops;
        st[4] = ood;
        st[5] = hyb ? 1 : 0;
        st[6] = s.nvis;
        st[7] = 0;
    }
}

// LDS variant: everything per query in static LDS (2^HL visited slots and a
// LIST-entry worklist per wave, W waves per workgroup)
template <typename T, int DP, bool HYB, int HL, int LIST, int W>
__global__ void __launch_bounds__(64 * W, 4)
k_join_lds(const JoinArgs *__restrict__ pa, const int32_t *qlist, const int32_t *qpos, int k0,
           int k1, int32_t *ovf, int32_t *ovf_count) {
    __shared__ int32_t sh_hash[W][1 << HL];
    __shared__ int32_t sh_il[W][LIST];
    __shared__ float sh_ild[W][LIST];
    __shared__ int32_t sh_stage[W][64];
    __shared__ float sh_hk[W][HYB ? kHeap : 1];
    __shared__ int32_t sh_hi[W][HYB ? kHeap : 1];
    const int lane = threadIdx.x & 63;
    const int wib = threadIdx.x >> 6;
    const int k = k0 + (int)blockIdx.x * W + wib;
    if (k >= k1) return;
    const JoinArgs &a = *pa;
    WaveMem m;
    m.hash = sh_hash[wib];
    m.hash_n = 1 << HL;
    m.hash_limit = (1 << HL) * 3 / 4 - 64;
    m.il = sh_il[wib];
    m.ild = sh_ild[wib];
    m.il_cap = LIST;
    m.stage = sh_stage[wib];
    m.hk = sh_hk[wib];
    m.hi = sh_hi[wib];
    run_query<T, DP>(a, m, k, qlist, qpos, ovf, ovf_count, lane);
}

// ---------------------------------------------------------------------------
// Cooperative tier: the W waves of one workgroup run ONE query on shared LDS
// tables (for the queries that outgrow the one-wave tier).  The in-range
// worklist is consumed in rounds: between two barriers wave 0 trims the
// out-range queue and takes a snapshot of the counters; every wave then
// takes its own NB nodes of the unprocessed part of the list.  The in-range
// closure does not depend on the order in which nodes are expanded, and the
// out-range queue holds the `beam` smallest (key, id) entries at every
// closure point whatever the insertion order, so the closure points, the
// queue at each of them and hence every pop and stop decision are those of
// a one-wave run.

template <int W> struct CoopShared {
    int tail, hc, nvis, abort;  // live counters (LDS atomics)
    int head, busy;             // BFS without rounds: next unclaimed entry, waves holding work
    int s_tail, s_hc, s_abort;  // snapshot written by wave 0 between barriers
    int hyb, ood;               // CheckHybrid decision of wave 0
    int wait;                   // persistent launch: 1 parent published, 2 deferred
    int ndist[W], nexp[W];
    float bk[W];
    int bi[W];
    unsigned long long base;    // output offset of the query's pairs
};

// per-wave running values (per lane for best_k / best_id, like QState)
struct CoopWave {
    int ndist;
    float best_k;
    int best_id;
    float d1sum;
    int c1;
    int32_t q;   // the query's node id
    float qn;    // |q| (bf16 margin of the inner product)
};

__device__ __forceinline__ int lds_load(const int *p) { return __atomic_load_n(p, __ATOMIC_RELAXED); }

// One candidate batch of one wave against the shared tables (see run_batch).
// probe: this lane's candidate is a neighbour of q in the probe of an ADAPT
// query, whose distance is needed (d1) even when it was already visited.
// Occupancy of the cooperative kernels is bound by LDS, so a pass keeps up
// to 16 16-byte loads per lane in flight.
// push_all: every newly visited node also goes to the queue (hk / hi): the
// greedy phase of separate indexes keeps in-range and out-range nodes there.
template <typename T, int DP, int W, int PGC>
__device__ __forceinline__ void coop_batch(const JoinArgs &a, const WaveMem &m, CoopShared<W> &sh,
                                           CoopWave &cw, const float *qf, int32_t v, bool probe,
                                           bool hyb_active, int heap_cap, int lane,
                                           bool push_all = false) {
    constexpr int CE = Elem<T>::CE;
    constexpr int CPR = DP / CE;
    constexpr int LPR = pick_lpr(CPR);
    constexpr int VPL = CPR / LPR;
    constexpr int RPP = 64 / LPR;
    constexpr int LCAP = kIsBf16<T> ? (PGC < 8 ? PGC : 8) : PGC;  // bf16: registers for the re-check
    constexpr int PG = (LCAP / VPL) < (64 / RPP) ? (LCAP / VPL) : (64 / RPP);
    const bool l2 = a.metric == VJ_L2;
    const int p = lane % LPR, rr = lane / LPR;
    const uint64_t ltmask = (1ull << lane) - 1ull;
    const T *vbase = reinterpret_cast<const T *>(a.rows);

    if (uni(lds_load(&sh.abort))) return;
    const bool valid = v >= 0 && v < a.nx;
    bool ovf = false;
    const bool isnew = visit(a, m, ovf, v, valid);
    const int nnew = __popcll(__ballot(isnew));
    int old = 0;
    if (lane == 0 && nnew) old = atomicAdd(&sh.nvis, nnew);
    old = uni(old);
    if (ovf || old + nnew > m.hash_limit) {
        if (lane == 0) atomicOr(&sh.abort, 1);
        return;
    }
    const bool need = probe ? valid : isnew;
    const uint64_t mneed = __ballot(need);
    const int cnt = __popcll(mneed);
    // staged entry: id, or ~id for a probe lane whose node was seen before;
    // bit 30 marks a probe lane (ids < 2^30)
    if (need) m.stage[__popcll(mneed & ltmask)] = (isnew ? v : ~v) ^ (probe ? (1 << 30) : 0);
    wave_sync();
    cw.ndist += cnt;
    for (int base = 0; base < cnt; base += RPP * PG) {
        uint4 buf[PG][VPL];
        int sid[PG];
        float2 sev[PG];  // fp8 rows: (scale, error bound) of each row
#pragma unroll
        for (int g = 0; g < PG; ++g) {
            const int c = base + g * RPP + rr;
            sid[g] = c < cnt ? m.stage[c] : 0;
            const int e = sid[g] >= 0 ? sid[g] : ~sid[g];
            const int id = e & ((1 << 30) - 1);
            const uint4 *row = reinterpret_cast<const uint4 *>(vbase + (size_t)id * DP);
#pragma unroll
            for (int w = 0; w < VPL; ++w)
                buf[g][w] = c < cnt ? row[p + w * LPR] : make_uint4(0, 0, 0, 0);
            if constexpr (kIsF8<T>) sev[g] = c < cnt ? a.f8meta[id] : make_float2(1.f, 0.f);
        }
        float keyv[PG];
        bool inrv[PG], uncv[PG];
        uint64_t unc_any = 0;
#pragma unroll
        for (int g = 0; g < PG; ++g) {
            const int c = base + g * RPP + rr;
            const bool lead = p == 0 && c < cnt;
            float acc;
            uncv[g] = false;
            if constexpr (kIsBf16<T>) {
                // |q - x~| differs from |q - x| by at most |x - x~|: for bf16
                // rows <= bf_u |x~|, for fp8 rows the bound stored with the
                // row (triangle inequality; q is exact); GB bounds the
                // relative error of the fp32 sums here and in the fp32 kernels
                constexpr float GB = (float)(2 * (VPL * CE + 5 + 16)) * 5.9604645e-8f;
                float xn2;
                float2 se = make_float2(1.f, 0.f);
                if constexpr (kIsF8<T>) se = sev[g];
                acc = row_partial_n<LPR, VPL, CE, T>(buf[g], qf, l2, xn2, se.x);
                const float xn = sqrtf(xn2) * (1.f + GB);
                const float exr = kIsF8<T> ? se.y * (1.f + GB) : a.bf_u * xn;
                bool sure;
                if (l2) {
                    const float dt = sqrtf(acc);
                    const float ex = exr;
                    const float hi = (dt * (1.f + GB) + ex) * (1.f + GB);
                    const float lo = fmaxf(0.f, dt * (1.f - GB) - ex) * (1.f - GB);
                    sure = hi * hi * (1.f + GB) < a.eps2 || lo * lo * (1.f - GB) >= a.eps2;
                } else {
                    const float mrg = kIsF8<T>
                                          ? cw.qn * (exr + 2.f * GB * xn) + GB * (1.f + fabsf(acc))
                                          : cw.qn * xn * (a.bf_u + 2.f * GB * (1.f + a.bf_u)) +
                                                GB * (1.f + fabsf(acc));
                    const float key = 1.0f - acc;
                    sure = key + mrg < a.eps || key - mrg >= a.eps;
                }
                // the greedy queue of separate indexes orders and stops by
                // the keys: those are always the fp32 kernels' values
                uncv[g] = lead && (!sure || push_all);
                unc_any |= __ballot(uncv[g]);
            } else {
                acc = row_partial<LPR, VPL, CE, T>(buf[g], qf, l2);
            }
            keyv[g] = l2 ? acc : 1.0f - acc;
            inrv[g] = l2 ? (acc < a.eps2) : (keyv[g] < a.eps);
        }
        if constexpr (kIsBf16<T>) {
            if (unc_any) {
                // re-decide the candidates inside the margin from the fp32 rows
                int nu = 0, pos[PG];
#pragma unroll
                for (int g = 0; g < PG; ++g) {
                    const uint64_t mg = __ballot(uncv[g]);
                    pos[g] = nu + __popcll(mg & ltmask);
                    if (uncv[g]) {
                        const int e = sid[g] >= 0 ? sid[g] : ~sid[g];
                        m.aux[pos[g]] = e & ((1 << 30) - 1);
                    }
                    nu += __popcll(mg);
                }
                wave_sync();
                constexpr int RPP32 = 64 / pick_lpr(DP / 4);
                constexpr int LPR32 = pick_lpr(DP / 4);
                for (int u0 = 0; u0 < nu; u0 += RPP32) {
                    const int ui = u0 + lane / LPR32;
                    const int32_t uid = ui < nu ? m.aux[ui] : 0;
                    const float v32 = fp32_value<DP>(a, cw.q, uid, l2, lane);
                    if (lane % LPR32 == 0 && ui < nu) m.auxf[ui] = v32;
                }
                wave_sync();
#pragma unroll
                for (int g = 0; g < PG; ++g) {
                    if (uncv[g]) {
                        const float v32 = m.auxf[pos[g]];
                        keyv[g] = l2 ? v32 : 1.0f - v32;
                        inrv[g] = l2 ? (v32 < a.eps2) : (keyv[g] < a.eps);
                    }
                }
                if (lane == 0) atomicAdd(a.nrecheck, (unsigned long long)nu);
                wave_sync();
            }
        }
#pragma unroll
        for (int g = 0; g < PG; ++g) {
            const int c = base + g * RPP + rr;
            const bool lead = p == 0 && c < cnt;
            const bool nw = sid[g] >= 0;
            const int e = nw ? sid[g] : ~sid[g];
            const bool pl = (e >> 30) & 1;
            const int id = e & ((1 << 30) - 1);
            const float key = keyv[g];
            const bool inr = inrv[g];
            if (lead && nw && (key < cw.best_k || (key == cw.best_k && id < cw.best_id))) {
                cw.best_k = key;
                cw.best_id = id;
            }
            if (pl && lead) {
                cw.d1sum += l2 ? sqrtf(key) : sqrtf(fmaxf(0.f, 2.f * key));
                cw.c1 += 1;
            }
            const bool ap = lead && nw && inr;
            const uint64_t ma = __ballot(ap);
            const int na = __popcll(ma);
            if (na) {
                int b0 = 0;
                if (lane == 0) b0 = atomicAdd(&sh.tail, na);
                b0 = uni(b0);
                if (b0 + na > m.il_cap) {
                    if (lane == 0) atomicOr(&sh.abort, 1);
                } else if (ap) {
                    const int o = b0 + __popcll(ma & ltmask);
                    m.il[o] = id;
                    m.ild[o] = key;
                }
            }
            if (hyb_active || push_all) {
                const bool hp = lead && nw && (push_all || !inr);
                const uint64_t mh = __ballot(hp);
                const int nh = __popcll(mh);
                if (nh) {
                    int b1 = 0;
                    if (lane == 0) b1 = atomicAdd(&sh.hc, nh);
                    b1 = uni(b1);
                    if (b1 + nh > heap_cap) {
                        if (lane == 0) atomicOr(&sh.abort, 1);
                    } else if (hp) {
                        const int o = b1 + __popcll(mh & ltmask);
                        m.hk[o] = key;
                        m.hi[o] = id;
                    }
                }
            }
        }
    }
    wave_sync();
}

// Runs slot k of the processing list on the tables of m.  Returns true
// (in every thread) when the query outgrew them: nothing was written but
// its stats row, and the caller re-runs it on larger tables.
// HYB: the kernel may run hybrid queries (an out-range queue); without it
// the hybrid code is compiled out
template <typename T, int DP, int W, int PGC, bool HYB, bool PERSIST = false>
__device__ __forceinline__ bool run_query_coop(const JoinArgs &a, const WaveMem &m,
                                               CoopShared<W> &sh, int heap_cap, int k,
                                               const int32_t *qlist, const int32_t *qpos,
                                               int flags) {
    constexpr int CE = Elem<T>::CE;
    constexpr int CPR = DP / CE;
    constexpr int LPR = pick_lpr(CPR);
    constexpr int VPL = CPR / LPR;
    constexpr int QF = VPL * CE;
    const int lane = threadIdx.x & 63;
    const int wib = threadIdx.x >> 6;
    const int R = a.R;
    const int qi = uni(qlist[k]);
    const int pos = uni(qpos[k]);
    int32_t *st = a.stats + (size_t)pos * 8;
    // whole-workgroup early exits (one query per workgroup: uniform)
    if (qi < 0 || qi >= a.nq) {
        if (threadIdx.x < 8) st[threadIdx.x] = 0;
        if (threadIdx.x == 0) atomicOr(a.err, 8);
        return false;
    }
    const int32_t q = (int32_t)(a.nx + qi);
    if (a.hyb == VJ_HYB_BUDGET && a.budget[pos] < 0) {
        if (threadIdx.x < 8) st[threadIdx.x] = threadIdx.x == 7 ? 2 : 0;
        if (threadIdx.x == 0) {
            if (a.ws == VJ_WS_SOFT) a.cache[qi] = -1;
            if (a.ws == VJ_WS_HARD) a.segn[qi] = 0;
            if (PERSIST && a.done != nullptr && (a.ws == VJ_WS_SOFT || a.ws == VJ_WS_HARD)) {
                __threadfence();
                __hip_atomic_store(&a.done[qi], (int32_t)a.gen, __ATOMIC_RELEASE,
                                   __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        return false;
    }

    float qf[QF];
    {
        const int p = lane % LPR;
        const float *qrow = a.rows32 + (size_t)q * DP;
#pragma unroll
        for (int w = 0; w < VPL; ++w) {
            const float4 *src = reinterpret_cast<const float4 *>(qrow + (p + w * LPR) * CE);
#pragma unroll
            for (int e = 0; e < CE / 4; ++e) {
                const float4 t = src[e];
                qf[w * CE + 4 * e + 0] = t.x; qf[w * CE + 4 * e + 1] = t.y;
                qf[w * CE + 4 * e + 2] = t.z; qf[w * CE + 4 * e + 3] = t.w;
            }
        }
    }
    for (int i = threadIdx.x; i < m.hash_n; i += 64 * W) m.hash[i] = -1;
    // list entries start unwritten (-1): without rounds a wave may claim an
    // entry whose slot is reserved but not yet written
    for (int i = threadIdx.x; i < m.il_cap; i += 64 * W) m.il[i] = -1;
    if (threadIdx.x == 0) {
        sh.tail = 0; sh.hc = 0; sh.nvis = 0; sh.abort = 0;
        sh.hyb = 0; sh.ood = 0;
        sh.head = 0; sh.busy = W;
        sh.wait = 0;
    }
    __syncthreads();

    CoopWave cw{};
    cw.best_k = INFINITY;
    cw.best_id = 0x7fffffff;
    cw.q = q;
    {
        float qn2 = 0.f;
#pragma unroll
        for (int i = 0; i < QF; ++i) qn2 = fmaf(qf[i], qf[i], qn2);
#pragma unroll
        for (int off = LPR / 2; off > 0; off >>= 1) qn2 += __shfl_xor(qn2, off);
        cw.qn = sqrtf(qn2) * (1.f + 1e-6f);
    }

    // ---- SeedPhase: wave 0 the entry and the soft cache, all waves the
    // parent's in-range list (hard), in chunks of 64
    int pcache = -1;
    int64_t pseg = 0;
    int pcnt = 0;
    if (a.ws == VJ_WS_SOFT || a.ws == VJ_WS_HARD) {
        const int32_t par = a.parent[qi];
        if (par >= a.nx && par < a.nx + a.nq && a.inb[par - a.nx] == (int32_t)a.gen) {
            const int pq = par - (int32_t)a.nx;
            if (PERSIST && a.done != nullptr) {
                // persistent launch: the parent's slot comes earlier in the
                // list, so a resident workgroup holds it; wait (bounded) for
                // its stamp.  A deferred parent defers this query as well.
                // (relaxed polls: an acquire per poll would invalidate the
                // XCD's L2 each time; one fence follows the stamp)
                if (threadIdx.x == 0) {
                    int st = 0, spin = 0;
                    for (;;) {
                        const int d = __hip_atomic_load(&a.done[pq], __ATOMIC_RELAXED,
                                                        __HIP_MEMORY_SCOPE_AGENT);
                        if (d == (int32_t)a.gen) { st = 1; break; }
                        if (d == ((int32_t)a.gen | kDeferred)) { st = 2; break; }
                        if (++spin > (1 << 22)) { st = 2; atomicOr(a.err, 256); break; }
                        __builtin_amdgcn_s_sleep(2);
                    }
                    sh.wait = st;
                }
                __syncthreads();
                if (sh.wait == 2) {
                    if (threadIdx.x < 8) st[threadIdx.x] = threadIdx.x == 7 ? 4 : 0;
                    return true;  // deferred: straight to the overflow list
                }
                __threadfence();
            }
            if (a.ws == VJ_WS_SOFT) {
                pcache = uni(a.cache[pq]);
            } else {
                pseg = a.seg[pq];
                pcnt = uni(a.segn[pq]);
                if (pseg < 0 || pseg + pcnt > a.cap) pcnt = 0;
            }
        }
    }
    // ---- seeds and the probe of N(q) in one batch of wave 0 (lanes 0..R-1
    // the neighbours of q, lanes R and R+1 the entry and the soft cache); the
    // other waves take the parent's in-range list (hard) meanwhile.  The
    // visited set and the in-range set after this phase are the same as
    // with seeds first, then the probe.  CheckHybrid follows on wave 0; the
    // first round's barriers publish it.
    // separate indexes launch the kernels with an out-range queue (HYB): the
    // greedy phase keeps its queue there; the BFS-only kernels compile it out
    const bool separate = HYB && a.merged == 0;
    if constexpr (HYB) {
    if (separate) {
        // ---- separate indexes: seeds {s} + the soft cache + the parent's
        // in-range list (hard, chunks of 64) on wave 0, every visited node
        // into the queue, which keeps its gbeam + 1 smallest entries (the
        // first pop's trim would drop the rest); then best-first greedy
        // with stop rules 1 and 2 (Algorithms 4-5), the queue trimmed to
        // gbeam after each pop.  The expansion starts from I alone, with the
        // greedy phase's visited set.
        if (wib == 0 && a.ws == VJ_WS_NNMAP) {
            // NN-Map (Section 6): certified empty when the witness is not
            // in range, else the witness is the only seed and the greedy
            // phase disappears; the stored OOD bit replaces d1/d2
            const bool in = a.nn_d[qi] < (double)a.eps;
            const int32_t sv = lane == 0 && in ? a.nn_w[qi] : -1;
            coop_batch<T, DP, W, PGC>(a, m, sh, cw, qf, sv, false, false, heap_cap, lane);
            if (lane == 0) {
                const bool ood = a.nn_ood[qi] != 0;
                sh.ood = a.hyb == VJ_HYB_ADAPT && ood ? 1 : 0;
                sh.hyb = a.hyb == VJ_HYB_FORCE || (a.hyb == VJ_HYB_ADAPT && ood) ||
                         (a.hyb == VJ_HYB_BUDGET && a.budget[pos] > 0);
            }
        } else if (wib == 0) {
            // the data graph's entry, or the query's own seed (the node its
            // descent through upper layers reached)
            const int32_t s0 = a.qseed ? a.qseed[qi] : a.entry;
            const int32_t sv = lane == 0 ? s0 : lane == 1 ? pcache : -1;
            coop_batch<T, DP, W, PGC>(a, m, sh, cw, qf, sv, false, false, heap_cap, lane, true);
            for (int t = 0; t < pcnt && t < a.nx + 64; t += 64) {
                const int32_t u = t + lane < pcnt ? a.out_x[pseg + t + lane] : -1;
                coop_batch<T, DP, W, PGC>(a, m, sh, cw, qf, u, false, false, heap_cap, lane, true);
                int hc = uni(lds_load(&sh.hc));
                if (hc > a.gbeam + 1) {
                    heap_trim(m, hc, a.gbeam + 1, lane);
                    if (lane == 0) sh.hc = hc;
                    wave_sync();
                }
            }
            const bool l2g = a.metric == VJ_L2;
            float best = INFINITY;
            int stall = 0, gpops = 0;
            for (int it = 0; it < m.hash_n + 4; ++it) {
                if (uni(lds_load(&sh.abort))) break;
                const int hc = uni(lds_load(&sh.hc));
                if (hc == 0) break;
                float bk = INFINITY;
                int bid = 0x7fffffff, bx = 0;
                for (int i = lane; i < hc; i += 64) {
                    const float kk = m.hk[i];
                    const int id = m.hi[i];
                    if (kk < bk || (kk == bk && id < bid)) { bk = kk; bid = id; bx = i; }
                }
                wave_best(bk, bid, bx, false);
                bid = uni(bid);
                bx = uni(bx);
                if (l2g ? bk < a.eps2 : bk < a.eps) break;          // rule 1
                if (bk < best) { best = bk; stall = 0; }
                else ++stall;
                if (a.conv > 0 && stall >= a.conv) break;           // rule 2
                if (lane == 0) {
                    m.hk[bx] = m.hk[hc - 1];
                    m.hi[bx] = m.hi[hc - 1];
                    sh.hc = hc - 1;
                }
                wave_sync();
                gpops += 1;
                if (bid < 0 || bid >= a.nx) {
                    if (lane == 0) { atomicOr(a.err, 32); atomicOr(&sh.abort, 1); }
                    break;
                }
                const int32_t v = lane < R ? a.adj[(size_t)bid * R + lane] : -1;
                coop_batch<T, DP, W, PGC>(a, m, sh, cw, qf, v, false, false, heap_cap, lane, true);
                int hc2 = uni(lds_load(&sh.hc));
                if (hc2 > a.gbeam) {
                    heap_trim(m, hc2, a.gbeam, lane);
                    if (lane == 0) sh.hc = hc2;
                    wave_sync();
                }
            }
            if (lane == 0) {
                sh.hc = 0;
                sh.ood = gpops;  // stats column 4 of separate indexes: greedy pops
                sh.hyb = a.hyb == VJ_HYB_FORCE || (a.hyb == VJ_HYB_BUDGET && a.budget[pos] > 0);
            }
        }
    }
    }
    if (!separate && wib == 0) {
        const int32_t nbq = lane < R ? a.adj[(size_t)q * R + lane] : -1;
        int32_t v = nbq;
        if (R <= 62) {
            if (lane == R) v = a.entry;
            if (lane == R + 1) v = pcache;
        } else {
            const int32_t sv = lane == 0 ? a.entry : lane == 1 ? pcache : -1;
            coop_batch<T, DP, W, PGC>(a, m, sh, cw, qf, sv, false, false, heap_cap, lane);
        }
        coop_batch<T, DP, W, PGC>(a, m, sh, cw, qf, v, a.hyb == VJ_HYB_ADAPT && lane < R, false,
                             heap_cap, lane);
        bool hyb = false;
        if (a.hyb == VJ_HYB_FORCE) {
            hyb = true;
        } else if (a.hyb == VJ_HYB_BUDGET) {
            hyb = a.budget[pos] > 0;
        } else if (a.hyb == VJ_HYB_ADAPT) {
            float s1 = cw.d1sum;
            int n1 = cw.c1;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) { s1 += __shfl_xor(s1, off); n1 += __shfl_xor(n1, off); }
            float s2 = 0.f;
            int n2 = 0;
            const int NB = 64 / R;
            for (int j0 = 0; j0 < R; j0 += NB) {
                const int b = lane / R, j = lane - b * R;
                const int yj = j0 + b;
                const bool ok = b < NB && yj < R;
                const int32_t y = __shfl(nbq, ok ? yj : 0);
                if (ok && y >= 0 && y < a.nx) {
                    const int32_t z = a.adj[(size_t)y * R + j];
                    if (z >= 0 && z < a.nx) { s2 += a.elen[(size_t)y * R + j]; n2 += 1; }
                }
            }
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) { s2 += __shfl_xor(s2, off); n2 += __shfl_xor(n2, off); }
            if (n1 == 0) hyb = true;
            else if (n2 == 0) hyb = false;
            else hyb = (s1 / (float)n1) / (s2 / (float)n2) > a.ood_ratio;
            if (lane == 0) sh.ood = hyb ? 1 : 0;
        }
        if (lane == 0) sh.hyb = hyb ? 1 : 0;
    }
    for (int t = wib * 64; !separate && t < pcnt && t < a.nx + 64; t += 64 * W) {
        const int32_t u = t + lane < pcnt ? a.out_x[pseg + t + lane] : -1;
        coop_batch<T, DP, W, PGC>(a, m, sh, cw, qf, u, false, false, heap_cap, lane);
    }
    __syncthreads();
    const bool hyb = sh.hyb != 0;
    const bool hyb_active = HYB && hyb && a.beam > 0;

    // ---- ExpansionPhase: BFS without rounds; hybrid in rounds (its queue
    // pops need the same snapshot in every wave)
    const int NB = 64 / R;
    int head = 0, unprod = 0, before = 0, hpops = 0, nexp = 0;
    bool pending = false;
    const int budget = a.hyb == VJ_HYB_BUDGET ? a.budget[pos] : 0;
    const int bound = m.il_cap + m.hash_n + 4;
    // candidates of this wave's nodes in round `head`, from [h, h + n) of
    // the list (lane b * R + j: neighbour j of node h + b)
    auto candidates = [&](int h, int n) -> int32_t {
        const int b = lane / R, j = lane - b * R;
        int32_t v = -1;
        if (b < n) {
            const int32_t u = m.il[h + b];
            if (u >= 0 && u < a.nx) v = a.adj[(size_t)u * R + j];
            else atomicOr(a.err, 32);
        }
        return v;
    };
    if (!hyb_active) {
        // BFS without rounds: the closure does not depend on the order of
        // expansion, so each wave claims the next NB listed nodes (LDS
        // compare-and-swap on head) and expands them as soon as they are
        // listed.  busy counts the waves that hold work (and may append):
        // a wave leaves when it reads busy == 0 and then nothing unclaimed.
        // Every wait is bounded (error flag 128 and abort past the bound).
        bool busy = true;
        int idle = 0;
        // claim the next NB listed nodes (lane 0; n = 0 when none is listed)
        auto claim = [&](int &h, int &n) {
            h = 0;
            n = 0;
            if (lane == 0) {
                int hh = lds_load(&sh.head);
                for (;;) {
                    const int tt = min(lds_load(&sh.tail), m.il_cap);
                    if (hh >= tt) break;
                    const int take = min(NB, tt - hh);
                    const int old = atomicCAS(&sh.head, hh, hh + take);
                    if (old == hh) { h = hh; n = take; break; }
                    hh = old;
                }
            }
            h = uni(h);
            n = uni(n);
        };
        // candidates of claimed nodes [h, h + n): lane b * R + j loads
        // neighbour j of node h + b once its entry is written
        auto load = [&](int h, int n, bool &stuck) -> int32_t {
            const int b = lane / R, j = lane - b * R;
            int32_t v = -1;
            if (b < n) {
                int32_t u = lds_load(&m.il[h + b]);
                for (int spin = 0; u < 0; ++spin) {
                    if (lds_load(&sh.abort)) break;
                    if (spin >= (1 << 20)) { stuck = true; break; }
                    __builtin_amdgcn_s_sleep(1);
                    u = lds_load(&m.il[h + b]);
                }
                if (u >= 0 && u < a.nx) v = a.adj[(size_t)u * R + j];
                else if (u >= 0) atomicOr(a.err, 32);
            }
            return v;
        };
        for (;;) {
            if (uni(lds_load(&sh.abort))) break;
            int h, n;
            claim(h, n);
            if (n > 0) {
                idle = 0;
                bool stuck = false;
                const int32_t v = load(h, n, stuck);
                if (__ballot(stuck)) {
                    if (lane == 0) { atomicOr(a.err, 128); atomicOr(&sh.abort, 1); }
                    break;
                }
                nexp += n;
                coop_batch<T, DP, W, PGC>(a, m, sh, cw, qf, v, false, false, heap_cap, lane);
                continue;
            }
            // nothing to claim: idle until work is listed or every wave is idle
            if (busy) {
                if (lane == 0) atomicSub(&sh.busy, 1);
                busy = false;
            }
            int bz = 0, hh = 0, tt = 0;
            if (lane == 0) {
                bz = lds_load(&sh.busy);
                hh = lds_load(&sh.head);
                tt = min(lds_load(&sh.tail), m.il_cap);
            }
            bz = uni(bz);
            hh = uni(hh);
            tt = uni(tt);
            if (hh < tt) {
                if (lane == 0) atomicAdd(&sh.busy, 1);
                busy = true;
                continue;
            }
            if (bz == 0) break;
            if (++idle > (1 << 20)) {
                if (lane == 0) { atomicOr(a.err, 128); atomicOr(&sh.abort, 1); }
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        if (busy && lane == 0) atomicSub(&sh.busy, 1);
    }
    int32_t pre_v = -1;  // candidates loaded one round ahead
    int pre_head = -1;   // the round (list head) they belong to
    for (int round = 0; round < bound && hyb_active; ++round) {
        __syncthreads();
        if (wib == 0) {
            if (hyb_active) {
                int hc = uni(lds_load(&sh.hc));
                if (hc > a.beam) {
                    heap_trim(m, hc, a.beam, lane);
                    if (lane == 0) sh.hc = hc;
                }
            }
            if (lane == 0) {
                sh.s_tail = lds_load(&sh.tail);
                sh.s_hc = lds_load(&sh.hc);
                sh.s_abort = lds_load(&sh.abort);
            }
        }
        __syncthreads();
        const int t = min(uni(sh.s_tail), m.il_cap);
        const int hc = uni(sh.s_hc);
        if (uni(sh.s_abort)) break;
        if (head < t) {
            const int take = min(W * NB, t - head);
            const int my0 = head + wib * NB;
            const int nmine = max(0, min(NB, head + take - my0));
            // a prefetch is only made for a round whose nodes were all known
            const int32_t v = pre_head == head ? pre_v : candidates(my0, nmine);
            // the next round takes W * NB nodes whatever this round appends
            // if that many are already listed: load their candidates now
            const int h2 = head + take;
            if (t - h2 >= W * NB) {
                pre_v = candidates(h2 + wib * NB, NB);
                pre_head = h2;
            }
            if (nmine > 0) {
                nexp += nmine;
                coop_batch<T, DP, W, PGC>(a, m, sh, cw, qf, v, false, hyb_active, heap_cap, lane);
            }
            head += take;
            continue;
        }
        // closure point: the same decision in every wave
        if (pending) { unprod = (t == before) ? unprod + 1 : 0; pending = false; }
        if (!hyb_active || hc == 0) break;
        if (a.hyb == VJ_HYB_BUDGET) { if (hpops >= budget) break; }
        else if (a.conv > 0 && unprod >= a.conv) break;
        hpops += 1;
        before = t;
        pending = true;
        if (wib == 0) {
            float bk = INFINITY;
            int bid = 0x7fffffff, bx = 0;
            for (int i = lane; i < hc; i += 64) {
                const float kk = m.hk[i];
                const int id = m.hi[i];
                if (kk < bk || (kk == bk && id < bid)) { bk = kk; bid = id; bx = i; }
            }
            wave_best(bk, bid, bx, false);
            bid = uni(bid);
            bx = uni(bx);
            if (lane == 0) {
                m.hk[bx] = m.hk[hc - 1];
                m.hi[bx] = m.hi[hc - 1];
                sh.hc = hc - 1;
            }
            wave_sync();
            nexp += 1;
            if (bid < 0 || bid >= a.nx) {
                if (lane == 0) { atomicOr(a.err, 32); atomicOr(&sh.abort, 1); }
            } else {
                const int32_t v = lane < R ? a.adj[(size_t)bid * R + lane] : -1;
                coop_batch<T, DP, W, PGC>(a, m, sh, cw, qf, v, false, hyb_active, heap_cap, lane);
            }
        }
    }
    {
        float bk = cw.best_k;
        int bid = cw.best_id, bx = 0;
        wave_best(bk, bid, bx, false);
        if (lane == 0) {
            sh.ndist[wib] = cw.ndist;
            sh.nexp[wib] = nexp;
            sh.bk[wib] = bk;
            sh.bi[wib] = bid;
        }
    }
    __syncthreads();
    const int tail = min(lds_load(&sh.tail), m.il_cap);
    if (lds_load(&sh.abort)) {
        if (threadIdx.x < 8) st[threadIdx.x] = threadIdx.x == 7 ? 4 : 0;
        return true;
    }

    // ---- emit pairs
    if (threadIdx.x == 0) sh.base = atomicAdd(a.out_count, (unsigned long long)tail);
    __syncthreads();
    const unsigned long long base = sh.base;
    const bool fits = base + (unsigned long long)tail <= (unsigned long long)a.cap;
    const bool l2 = a.metric == VJ_L2;
    if (fits) {
        for (int i = threadIdx.x; i < tail; i += 64 * W) {
            a.out_q[base + i] = qi;
            a.out_x[base + i] = m.il[i];
            const float kk = m.ild[i];
            a.out_d[base + i] = l2 ? sqrtf(kk) : kk;
        }
    }
    if (threadIdx.x == 0) {
        float bk = INFINITY;
        int bid = 0x7fffffff, nd = 0, ne = 0;
        for (int w = 0; w < W; ++w) {
            if (sh.bk[w] < bk || (sh.bk[w] == bk && sh.bi[w] < bid)) { bk = sh.bk[w]; bid = sh.bi[w]; }
            nd += sh.ndist[w];
            ne += sh.nexp[w];
        }
        // ---- UpdateCache
        if (a.ws == VJ_WS_SOFT) a.cache[qi] = bid == 0x7fffffff ? -1 : bid;
        else if (a.ws == VJ_WS_HARD) {
            a.seg[qi] = (int64_t)base;
            a.segn[qi] = fits ? tail : 0;
        }
        st[0] = tail;
        st[1] = nd;
        st[2] = ne;
        st[3] = hpops;
        st[4] = sh.ood;
        st[5] = hyb ? 1 : 0;
        st[6] = lds_load(&sh.nvis);
        st[7] = flags;
    }
    if (PERSIST && a.done != nullptr && (a.ws == VJ_WS_SOFT || a.ws == VJ_WS_HARD)) {
        // publish: every thread's pair writes, then the cache / segment, then
        // the stamp (release at device scope)
        __threadfence();
        __syncthreads();
        if (threadIdx.x == 0)
            __hip_atomic_store(&a.done[qi], (int32_t)a.gen, __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
    return false;
}

// Global tables of one query: 2^hash_log2 visited slots and il_cap in-range
// entries in region r of gh / gil / gild.
struct GlobalTables {
    int32_t *gh;
    int32_t *gil;
    float *gild;
    int hash_log2, il_cap;
    int32_t *next;  // slot counter of in-launch promotion
    int cap;        // regions available to it
};

__device__ __forceinline__ void use_global(WaveMem &m, const GlobalTables &g, size_t r) {
    m.hash = g.gh + (r << g.hash_log2);
    m.hash_n = 1 << g.hash_log2;
    m.hash_limit = (1 << g.hash_log2) / 2;
    m.il = g.gil + r * (size_t)g.il_cap;
    m.ild = g.gild + r * (size_t)g.il_cap;
    m.il_cap = g.il_cap;
}

// cooperative tier: one query per workgroup of W waves, 2^HL visited slots
// and LIST in-range entries in LDS.  A query that outgrows them takes a free
// region of global tables (if any is left) and runs again in this launch;
// otherwise, or if it outgrows those too, its slot goes to the overflow list.
// claim: persistent launch -- each workgroup claims slots in list order from
// the counter until they run out (null: one workgroup per slot).
template <typename T, int DP, bool HYB, int HS, int LIST, int W, int PGC, int MINW,
          bool PERSIST = false>
__global__ void __launch_bounds__(64 * W, MINW)
k_join_coop(const JoinArgs *__restrict__ pa, const int32_t *qlist, const int32_t *qpos, int k0,
            int k1, const int32_t *cnt_dev, GlobalTables g, int32_t *ovf, int32_t *ovf_count,
            int32_t *claim) {
    constexpr int HC = HYB ? kBeamMax + 64 * W : 1;
    __shared__ int32_t sh_hash[HS];
    __shared__ int32_t sh_il[LIST];
    __shared__ float sh_ild[LIST];
    __shared__ int32_t sh_stage[W][64];
    __shared__ float sh_hk[HC];
    __shared__ int32_t sh_hi[HC];
    __shared__ CoopShared<W> sh;
    __shared__ int sh_region;
    __shared__ int32_t sh_aux[kIsBf16<T> ? W : 1][64];
    __shared__ float sh_auxf[kIsBf16<T> ? W : 1][64];
    __shared__ int sh_k;
    const int kend = cnt_dev != nullptr ? min(k1, k0 + *cnt_dev) : k1;
    const JoinArgs &a = *pa;
    WaveMem m;
    m.hash = sh_hash;
    m.hash_n = HS;
    m.hash_limit = HS * 3 / 4 - 64 * W;
    m.il = sh_il;
    m.ild = sh_ild;
    m.il_cap = LIST;
    m.stage = sh_stage[threadIdx.x >> 6];
    m.hk = sh_hk;
    m.hi = sh_hi;
    m.aux = sh_aux[kIsBf16<T> ? threadIdx.x >> 6 : 0];
    m.auxf = sh_auxf[kIsBf16<T> ? threadIdx.x >> 6 : 0];
    if constexpr (!PERSIST) {
        // one workgroup per slot
        const int k = k0 + (int)blockIdx.x;
        if (k >= kend) return;
        if (!run_query_coop<T, DP, W, PGC, HYB>(a, m, sh, HC, k, qlist, qpos, 1)) return;
        if (threadIdx.x == 0) sh_region = g.cap > 0 ? atomicAdd(g.next, 1) : 0;
        __syncthreads();
        const int r = sh_region;
        bool again = true;
        if (r < g.cap) {
            use_global(m, g, (size_t)r);
            again = run_query_coop<T, DP, W, PGC, HYB>(a, m, sh, HC, k, qlist, qpos, 1 | 8);
        }
        if (again && threadIdx.x == 0) ovf[atomicAdd(ovf_count, 1)] = k;
    } else {
        // persistent: claim slots in list order until they run out
        const WaveMem lds = m;
        for (;;) {
            if (threadIdx.x == 0) sh_k = k0 + atomicAdd(claim, 1);
            __syncthreads();
            const int k = sh_k;
            __syncthreads();  // every thread read sh_k before the next claim
            if (k >= kend) break;
            m = lds;
            if (!run_query_coop<T, DP, W, PGC, HYB, true>(a, m, sh, HC, k, qlist, qpos, 1)) continue;
            // a deferred query (its parent was deferred) takes no region
            const bool deferred = a.done != nullptr && sh.wait == 2;
            if (threadIdx.x == 0) sh_region = g.cap > 0 && !deferred ? atomicAdd(g.next, 1) : g.cap;
            __syncthreads();
            const int r = sh_region;
            bool again = true;
            if (r < g.cap) {
                use_global(m, g, (size_t)r);
                again = run_query_coop<T, DP, W, PGC, HYB, true>(a, m, sh, HC, k, qlist, qpos, 1 | 8);
            }
            if (again && threadIdx.x == 0) {
                ovf[atomicAdd(ovf_count, 1)] = k;
                if (a.done != nullptr && (a.ws == VJ_WS_SOFT || a.ws == VJ_WS_HARD))
                    __hip_atomic_store(&a.done[uni(qlist[k])], (int32_t)a.gen | kDeferred,
                                       __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
            __syncthreads();  // the next query clears the tables
        }
    }
}

// cooperative tier on global tables: one query at a time per workgroup of W
// waves, its tables in region (block index) of g; a workgroup takes the
// entries k0 + blockIdx.x, + gridDim.x, ... below k1 (and below k0 +
// *cnt_dev when the count is on the device).  Entry k is slot k of qlist, or
// slot slots[k] when a slot list is given; overflowing slots are appended
// to ovf as slots of qlist.
template <typename T, int DP, bool HYB, int W, int PGC>
__global__ void __launch_bounds__(64 * W)
k_join_coop_global(const JoinArgs *__restrict__ pa, const int32_t *qlist, const int32_t *qpos,
                   const int32_t *slots, int k0, int k1, const int32_t *cnt_dev, GlobalTables g,
                   int32_t *ovf, int32_t *ovf_count) {
    constexpr int HC = HYB ? kBeamMax + 64 * W : 1;
    __shared__ int32_t sh_stage[W][64];
    __shared__ float sh_hk[HC];
    __shared__ int32_t sh_hi[HC];
    __shared__ CoopShared<W> sh;
    __shared__ int32_t sh_aux[kIsBf16<T> ? W : 1][64];
    __shared__ float sh_auxf[kIsBf16<T> ? W : 1][64];
    const int kend = cnt_dev != nullptr ? min(k1, k0 + *cnt_dev) : k1;
    const JoinArgs &a = *pa;
    WaveMem m;
    use_global(m, g, blockIdx.x);
    m.stage = sh_stage[threadIdx.x >> 6];
    m.hk = sh_hk;
    m.hi = sh_hi;
    m.aux = sh_aux[kIsBf16<T> ? threadIdx.x >> 6 : 0];
    m.auxf = sh_auxf[kIsBf16<T> ? threadIdx.x >> 6 : 0];
    for (int k = k0 + (int)blockIdx.x; k < kend; k += (int)gridDim.x) {
        const int slot = slots != nullptr ? slots[k] : k;
        if (run_query_coop<T, DP, W, PGC, HYB>(a, m, sh, HC, slot, qlist, qpos, 1 | 8 | 16) &&
            threadIdx.x == 0)
            ovf[atomicAdd(ovf_count, 1)] = slot;
        __syncthreads();  // the next query clears the region's tables
    }
}

template <typename T, int DP, bool HYB>
void launch_tier(const JoinLaunch &L, hipStream_t s) {
    const int k0 = L.first, k1 = L.first + L.count;
    if (L.tier == 0) {
        // the one-wave tier reads fp32 or exact u8 rows only
        if constexpr (!kIsBf16<T>) {
            const unsigned blocks = (unsigned)((L.count + kWaves - 1) / kWaves);
            hipLaunchKernelGGL((k_join_lds<T, DP, HYB, 10, 512, kWaves>), dim3(blocks),
                               dim3(64 * kWaves), 0, s, L.args, L.qlist, L.qpos, k0, k1, L.ovf,
                               L.ovf_count);
        }
    } else {
        GlobalTables g;
        g.gh = L.gh;
        g.gil = L.gil;
        g.gild = L.gild;
        g.hash_log2 = L.hash_log2;
        g.il_cap = L.il_cap;
        g.next = L.promo_next;
        g.cap = L.promo_cap;
        // workgroup tier: large LDS tables (8,192 visited slots, 768 in-range
        // pairs: 40 KB, four workgroups per CU) or small ones (4,096 slots,
        // 1,024 pairs); both cap registers at 128 for four waves per SIMD
        // up to 256-wide rows.  The visited set fills first: a query visits
        // about 15 nodes per in-range node
        // grid: one workgroup per slot, or L.grid workgroups looping over
        // the slots (global tables: one region per workgroup)
        const unsigned blocks = (unsigned)(L.grid > 0 ? L.grid : L.count);
        // tier 1: one workgroup per slot, or a persistent grid claiming slots
        const unsigned t1grid = (unsigned)(L.claim != nullptr && L.grid > 0 ? L.grid : L.count);
        if (L.tier == 1 && L.coop_small)
            // one workgroup per slot (the small tables have no persistent form)
            hipLaunchKernelGGL((k_join_coop<T, DP, HYB, 4096, 1024, kWaves, 12, (DP <= 256 ? 4 : 1)>),
                               dim3((unsigned)L.count), dim3(64 * kWaves), 0, s, L.args, L.qlist,
                               L.qpos, k0, k1, L.count_dev, g, L.ovf, L.ovf_count, nullptr);
        else if (L.tier == 1 && L.claim != nullptr) {
            // persistent: resident workgroups claim the slots in order
            if constexpr (kIsBf16<T> && DP <= 256)
                hipLaunchKernelGGL((k_join_coop<T, DP, HYB, 7680, 768, kWaves, 4, 4, true>),
                                   dim3(t1grid), dim3(64 * kWaves), 0, s, L.args,
                                   L.qlist, L.qpos, k0, k1, L.count_dev, g, L.ovf, L.ovf_count,
                                   L.claim);
            else
                hipLaunchKernelGGL((k_join_coop<T, DP, HYB, 8192, 768, kWaves, 12, (DP <= 256 ? 4 : 1), true>),
                                   dim3(t1grid), dim3(64 * kWaves), 0, s, L.args,
                                   L.qlist, L.qpos, k0, k1, L.count_dev, g, L.ovf, L.ovf_count,
                                   L.claim);
        } else if (L.tier == 1) {
            if constexpr (kIsBf16<T> && DP <= 256)
                // bf16 rows: the re-check buffers take 2 KB of LDS and the
                // margin registers, so 7,680 visited slots and 4 loads per
                // lane in flight keep four workgroups per CU (a row takes at
                // most 4 loads per lane up to 256 wide)
                hipLaunchKernelGGL((k_join_coop<T, DP, HYB, 7680, 768, kWaves, 4, 4>),
                                   dim3(t1grid), dim3(64 * kWaves), 0, s, L.args,
                                   L.qlist, L.qpos, k0, k1, L.count_dev, g, L.ovf, L.ovf_count,
                                   L.claim);
            else
                hipLaunchKernelGGL((k_join_coop<T, DP, HYB, 8192, 768, kWaves, 12, (DP <= 256 ? 4 : 1)>),
                                   dim3(t1grid), dim3(64 * kWaves), 0, s, L.args,
                                   L.qlist, L.qpos, k0, k1, L.count_dev, g, L.ovf, L.ovf_count,
                                   L.claim);
        }
        else
            hipLaunchKernelGGL((k_join_coop_global<T, DP, HYB, kWaves, 16>), dim3(blocks),
                               dim3(64 * kWaves), 0, s, L.args, L.qlist, L.qpos, L.slots, k0, k1,
                               L.count_dev, g, L.ovf, L.ovf_count);
    }
}

template <typename T, int DP>
bool launch_dp(const JoinLaunch &L, hipStream_t s) {
    if (L.count <= 0) return true;
    if (L.hyb) launch_tier<T, DP, true>(L, s);
    else launch_tier<T, DP, false>(L, s);
    return true;
}

template <typename T>
bool launch_elem(const JoinLaunch &L, hipStream_t s) {
    switch (L.dp) {
    case 32: return launch_dp<T, 32>(L, s);
    case 64: return launch_dp<T, 64>(L, s);
    case 96: return launch_dp<T, 96>(L, s);
    case 128: return launch_dp<T, 128>(L, s);
    case 192: return launch_dp<T, 192>(L, s);
    case 256: return launch_dp<T, 256>(L, s);
    case 384: return launch_dp<T, 384>(L, s);
    case 512: return launch_dp<T, 512>(L, s);
    case 768: return launch_dp<T, 768>(L, s);
    case 1024: return launch_dp<T, 1024>(L, s);
    default: return false;
    }
}

}  // namespace wj
}  // namespace vj
