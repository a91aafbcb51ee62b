// Persistent merged-index join kernel (the online path of Algorithm 1 with
// cfg.merged = true, Sections 4.1-4.4).  Included by one translation unit per
// element type so the variants compile in parallel.
//
// Shape: every wavefront (64 lanes) owns one query at a time and pulls the
// next one from an atomic counter, so queries of very different result sizes
// share one launch.  Per query:
//   seeds      {s} (+ the parent's cached node in soft mode, its result in
//              hard mode)                                   Algorithm 3
//   probe      the neighbours of the query node q           Algorithms 4-5
//   check      d1/d2 OOD test or a per-query budget         Algorithm 6
//   expand     in-range data nodes to closure; in hybrid mode the closest
//              out-range node of a bounded queue is expanded whenever the
//              in-range worklist is empty                   Algorithm 7
//   cache      closest visited data node (soft)             Algorithm 8
// Candidate ids are checked against a visited hash that lives in LDS (or in
// a per-wave global table on the spill path), new ids are compacted, and
// their rows are gathered LPR lanes per row (16 bytes per lane per load, so
// every load instruction of a row group covers whole 128-byte lines) and
// reduced with xor shuffles inside the lane group.
#pragma once

#include "vj_internal.h"

namespace vj {
namespace trav {

constexpr int32_t kAborted = 0x7ffffffe;

template <typename T> struct Elem;
template <> struct Elem<float> { static constexpr int CE = 4; };
template <> struct Elem<uint16_t> { static constexpr int CE = 8; };   // bf16 bits
template <> struct Elem<uint8_t> { static constexpr int CE = 16; };

// lanes per row: 16-byte chunks per lane kept <= 8, groups a power of two
constexpr int pick_lpr(int cpr) {
    int l = 8;
    while (l > 1 && cpr % l) l >>= 1;
    if (cpr / l > 8) {
        l = 16;
        while ((l < 64) && (cpr % l || cpr / l > 8)) l <<= 1;
    }
    return l;
}

__device__ __forceinline__ void chunk_to_float(const uint4 &r, float *f, float) {
    f[0] = __uint_as_float(r.x); f[1] = __uint_as_float(r.y);
    f[2] = __uint_as_float(r.z); f[3] = __uint_as_float(r.w);
}
__device__ __forceinline__ void chunk_to_float(const uint4 &r, float *f, uint16_t) {
    const uint32_t w[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        f[2 * i] = __uint_as_float(w[i] << 16);
        f[2 * i + 1] = __uint_as_float(w[i] & 0xffff0000u);
    }
}
__device__ __forceinline__ void chunk_to_float(const uint4 &r, float *f, uint8_t) {
    const uint32_t w[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        f[4 * i + 0] = (float)(w[i] & 0xffu);
        f[4 * i + 1] = (float)((w[i] >> 8) & 0xffu);
        f[4 * i + 2] = (float)((w[i] >> 16) & 0xffu);
        f[4 * i + 3] = (float)(w[i] >> 24);
    }
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ uint32_t hash32(uint32_t v) { return v * 0x9E3779B1u; }

__device__ __forceinline__ int bcast(int v) { return __shfl(v, 0); }

// wave-wide reduction of (key, id, slot) keeping the min (or max) by (key, id)
__device__ __forceinline__ void wave_argbest(float &k, int &id, int &slot, bool want_max) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        float ok = __shfl_xor(k, off);
        int oid = __shfl_xor(id, off);
        int os = __shfl_xor(slot, off);
        bool take = want_max ? (ok > k || (ok == k && oid > id)) : (ok < k || (ok == k && oid < id));
        if (take) { k = ok; id = oid; slot = os; }
    }
}

template <typename T, int DP, bool SPILL>
__global__ void __launch_bounds__(256) k_traverse(TraverseLaunch a) {
    constexpr int CE = Elem<T>::CE;
    constexpr int CPR = DP / CE;
    constexpr int LPR = pick_lpr(CPR);
    constexpr int VPL = CPR / LPR;
    static_assert(VPL * LPR == CPR, "row split");
    constexpr int RPP = 64 / LPR;
    constexpr int PG = VPL >= 8 ? 1 : 8 / VPL;
    constexpr int QF = VPL * CE;

    extern __shared__ int32_t lds[];
    const int lane = threadIdx.x & 63;
    const int wib = threadIdx.x >> 6;
    const int slot = blockIdx.x * (blockDim.x >> 6) + wib;
    const int p = lane % LPR, rr = lane / LPR;
    const uint64_t ltmask = (1ull << lane) - 1ull;
    const int HS = 1 << a.hash_log2;
    const int hmask = HS - 1;
    const int R = a.R;
    const bool l2 = a.metric == VJ_L2;

    int32_t *wl = lds + wib * a.lds_ints_per_wave;
    int32_t *htab = wl;
    int32_t *stage = wl + (SPILL ? 0 : HS);
    float *hkey = reinterpret_cast<float *>(stage + 64);
    int32_t *hid = reinterpret_cast<int32_t *>(hkey + a.beam + 64);
    unsigned long long *gtab =
        SPILL ? reinterpret_cast<unsigned long long *>(a.ghash) + (size_t)slot * HS : nullptr;
    int32_t *il_id = a.il_id + (size_t)slot * a.il_cap;
    float *il_d = a.il_d + (size_t)slot * a.il_cap;
    const T *vbase = reinterpret_cast<const T *>(a.vec);

    for (;;) {
        int k = 0;
        if (lane == 0) k = atomicAdd(a.work, 1);
        k = bcast(k);
        if (k >= a.n) break;

        const int qi = a.qlist[k];
        const int pos = a.qpos[k];
        if (qi < 0 || qi >= a.nq) {
            if (lane == 0) {
                atomicOr(a.err, 8);
                int32_t *st = a.stats + (size_t)pos * 8;
                for (int t = 0; t < 8; ++t) st[t] = 0;
            }
            continue;
        }
        const int32_t q = (int32_t)(a.nx + qi);

        // routed to the brute-force tiles by a negative budget: no traversal
        if (a.hyb == VJ_HYB_BUDGET && a.budget[pos] < 0) {
            if (a.ws != VJ_WS_SELF && lane == 0)
                __hip_atomic_store(&a.pub[qi], ((unsigned long long)a.gen << 32) | 0xffffffffull,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (lane == 0) {
                int32_t *st = a.stats + (size_t)pos * 8;
                for (int t = 0; t < 7; ++t) st[t] = 0;
                st[7] = 2;
            }
            continue;
        }

        // the query's slice of dimensions, fp32
        float qf[QF];
        {
            const float *qrow = a.vec32 + (size_t)q * DP;
#pragma unroll
            for (int v = 0; v < VPL; ++v) {
                const float4 *src = reinterpret_cast<const float4 *>(qrow + (p + v * LPR) * CE);
#pragma unroll
                for (int e = 0; e < CE / 4; ++e) {
                    float4 t = src[e];
                    qf[v * CE + 4 * e + 0] = t.x; qf[v * CE + 4 * e + 1] = t.y;
                    qf[v * CE + 4 * e + 2] = t.z; qf[v * CE + 4 * e + 3] = t.w;
                }
            }
        }

        // fresh visited set
        uint32_t stamp = 0;
        if (!SPILL) {
            for (int i = lane; i < HS; i += 64) htab[i] = -1;
        } else {
            if (lane == 0) stamp = ++a.gstamp[slot];
            stamp = (uint32_t)bcast((int)stamp);
        }
        wave_sync();

        int tail = 0, head = 0, hc = 0;
        int nvis = 0, ndist = 0, nexp = 0, hpops = 0;
        bool abort = false, hyb = false, hyb_active = false;
        float best_k = INFINITY;
        int best_id = 0x7fffffff;
        float d1sum = 0.f;
        int c1 = 0;

        // insert a lane's candidate into the visited set; true if it was new
        auto visit = [&](int32_t v, bool active) -> bool {
            bool isnew = false;
            uint32_t h = hash32((uint32_t)v) >> (32 - a.hash_log2);
            for (;;) {
                if (__ballot(active) == 0) break;
                if (active) {
                    if (!SPILL) {
                        int old = atomicCAS(&htab[h], -1, v);
                        if (old == -1) { isnew = true; active = false; }
                        else if (old == v) active = false;
                        else h = (h + 1) & hmask;
                    } else {
                        unsigned long long cur =
                            __hip_atomic_load(&gtab[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                        if ((uint32_t)(cur >> 32) == stamp) {
                            if ((int32_t)(uint32_t)cur == v) active = false;
                            else h = (h + 1) & hmask;
                        } else {
                            unsigned long long nv = ((unsigned long long)stamp << 32) | (uint32_t)v;
                            if (atomicCAS(&gtab[h], cur, nv) == cur) { isnew = true; active = false; }
                        }
                    }
                }
            }
            return isnew;
        };

        auto heap_trim = [&]() {
            while (hc > a.beam) {
                float bk = -INFINITY;
                int bid = -1, bs = -1;
                for (int i = lane; i < hc; i += 64) {
                    float kk = hkey[i];
                    int id = hid[i];
                    if (kk > bk || (kk == bk && id > bid)) { bk = kk; bid = id; bs = i; }
                }
                wave_argbest(bk, bid, bs, true);
                if (lane == 0) { hkey[bs] = hkey[hc - 1]; hid[bs] = hid[hc - 1]; }
                --hc;
                wave_sync();
            }
        };

        // one batch: <= 1 candidate per lane.  probe: distances for every
        // valid data candidate (the d1 feature needs them), not only new ones
        auto run_batch = [&](int32_t v, bool probe) {
            const bool valid = v >= 0 && v < a.nx;
            const bool isnew = visit(v, valid);
            nvis += __popcll(__ballot(isnew));
            if (nvis > a.hash_limit) { abort = true; return; }
            const bool need = probe ? valid : isnew;
            const uint64_t mneed = __ballot(need);
            const int cnt = __popcll(mneed);
            if (need) stage[__popcll(mneed & ltmask)] = isnew ? v : ~v;
            wave_sync();
            ndist += cnt;
            for (int base = 0; base < cnt; base += RPP * PG) {
                uint4 buf[PG][VPL];
                int sid[PG];
#pragma unroll
                for (int g = 0; g < PG; ++g) {
                    const int c = base + g * RPP + rr;
                    sid[g] = c < cnt ? stage[c] : 0;
                    const int id = sid[g] >= 0 ? sid[g] : ~sid[g];
                    const uint4 *row = reinterpret_cast<const uint4 *>(vbase + (size_t)id * DP);
#pragma unroll
                    for (int w = 0; w < VPL; ++w)
                        buf[g][w] = c < cnt ? row[p + w * LPR] : make_uint4(0, 0, 0, 0);
                }
#pragma unroll
                for (int g = 0; g < PG; ++g) {
                    float acc = 0.f;
#pragma unroll
                    for (int w = 0; w < VPL; ++w) {
                        float f[CE];
                        chunk_to_float(buf[g][w], f, T());
#pragma unroll
                        for (int e = 0; e < CE; ++e) {
                            if (l2) { float t = f[e] - qf[w * CE + e]; acc = fmaf(t, t, acc); }
                            else acc = fmaf(f[e], qf[w * CE + e], acc);
                        }
                    }
#pragma unroll
                    for (int off = LPR / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
                    const int c = base + g * RPP + rr;
                    const bool lead = p == 0 && c < cnt;
                    const bool nw = sid[g] >= 0;
                    const int id = nw ? sid[g] : ~sid[g];
                    const float key = l2 ? acc : 1.0f - acc;
                    const bool inr = l2 ? (acc < a.eps2) : (key < a.eps);
                    if (lead && nw && (key < best_k || (key == best_k && id < best_id))) {
                        best_k = key;
                        best_id = id;
                    }
                    if (probe && lead) {
                        d1sum += l2 ? sqrtf(key) : sqrtf(fmaxf(0.f, 2.f * key));
                        c1 += 1;
                    }
                    const bool ap = lead && nw && inr;
                    const uint64_t ma = __ballot(ap);
                    const int na = __popcll(ma);
                    if (tail + na > a.il_cap) {
                        abort = true;
                    } else {
                        if (ap) {
                            const int o = tail + __popcll(ma & ltmask);
                            il_id[o] = id;
                            il_d[o] = key;
                        }
                        tail += na;
                    }
                    if (hyb_active) {
                        const bool hp = lead && nw && !inr;
                        const uint64_t mh = __ballot(hp);
                        if (hp) {
                            const int o = hc + __popcll(mh & ltmask);
                            hkey[o] = key;
                            hid[o] = id;
                        }
                        hc += __popcll(mh);
                    }
                }
                if (hyb_active && hc > a.beam) { wave_sync(); heap_trim(); }
            }
            wave_sync();
        };

        // ---- SeedPhase: s, plus the parent's cache in soft / hard mode
        int pcache = -1;
        int64_t pseg = 0;
        int pcnt = 0;
        if (a.ws != VJ_WS_SELF) {
            const int32_t par = a.parent[qi];
            if (par >= 0 && a.inb[par - a.nx] == (int32_t)a.gen_first) {
                const int pq = par - (int32_t)a.nx;
                unsigned long long pv = 0;
                int spins = 0;
                // a parent processed at level j publishes (gen_first + j, node);
                // one that overflowed publishes kAborted and is re-run at a
                // later level of this call, parents before children
                const uint32_t lvl = a.gen - a.gen_first;
                for (;;) {
                    pv = __hip_atomic_load(&a.pub[pq], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    const uint32_t hi = (uint32_t)(pv >> 32);
                    const int32_t lo = (int32_t)(uint32_t)pv;
                    const uint32_t rel = hi - a.gen_first;
                    if (rel <= lvl && lo != kAborted) break;
                    if (rel == lvl && lo == kAborted) break;
                    if (++spins > (1 << 26)) { if (lane == 0) atomicOr(a.err, 2); pv = 0; break; }
                    __builtin_amdgcn_s_sleep(2);
                }
                const uint32_t rel = (uint32_t)(pv >> 32) - a.gen_first;
                const int32_t lo = (int32_t)(uint32_t)pv;
                if (rel <= lvl && lo == kAborted) {
                    abort = true;  // the parent moves to the next level: so does the child
                } else if (rel <= lvl) {
                    if (a.ws == VJ_WS_HARD) {
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                        pseg = a.seg[pq];
                        pcnt = a.segn[pq];
                    } else {
                        pcache = lo;
                    }
                }
            }
        }
        if (!abort) {
            int32_t v = -1;
            if (lane == 0) v = a.entry;
            if (lane == 1) v = pcache;
            run_batch(v, false);
            for (int t = 0; !abort && t < pcnt; t += 64) {
                int32_t u = t + lane < pcnt ? a.out_x[pseg + t + lane] : -1;
                run_batch(u, false);
            }
        }

        // ---- GreedySearchPhase on the merged index: probe N(q), then stop
        const int32_t nbq = lane < R ? a.adj[(size_t)q * R + lane] : -1;
        if (!abort) run_batch(nbq, a.hyb == VJ_HYB_ADAPT);

        // ---- CheckHybrid
        int ood = 0;
        if (!abort) {
            if (a.hyb == VJ_HYB_FORCE) {
                hyb = true;
            } else if (a.hyb == VJ_HYB_BUDGET) {
                hyb = a.budget[pos] > 0;
            } else if (a.hyb == VJ_HYB_ADAPT) {
                // d2: mean edge length from q's data neighbours to their data neighbours
                float s1 = d1sum;
                for (int off = 32; off > 0; off >>= 1) s1 += __shfl_xor(s1, off);
                int n1 = c1;
                for (int off = 32; off > 0; off >>= 1) n1 += __shfl_xor(n1, off);
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
                        if (z >= 0 && z < a.nx && z != q) {
                            s2 += a.elen[(size_t)y * R + j];
                            n2 += 1;
                        }
                    }
                }
                for (int off = 32; off > 0; off >>= 1) s2 += __shfl_xor(s2, off);
                for (int off = 32; off > 0; off >>= 1) n2 += __shfl_xor(n2, off);
                if (n1 == 0) hyb = true;
                else if (n2 == 0) hyb = false;
                else hyb = (s1 / (float)n1) / (s2 / (float)n2) > a.ood_ratio;
                ood = hyb ? 1 : 0;
            }
        }
        hyb_active = hyb && a.beam > 0;

        // ---- ExpansionPhase
        const int NB = 64 / R;
        int unprod = 0, before = 0;
        bool pending = false;
        while (!abort) {
            while (!abort && head < tail) {
                wave_sync();
                const int nb = min(NB, tail - head);
                const int b = lane / R, j = lane - b * R;
                int32_t v = -1;
                if (b < nb) {
                    const int32_t u = il_id[head + b];
                    v = a.adj[(size_t)u * R + j];
                }
                head += nb;
                nexp += nb;
                run_batch(v, false);
            }
            if (abort) break;
            if (pending) { unprod = (tail == before) ? unprod + 1 : 0; pending = false; }
            if (!hyb_active || hc == 0) break;
            if (a.hyb == VJ_HYB_BUDGET) { if (hpops >= a.budget[pos]) break; }
            else if (a.conv > 0 && unprod >= a.conv) break;
            // pop the closest out-range node
            float bk = INFINITY;
            int bid = 0x7fffffff, bs = -1;
            for (int i = lane; i < hc; i += 64) {
                const float kk = hkey[i];
                const int id = hid[i];
                if (kk < bk || (kk == bk && id < bid)) { bk = kk; bid = id; bs = i; }
            }
            wave_argbest(bk, bid, bs, false);
            if (lane == 0) { hkey[bs] = hkey[hc - 1]; hid[bs] = hid[hc - 1]; }
            --hc;
            wave_sync();
            ++hpops;
            ++nexp;
            before = tail;
            pending = true;
            const int32_t v = lane < R ? a.adj[(size_t)bid * R + lane] : -1;
            run_batch(v, false);
        }

        // ---- emit pairs
        if (!abort) {
            wave_sync();
            unsigned long long base = 0;
            if (lane == 0) base = atomicAdd(a.out_count, (unsigned long long)tail);
            const uint32_t blo = __shfl((uint32_t)base, 0), bhi = __shfl((uint32_t)(base >> 32), 0);
            base = ((unsigned long long)bhi << 32) | blo;
            const bool fits = base + (unsigned long long)tail <= (unsigned long long)a.cap;
            if (fits) {
                for (int i = lane; i < tail; i += 64) {
                    a.out_q[base + i] = qi;
                    a.out_x[base + i] = il_id[i];
                    const float kk = il_d[i];
                    a.out_d[base + i] = l2 ? sqrtf(kk) : kk;
                }
            }
            if (a.ws == VJ_WS_HARD && lane == 0) {
                a.seg[qi] = (int64_t)base;
                a.segn[qi] = fits ? tail : 0;
            }
        }

        // ---- UpdateCache and publication to children
        if (a.ws != VJ_WS_SELF) {
            float bk = best_k;
            int bid = best_id, bs = 0;
            wave_argbest(bk, bid, bs, false);
            int32_t val = abort ? kAborted : (bid == 0x7fffffff ? -1 : bid);
            if (a.ws == VJ_WS_HARD) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            if (lane == 0)
                __hip_atomic_store(&a.pub[qi], ((unsigned long long)a.gen << 32) | (uint32_t)val,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }

        if (lane == 0) {
            int32_t *st = a.stats + (size_t)pos * 8;
            st[0] = abort ? 0 : tail;
            st[1] = ndist;
            st[2] = nexp;
            st[3] = hpops;
            st[4] = ood;
            st[5] = hyb ? 1 : 0;
            st[6] = nvis;
            st[7] = (SPILL ? 1 : 0) | (abort ? 4 : 0);
            if (abort) a.ovf[atomicAdd(a.ovf_count, 1)] = k;
        }
    }
}

template <typename T, int DP>
int launch_dp(const TraverseLaunch &a, bool spill, int max_blocks, int wpb, hipStream_t s) {
    const size_t lds = (size_t)a.lds_ints_per_wave * wpb * sizeof(int32_t);
    const void *fn = spill ? reinterpret_cast<const void *>(&k_traverse<T, DP, true>)
                           : reinterpret_cast<const void *>(&k_traverse<T, DP, false>);
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64 * wpb, lds) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    int blocks = per_cu * num_cus();
    if (blocks > max_blocks) blocks = max_blocks;
    if (spill)
        hipLaunchKernelGGL((k_traverse<T, DP, true>), dim3(blocks), dim3(64 * wpb), lds, s, a);
    else
        hipLaunchKernelGGL((k_traverse<T, DP, false>), dim3(blocks), dim3(64 * wpb), lds, s, a);
    return blocks * wpb;
}

template <typename T>
int launch_elem(const TraverseLaunch &a, bool spill, int max_blocks, int wpb, hipStream_t s) {
    switch (a.dp) {
    case 32: return launch_dp<T, 32>(a, spill, max_blocks, wpb, s);
    case 64: return launch_dp<T, 64>(a, spill, max_blocks, wpb, s);
    case 96: return launch_dp<T, 96>(a, spill, max_blocks, wpb, s);
    case 128: return launch_dp<T, 128>(a, spill, max_blocks, wpb, s);
    case 192: return launch_dp<T, 192>(a, spill, max_blocks, wpb, s);
    case 256: return launch_dp<T, 256>(a, spill, max_blocks, wpb, s);
    case 384: return launch_dp<T, 384>(a, spill, max_blocks, wpb, s);
    case 512: return launch_dp<T, 512>(a, spill, max_blocks, wpb, s);
    case 768: return launch_dp<T, 768>(a, spill, max_blocks, wpb, s);
    case 1024: return launch_dp<T, 1024>(a, spill, max_blocks, wpb, s);
    default: return 0;
    }
}

}  // namespace trav
}  // namespace vj
