// Exact epsilon-join on MFMA tiles (the nested-loop join of Section 2.2, run
// as a GEMM):  d^2(q, x) = |q|^2 + |x|^2 - 2 <q, x>  (L2)  or  1 - <q, x>  (IP)
// with <q, x> from bf16 MFMA tiles and fp32 accumulation.  Every pair whose
// tile value lies below eps plus a proven bound on the tile's error becomes a
// candidate; each candidate is re-decided from the fp32 inputs in fp64, so the
// result equals the exact decision dist < eps computed in fp64.
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "lds_ring.h"
#include "mfma_tile.h"
#include "tiles.h"

namespace vj {
namespace {

using mt::floatx4;

__device__ __forceinline__ uint16_t bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// One wave per row, grid-stride: bf16 hi (and lo) copies padded to Kp,
// squared norm (fp64 sum rounded to fp32), and flags: bit 0 set if a value
// is not an integer of magnitude <= 256; max |value| and max norm via one
// atomicMax per workgroup on the (non-negative) float bits (same-address
// atomics serialise, so not one per row).
__global__ void __launch_bounds__(256)
k_prep(const float *src, int64_t rows, int d, int Kp, uint16_t *hi, uint16_t *lo, float *norm2,
       unsigned *maxabs, unsigned *maxnorm, int *flags) {
    __shared__ float s_abs[4], s_norm[4];
    __shared__ int s_nonint[4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    float mabs = 0.f, mnorm = 0.f;
    bool nonint = false;
    for (int64_t r = (int64_t)blockIdx.x * 4 + w; r < rows; r += (int64_t)gridDim.x * 4) {
        double acc = 0.0;
        for (int k = lane; k < Kp; k += 64) {
            const float f = k < d ? src[r * d + k] : 0.f;
            const uint16_t h = bf16_rne(f);
            hi[r * Kp + k] = h;
            if (lo) lo[r * Kp + k] = bf16_rne(f - bf16_to_f(h));
            acc += (double)f * (double)f;
            mabs = fmaxf(mabs, fabsf(f));
            nonint |= !(rintf(f) == f && fabsf(f) <= 256.f);
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
        if (lane == 0) norm2[r] = (float)acc;
        mnorm = fmaxf(mnorm, (float)sqrt(acc));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mabs = fmaxf(mabs, __shfl_xor(mabs, off));
    const bool wn = __ballot(nonint) != 0;
    if (lane == 0) { s_abs[w] = mabs; s_norm[w] = mnorm; s_nonint[w] = wn; }
    __syncthreads();
    if (threadIdx.x == 0) {
        float a = 0.f, n = 0.f;
        int f = 0;
        for (int i = 0; i < 4; ++i) { a = fmaxf(a, s_abs[i]); n = fmaxf(n, s_norm[i]); f |= s_nonint[i]; }
        if (f) atomicOr(flags, 1);
        atomicMax(maxabs, __float_as_uint(a));
        atomicMax(maxnorm, __float_as_uint(n));
    }
}

// per-query-row threshold on the tile value, including its error bound
__global__ void k_thresholds(const float *nq2, int64_t nq, double eps, int metric, double e_dot,
                             double e_fin, float maxnorm_x, float *thr) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nq) return;
    const double qn = sqrt((double)nq2[i]), xn = (double)maxnorm_x;
    if (metric == VJ_L2) {
        const double m2 = 2.0 * e_dot * qn * xn + e_fin * (qn + xn) * (qn + xn);
        thr[i] = __double2float_ru(eps * eps + m2);            // candidate iff d~^2 < thr
    } else {
        const double m = e_dot * qn * xn + e_fin;
        thr[i] = __double2float_rd(1.0 - eps - m);              // candidate iff <q,x>~ > thr
    }
}

// 64 query rows x 128 data rows per workgroup; wave w takes data rows 32w..32w+31
template <int NSPLIT>
__global__ void __launch_bounds__(256)
k_range_tiles(const uint16_t *Qh, const uint16_t *Ql, int64_t nq, const uint16_t *Xh,
              const uint16_t *Xl, int64_t nx, int Kp, const float *nq2, const float *nx2,
              const float *thr, int metric, int32_t *cq, int32_t *cx, int64_t cap,
              unsigned long long *count) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t q0 = (int64_t)blockIdx.y * 64;
    const int64_t x0 = (int64_t)blockIdx.x * 128 + w * 32;
    floatx4 acc[4][2];
    mt::tile_64x32<NSPLIT>(Qh, Ql, q0, nq, Xh, Xl, x0, nx, Kp, lane, acc);
    uint32_t hits = 0;  // bit (rt*8 + ct*4 + i)
    // the tile's row and column terms, read once per lane (16 rows, 2
    // columns), indices in 32 bits (nq, nx < 2^31); the same comparisons
    const int nq32 = (int)nq, nx32 = (int)nx, qb = (int)q0, xb = (int)x0;
    float rq2[4][4], rthr[4][4], cx2[2];
    bool rok[4][4], cok[2];
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
        const int x = xb + mt::tile_brow(ct, lane);
        cok[ct] = x < nx32;
        cx2[ct] = cok[ct] ? nx2[x] : 0.f;
    }
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int q = qb + mt::tile_arow(rt, i, lane);
            rok[rt][i] = q < nq32;
            rq2[rt][i] = rok[rt][i] ? nq2[q] : 0.f;
            rthr[rt][i] = rok[rt][i] ? thr[q] : 0.f;
        }
    if (metric == VJ_L2) {
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
            for (int ct = 0; ct < 2; ++ct)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (rok[rt][i] && cok[ct] &&
                        rq2[rt][i] + cx2[ct] - 2.f * acc[rt][ct][i] < rthr[rt][i])
                        hits |= 1u << (rt * 8 + ct * 4 + i);
    } else {
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
            for (int ct = 0; ct < 2; ++ct)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (rok[rt][i] && cok[ct] && acc[rt][ct][i] > rthr[rt][i])
                        hits |= 1u << (rt * 8 + ct * 4 + i);
    }
    if (__ballot(hits != 0) == 0) return;
    int excl;
    const int total = mt::wave_scan(__popc(hits), lane, excl);
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(count, (unsigned long long)total);
    base = __shfl(base, 0);
    int o = 0;
    for (int b = 0; b < 32; ++b) {
        if (!(hits & (1u << b))) continue;
        const int rt = b >> 3, ct = (b >> 2) & 1, i = b & 3;
        const unsigned long long at = base + excl + o++;
        if (at < (unsigned long long)cap) {
            cq[at] = (int32_t)(q0 + mt::tile_arow(rt, i, lane));
            cx[at] = (int32_t)(x0 + mt::tile_brow(ct, lane));
        }
    }
}

// The same candidate test on register-row tiles (Kp <= 1,024): a workgroup of
// 4 waves holds 4 * RT * 16 query rows in registers and sweeps the data rows
// [cb, ce) of its split (blockIdx.y) 32 at a time through a ring of LDS
// stages filled by direct global-to-LDS loads (see lds_ring.h).  Per
// element one compare of the tile value with the query row's threshold, in
// the same arithmetic as k_range_tiles; a step with a passing element
// recomputes its hit bits and appends the candidates to the wave's own
// buffer of kRangeBuf entries in LDS, which goes out to the candidate
// arrays with one global atomic when the next append would overflow it and
// at the end.  (Same-address device atomics serialise across the chip: one
// per appending wave-step took more time than the tiles.)
constexpr int kRangeBuf = 64;

template <int NSPLIT, int KP, bool L2>
__global__ void __launch_bounds__(256, 2)
k_range_reg(const uint16_t *Qh, const uint16_t *Ql, int32_t nq, const uint16_t *Xh,
            const uint16_t *Xl, int32_t nx, const float *nq2, const float *nx2, const float *thr,
            int32_t cols_per_split, int32_t *cq, int32_t *cx, int64_t cap,
            unsigned long long *count) {
    using S = ring::Shape<NSPLIT, KP>;
    constexpr int RT = S::RT, CT = S::CT, KS = S::KS, BN = S::BN, CPR = S::CPR, SPR = S::SPR;
    constexpr int IPW = S::IPW, TERMS = S::TERMS, PART = S::PART, STAGE = S::STAGE, NB = S::NB;
    constexpr int LPT = S::LPT, KC = S::KC, NCH = S::NCH, KCS = S::KCS;
    __shared__ __attribute__((aligned(1024))) char sring[NB * STAGE];
    __shared__ int2 sbuf[4][kRangeBuf];
    static_assert(NB * STAGE + sizeof(sbuf) <= 80 * 1024, "two workgroups per CU");
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int r16 = lane & 15, kq = (lane >> 4) * 8, rq = (lane >> 4) * 4;
    const int32_t prow0 = (int32_t)blockIdx.x * S::ROWS + w * RT * 16;
    int2 *wbuf = sbuf[w];
    int nbuf = 0;  // entries in the wave's buffer (wave-uniform)
    // the buffer to the candidate arrays: one atomic, then lane-strided
    // copies (entries past cap are counted, not written)
    auto flush = [&]() {
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(count, (unsigned long long)nbuf);
        base = __shfl(base, 0);
        for (int e = lane; e < nbuf; e += 64) {
            const unsigned long long at = base + e;
            if (at < (unsigned long long)cap) {
                const int2 v = wbuf[e];
                cq[at] = v.x;
                cx[at] = v.y;
            }
        }
        __builtin_amdgcn_wave_barrier();
        nbuf = 0;
    };
    const int32_t cb = (int32_t)blockIdx.y * cols_per_split;
    const int32_t ce = min(nx, cb + cols_per_split);
    // the query rows' fragments and terms; rows past nq never pass
    mt::bf16x8 a[RT][KS], al[NSPLIT == 3 ? RT : 1][NSPLIT == 3 ? KS : 1];
    float rq2[RT][4], rthr[RT][4];
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            a[rt][ks] = mt::load8(Qh, prow0 + rt * 16 + r16, nq, KP, ks * 32 + kq);
            if (NSPLIT == 3) al[rt][ks] = mt::load8(Ql, prow0 + rt * 16 + r16, nq, KP, ks * 32 + kq);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int32_t q = prow0 + rt * 16 + rq + i;
            rq2[rt][i] = q < nq ? nq2[q] : 0.f;
            rthr[rt][i] = q < nq ? thr[q] : (L2 ? -INFINITY : INFINITY);
        }
    }
    // the rows' loads land here, once: the compiler does not see the ring's
    // loads (inline asm), so without this it waits for them all (vmcnt 0)
    // before every tile's first MFMA
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    // loads of the data tile at row c0 into stage st (rows past nx load row
    // nx - 1, masked in the test; pad slots load the tile's first chunk)
    const uint32_t ring0 = ring::lds_byte_addr(sring);
    uint32_t soff[IPW];
    int srow[IPW];
#pragma unroll
    for (int j = 0; j < IPW; ++j) {
        const int sl = (w * IPW + j) * 64 + lane;
        const int rr = sl / SPR, ch = sl - rr * SPR;
        const bool real = rr < BN && ch < CPR;
        srow[j] = real ? rr : 0;
        soff[j] = real ? (uint32_t)((rr * KP + ch * 8) * 2) : 0u;
    }
    const int ntile = ce > cb ? (ce - cb + BN - 1) / BN : 0;
    const int nstage = ntile * NCH;  // (tile, chunk) stages of this split, in order
    // stage sg (tile sg / NCH, dimensions (sg % NCH) * KC ..) into ring slot
    // st; an empty split (cb may lie past nx) loads from row 0
    auto issue = [&](int sg, int st) {
        const int32_t c0 = ntile > 0 ? cb + (sg / NCH) * BN : 0;
        const int kc0 = (sg % NCH) * KC;
        const uint32_t sbase = ring0 + (uint32_t)(st * STAGE);
        const char *th = reinterpret_cast<const char *>(Xh + (int64_t)c0 * KP + kc0);
        const char *tl = NSPLIT == 3 ? reinterpret_cast<const char *>(Xl + (int64_t)c0 * KP + kc0) : nullptr;
        const bool whole = c0 + BN <= nx;
#pragma unroll
        for (int j = 0; j < IPW; ++j) {
            uint32_t off = soff[j];
            if (!whole && c0 + srow[j] > nx - 1)
                off = (uint32_t)(((nx - 1 - c0) * KP) * 2) + (off - (uint32_t)(srow[j] * KP * 2));
            const uint32_t dst = sbase + (uint32_t)((w * IPW + j) * 1024);
            ring::lds_dma16(th, off, dst);
            if (NSPLIT == 3) ring::lds_dma16(tl, off, dst + PART);
        }
        const int nr = min(lane < BN ? lane : 0, nx - 1 - c0);
        ring::lds_dma4(nx2 + c0, (uint32_t)(nr * 4), sbase + TERMS * PART + w * 256);
        // the second slot is unused here; the load keeps LPT loads per stage
        ring::lds_dma4(nx2 + c0, (uint32_t)(nr * 4), sbase + TERMS * PART + 1024 + w * 256);
    };
    // prologue: stages 0 .. NB-2 in flight; a slot past the last stage
    // re-loads stage 0 into the last ring slot, which no stage reads before
    // it is re-issued
#pragma unroll
    for (int p = 0; p < NB - 1; ++p) issue(p < nstage ? p : 0, p < nstage ? p : NB - 1);
    floatx4 acc[RT][CT];
    for (int it = 0; it < ntile; ++it) {
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) {
        const int sidx = it * NCH + ch;
        const int st = sidx % NB;
        ring::wait_barrier<(NB - 2) * LPT>();
        {
            const int nxs = sidx + NB - 1;
            issue(nxs < nstage ? nxs : 0, nxs % NB);
        }
        const char *sp = sring + st * STAGE;
        if (ch == 0) {
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int ct = 0; ct < CT; ++ct) acc[rt][ct] = floatx4{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
        for (int kk = 0; kk < KCS; ++kk) {
            const int ks = ch * KCS + kk;
            mt::bf16x8 b[CT], bl[NSPLIT == 3 ? CT : 1];
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) {
                const int off = ((ct * 16 + r16) * SPR + kk * 4 + (lane >> 4)) * 16;
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
        if (ch < NCH - 1) continue;
        const int32_t c0 = cb + it * BN;
        const float *snc = reinterpret_cast<const float *>(sp + TERMS * PART + w * 256);
        // columns past the split's end (rows past nx load row nx - 1) occur
        // only in its last tile: +inf norms (L2) / -inf values (IP) there
        const bool whole = c0 + BN <= ce;
        float nc[CT];
        bool cok[CT];
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
            cok[ct] = c0 + ct * 16 + r16 < ce;
            const float v = snc[ct * 16 + r16];
            nc[ct] = cok[ct] ? v : INFINITY;
        }
        if (!L2 && !whole) {
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int ct = 0; ct < CT; ++ct)
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        acc[rt][ct][i] = cok[ct] ? acc[rt][ct][i] : -INFINITY;
        }
        // the tile values of k_range_tiles' test, in the same arithmetic,
        // computed once: d~^2 (L2) or <q, x>~ (IP)
        if (L2) {
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int ct = 0; ct < CT; ++ct)
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        acc[rt][ct][i] = rq2[rt][i] + nc[ct] - 2.f * acc[rt][ct][i];
        }
        auto pass = [&](int rt, int ct, int i) {
            return L2 ? acc[rt][ct][i] < rthr[rt][i] : acc[rt][ct][i] > rthr[rt][i];
        };
        // a row passes somewhere iff the extreme of its values does (min /
        // max are exact): one compare per row and lane
        bool any = false;
#pragma unroll
        for (int rt = 0; rt < RT; ++rt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                float e = acc[rt][0][i];
#pragma unroll
                for (int ct = 1; ct < CT; ++ct)
                    e = L2 ? fminf(e, acc[rt][ct][i]) : fmaxf(e, acc[rt][ct][i]);
                any |= L2 ? e < rthr[rt][i] : e > rthr[rt][i];
            }
        if (__ballot(any)) {
            uint32_t hits = 0;  // bit (rt * CT + ct) * 4 + i
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int ct = 0; ct < CT; ++ct)
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        if (pass(rt, ct, i)) hits |= 1u << ((rt * CT + ct) * 4 + i);
            int excl;
            const int total =
                __builtin_amdgcn_readfirstlane(mt::wave_scan(__popc(hits), lane, excl));
            if (nbuf + total > kRangeBuf) flush();
            // a lane walks only its set hit bits (usually one or two)
            if (total <= kRangeBuf) {
                int o = nbuf + excl;
                for (uint32_t hm = hits; hm; hm &= hm - 1) {
                    const int bt = __builtin_ctz(hm);
                    const int rt = bt / (CT * 4), ct = (bt / 4) % CT, i = bt & 3;
                    wbuf[o++] = make_int2(prow0 + rt * 16 + rq + i, c0 + ct * 16 + r16);
                }
                __builtin_amdgcn_wave_barrier();
                nbuf += total;
            } else {
                // more than the buffer holds: straight to the arrays
                unsigned long long base = 0;
                if (lane == 0) base = atomicAdd(count, (unsigned long long)total);
                base = __shfl(base, 0);
                int o = 0;
                for (uint32_t hm = hits; hm; hm &= hm - 1) {
                    const int bt = __builtin_ctz(hm);
                    const int rt = bt / (CT * 4), ct = (bt / 4) % CT, i = bt & 3;
                    const unsigned long long at = base + excl + o++;
                    if (at < (unsigned long long)cap) {
                        cq[at] = prow0 + rt * 16 + rq + i;
                        cx[at] = c0 + ct * 16 + r16;
                    }
                }
            }
        }
    }
    }
    if (nbuf > 0) flush();
    ring::wait_barrier<0>();
}

template <int NSPLIT, int KP>
bool launch_range_reg_t(const TileRows &tq, const TileRows &tx, int64_t nq, int64_t nx,
                        const float *thr, int metric, int32_t *cq, int32_t *cx, int64_t cap,
                        unsigned long long *count, hipStream_t s) {
    using S = ring::Shape<NSPLIT, KP>;
    if constexpr (!S::OK) {
        return false;
    } else {
        const int64_t nb = (nq + S::ROWS - 1) / S::ROWS;
        const int64_t T = (nx + S::BN - 1) / S::BN;
        int splits = 1;
        // no merge across splits here: split until the grid fills the chip
        // several times over, keeping at least 64 tiles per split
        while (nb * splits < 4096 && T / (splits * 2) >= 64 && splits < 256) splits *= 2;
        const int64_t cps = (T + splits - 1) / splits * S::BN;
        auto kern = metric == VJ_L2 ? k_range_reg<NSPLIT, KP, true> : k_range_reg<NSPLIT, KP, false>;
        hipLaunchKernelGGL(kern, dim3((unsigned)nb, (unsigned)splits), dim3(256), 0, s,
                           tq.hi.as<uint16_t>(), NSPLIT == 3 ? tq.lo.as<uint16_t>() : nullptr,
                           (int32_t)nq, tx.hi.as<uint16_t>(),
                           NSPLIT == 3 ? tx.lo.as<uint16_t>() : nullptr, (int32_t)nx,
                           tq.norm2.as<float>(), tx.norm2.as<float>(), thr, (int32_t)cps, cq, cx,
                           cap, count);
        return true;
    }
}

// the register-row tiles for the listed row widths (up to 1,024; wider rows
// staged in chunks), else false
bool launch_range_reg(int nsplit, int Kp, const TileRows &tq, const TileRows &tx, int64_t nq,
                      int64_t nx, const float *thr, int metric, int32_t *cq, int32_t *cx,
                      int64_t cap, unsigned long long *count, hipStream_t s) {
    if (nq <= 0 || nx <= 0 || nq >= (1ll << 31) || nx >= (1ll << 31)) return false;
#define VJ_RANGE_CASE(kp)                                                                         \
    case kp:                                                                                      \
        return nsplit == 3 ? launch_range_reg_t<3, kp>(tq, tx, nq, nx, thr, metric, cq, cx, cap, count, s) \
                           : launch_range_reg_t<1, kp>(tq, tx, nq, nx, thr, metric, cq, cx, cap, count, s);
    switch (Kp) {
        VJ_RANGE_CASE(32) VJ_RANGE_CASE(64) VJ_RANGE_CASE(96) VJ_RANGE_CASE(128)
        VJ_RANGE_CASE(192) VJ_RANGE_CASE(256) VJ_RANGE_CASE(384) VJ_RANGE_CASE(512)
        VJ_RANGE_CASE(768) VJ_RANGE_CASE(960) VJ_RANGE_CASE(1024)
    default: return false;
    }
#undef VJ_RANGE_CASE
}

// fp64 decision for every candidate: 8 lanes per candidate
__global__ void k_recheck(const float *Q, const float *X, int d, int metric, double eps,
                          const int32_t *cq, const int32_t *cx, int64_t n, int32_t *oq,
                          int32_t *ox, int ostride, float *od, int64_t ocap,
                          unsigned long long *count) {
    const int lane = threadIdx.x & 63;
    const int64_t c = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 3;
    const int p = lane & 7;
    const bool ok = c < n;
    const int32_t q = ok ? cq[c] : 0, x = ok ? cx[c] : 0;
    double acc = 0.0;
    if (ok) {
        for (int k = p; k < d; k += 8) {
            const double a = Q[(int64_t)q * d + k], b = X[(int64_t)x * d + k];
            if (metric == VJ_L2) { const double t = a - b; acc += t * t; }
            else acc += a * b;
        }
    }
#pragma unroll
    for (int off = 4; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    const double dist = metric == VJ_L2 ? sqrt(acc) : 1.0 - acc;
    const bool keep = ok && p == 0 && dist < eps;
    const uint64_t m = __ballot(keep);
    if (m == 0) return;
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(count, (unsigned long long)__popcll(m));
    base = __shfl(base, 0);
    if (keep) {
        const unsigned long long at = base + __popcll(m & ((1ull << lane) - 1ull));
        if (at < (unsigned long long)ocap) {
            oq[at * ostride] = q;
            ox[at * ostride] = x;
            if (od) od[at] = (float)dist;
        }
    }
}

__global__ void k_zero_u64(unsigned long long *p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0ull;
}

// ------------------------------------------------------ exact top-1 -----
// Order-preserving maps of floats / doubles to unsigned integers (for
// atomicMin on keys that may be negative).
__device__ __forceinline__ unsigned ord32(float f) {
    const unsigned u = __float_as_uint(f);
    return (u >> 31) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float unord32(unsigned u) {
    return __uint_as_float((u >> 31) ? (u & 0x7fffffffu) : ~u);
}
__device__ __forceinline__ unsigned long long ord64(double f) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(f);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}
__device__ __forceinline__ double unord64(unsigned long long u) {
    return __longlong_as_double((long long)((u >> 63) ? (u & 0x7fffffffffffffffull) : ~u));
}

// tile value of the key: L2 the squared distance (clamped at 0), IP 1 - <q, x>
__device__ __forceinline__ float tile_key(float q2, float x2, float dot, int metric) {
    return metric == VJ_L2 ? fmaxf(q2 + x2 - 2.f * dot, 0.f) : 1.f - dot;
}

// pass 1: the smallest tile key of every query row
template <int NSPLIT>
__global__ void __launch_bounds__(256)
k_top1_min(const uint16_t *Qh, const uint16_t *Ql, int64_t nq, const uint16_t *Xh,
           const uint16_t *Xl, int64_t nx, int Kp, const float *nq2, const float *nx2, int metric,
           unsigned *minkey) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t q0 = (int64_t)blockIdx.y * 64;
    const int64_t x0 = (int64_t)blockIdx.x * 128 + w * 32;
    floatx4 acc[4][2];
    mt::tile_64x32<NSPLIT>(Qh, Ql, q0, nq, Xh, Xl, x0, nx, Kp, lane, acc);
    float cx2[2];
    bool cok[2];
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
        const int64_t x = x0 + mt::tile_brow(ct, lane);
        cok[ct] = x < nx;
        cx2[ct] = cok[ct] ? nx2[x] : 0.f;
    }
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t q = q0 + mt::tile_arow(rt, i, lane);
            const float rq2 = q < nq ? nq2[q] : 0.f;
            unsigned k = 0xffffffffu;
#pragma unroll
            for (int ct = 0; ct < 2; ++ct)
                if (cok[ct]) k = min(k, ord32(tile_key(rq2, cx2[ct], acc[rt][ct][i], metric)));
            // the 16 lanes of one row group hold its 32 columns
#pragma unroll
            for (int off = 1; off < 16; off <<= 1) k = min(k, (unsigned)__shfl_xor((int)k, off));
            if ((lane & 15) == 0 && q < nq && k != 0xffffffffu) atomicMin(&minkey[q], k);
        }
}

// per row: the largest tile key a nearest row can have, min + 2 * bound
__global__ void k_top1_thr(const unsigned *minkey, const float *nq2, int64_t nq, int metric,
                           double e_dot, double e_fin, float maxnorm_x, float *thr) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nq) return;
    const double qn = sqrt((double)nq2[i]), xn = (double)maxnorm_x;
    // IP: plus the rounding of the key's fp32 subtraction 1 - dot~
    const double m = metric == VJ_L2
                         ? 2.0 * e_dot * qn * xn + e_fin * (qn + xn) * (qn + xn)
                         : e_dot * qn * xn + e_fin + 1.2e-7 * (1.0 + qn * xn * (1.0 + e_dot));
    thr[i] = __double2float_ru((double)unord32(minkey[i]) + 2.0 * m);
}

// pass 2: every (q, x) whose tile key is within the bound of the row's min
template <int NSPLIT>
__global__ void __launch_bounds__(256)
k_top1_cand(const uint16_t *Qh, const uint16_t *Ql, int64_t nq, const uint16_t *Xh,
            const uint16_t *Xl, int64_t nx, int Kp, const float *nq2, const float *nx2,
            const float *thr, int metric, int32_t *cq, int32_t *cx, int64_t cap,
            unsigned long long *count) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t q0 = (int64_t)blockIdx.y * 64;
    const int64_t x0 = (int64_t)blockIdx.x * 128 + w * 32;
    floatx4 acc[4][2];
    mt::tile_64x32<NSPLIT>(Qh, Ql, q0, nq, Xh, Xl, x0, nx, Kp, lane, acc);
    uint32_t hits = 0;
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t q = q0 + mt::tile_arow(rt, i, lane);
            if (q >= nq) continue;
            const float rq2 = nq2[q], t = thr[q];
#pragma unroll
            for (int ct = 0; ct < 2; ++ct) {
                const int64_t x = x0 + mt::tile_brow(ct, lane);
                if (x < nx && tile_key(rq2, nx2[x], acc[rt][ct][i], metric) <= t)
                    hits |= 1u << (rt * 8 + ct * 4 + i);
            }
        }
    if (__ballot(hits != 0) == 0) return;
    int excl;
    const int total = mt::wave_scan(__popc(hits), lane, excl);
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(count, (unsigned long long)total);
    base = __shfl(base, 0);
    int o = 0;
    for (int b = 0; b < 32; ++b) {
        if (!(hits & (1u << b))) continue;
        const int rt = b >> 3, ct = (b >> 2) & 1, i = b & 3;
        const unsigned long long at = base + excl + o++;
        if (at < (unsigned long long)cap) {
            cq[at] = (int32_t)(q0 + mt::tile_arow(rt, i, lane));
            cx[at] = (int32_t)(x0 + mt::tile_brow(ct, lane));
        }
    }
}

// fp64 key of every candidate (8 lanes each) and the row's exact minimum
__global__ void k_top1_recheck(const float *Q, const float *X, int d, int metric, const int32_t *cq,
                               const int32_t *cx, int64_t n, double *key,
                               unsigned long long *min64) {
    const int lane = threadIdx.x & 63;
    const int64_t c = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 3;
    const int p = lane & 7;
    const bool ok = c < n;
    const int32_t q = ok ? cq[c] : 0, x = ok ? cx[c] : 0;
    double acc = 0.0;
    if (ok)
        for (int k = p; k < d; k += 8) {
            const double a = Q[(int64_t)q * d + k], b = X[(int64_t)x * d + k];
            if (metric == VJ_L2) { const double t = a - b; acc += t * t; }
            else acc += a * b;
        }
#pragma unroll
    for (int off = 4; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (ok && p == 0) {
        const double kk = metric == VJ_L2 ? acc : 1.0 - acc;
        key[c] = kk;
        atomicMin(&min64[q], ord64(kk));
    }
}

// the smallest index among the candidates at the exact minimum
__global__ void k_top1_tie(const int32_t *cq, const int32_t *cx, int64_t n, const double *key,
                           const unsigned long long *min64, int32_t *wid) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const int32_t q = cq[c];
    if (ord64(key[c]) == min64[q]) atomicMin(&wid[q], cx[c]);
}

__global__ void k_top1_out(const unsigned long long *min64, const int32_t *wid, int64_t nq,
                           int metric, int32_t *w, double *dist) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nq) return;
    const double kk = unord64(min64[i]);
    w[i] = wid[i];
    dist[i] = metric == VJ_L2 ? sqrt(kk) : kk;
}

__global__ void k_fill_u32(unsigned *p, int64_t n, unsigned v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void k_fill_u64(unsigned long long *p, int64_t n, unsigned long long v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

inline unsigned g1(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

void prepare_rows(const float *src, int64_t rows, int d, int Kp, bool split, TileRows &t,
                  hipStream_t s, Arena *arena) {
    Arena fresh;
    Arena &A = arena ? *arena : fresh;
    t.rows = rows;
    t.Kp = Kp;
    t.hi = A.take((size_t)std::max<int64_t>(rows, 1) * Kp * sizeof(uint16_t));
    if (split) t.lo = A.take((size_t)std::max<int64_t>(rows, 1) * Kp * sizeof(uint16_t));
    else t.lo.release();
    t.norm2 = A.take((size_t)std::max<int64_t>(rows, 1) * sizeof(float));
    DevBuf stats = A.take(16);
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, stats.as<unsigned long long>(), 2);
    unsigned *u = stats.as<unsigned>();
    if (rows > 0)
        hipLaunchKernelGGL(k_prep, dim3(std::min<unsigned>(g1(rows, 4), 4096)), dim3(256), 0, s, src, rows, d, Kp,
                           t.hi.as<uint16_t>(), split ? t.lo.as<uint16_t>() : nullptr,
                           t.norm2.as<float>(), u, u + 1, reinterpret_cast<int *>(u + 2));
    VJ_HIP(hipGetLastError());
    unsigned h[4] = {0, 0, 0, 0};
    VJ_HIP(hipMemcpyAsync(h, stats.p, 16, hipMemcpyDeviceToHost, s));
    VJ_HIP(hipStreamSynchronize(s));
    std::memcpy(&t.maxabs, &h[0], 4);
    std::memcpy(&t.maxnorm, &h[1], 4);
    t.small_int = (h[2] & 1) == 0;
}

void tile_error_bounds(const TileRows &a, const TileRows &b, int nsplit, double &e_dot,
                       double &e_fin) {
    const int Kp = a.Kp;
    const double u32 = std::ldexp(1.0, -24);
    const double amax = std::max(a.maxabs, b.maxabs);
    // integer inputs with |v| <= 256 are exact in bf16, and every partial sum
    // of products, every norm and |q|^2 + |x|^2 stay integers below 2^24: the
    // tile value is then the exact squared distance
    if (a.small_int && b.small_int && 2.0 * Kp * amax * amax < 16777216.0) {
        e_dot = 0.0;
        e_fin = 0.0;
        return;
    }
    const double u = std::ldexp(1.0, -8);                   // bf16 unit roundoff
    const double e_in = nsplit == 3 ? 4.0 * u * u : 2.0 * u + u * u;
    const double n = (double)nsplit * Kp;
    const double gam = 1.01 * n * u32;                       // fp32 accumulation
    e_dot = e_in * (1.0 + gam) + gam;                        // |dot~ - dot| <= e_dot |q||x|
    e_fin = 5.0 * u32;                                       // norms and the final adds
}

namespace {

// Where the kept pairs go: q / x with a stride (1: two arrays, 2: one
// interleaved array), dist (may be null), room for cap pairs.
struct PairSink {
    int32_t *q = nullptr, *x = nullptr;
    int stride = 1;
    float *dist = nullptr;
    int64_t cap = 0;
};

// The brute-force join's steps with its temporaries from `A`.  With a fixed
// region the candidate list gets what is left of it (one attempt); with
// fresh allocations it grows until the candidates fit.  `sink(ncand)` gives
// the output once the candidate count is known.  Returns the pair count
// (not capped) and the candidate count in *ncand_out.
template <typename SinkFn>
int64_t bruteforce_core(const float *Q, int64_t nq, const float *X, int64_t nx, int d, float eps,
                        vj_metric metric, vj_precision prec, hipStream_t s, Arena &A,
                        SinkFn sink, int64_t *ncand_out) {
    *ncand_out = 0;
    if (nq == 0 || (metric == VJ_L2 && eps <= 0.0f)) { sink(0); return 0; }
    const int Kp = ((d + 31) / 32) * 32;
    const int nsplit = prec == VJ_PREC_FP32 ? 3 : 1;
    const dim3 grid(g1(nx, 128), g1(nq, 64));
    VJ_CHECK(grid.y <= 65535u, VJ_ERR_UNSUPPORTED, "too many query rows for one call");
    TileRows tq, tx;
    prepare_rows(Q, nq, d, Kp, nsplit == 3, tq, s, &A);
    prepare_rows(X, nx, d, Kp, nsplit == 3, tx, s, &A);
    double e_dot, e_fin;
    tile_error_bounds(tq, tx, nsplit, e_dot, e_fin);
    DevBuf thr = A.take((size_t)nq * sizeof(float));
    hipLaunchKernelGGL(k_thresholds, dim3(g1(nq, 256)), dim3(256), 0, s, tq.norm2.as<float>(), nq,
                       (double)eps, (int)metric, e_dot, e_fin, tx.maxnorm, thr.as<float>());
    DevBuf ctr = A.take(16);
    const bool fixed = A.base != nullptr;
    // fixed region: two candidate arrays in what is left (less alignment)
    const int64_t room = (int64_t)A.left();
    int64_t cap = fixed ? (room > 2048 ? (room / 2 - 512) / (int64_t)sizeof(int32_t) : 0)
                        : std::max<int64_t>(1 << 20, nq * 64);
    VJ_CHECK(cap >= 1024, VJ_ERR_UNSUPPORTED, "no room for candidates in the fixed scratch region");
    DevBuf cq, cx;
    unsigned long long ncand = 0;
    for (int attempt = 0; attempt < 3; ++attempt) {
        cq = A.take((size_t)cap * sizeof(int32_t));
        cx = A.take((size_t)cap * sizeof(int32_t));
        hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, ctr.as<unsigned long long>(), 2);
        if (launch_range_reg(nsplit, Kp, tq, tx, nq, nx, thr.as<float>(), (int)metric,
                             cq.as<int32_t>(), cx.as<int32_t>(), cap, ctr.as<unsigned long long>(), s))
            ;
        else if (nsplit == 3)
            hipLaunchKernelGGL(k_range_tiles<3>, grid, dim3(256), 0, s, tq.hi.as<uint16_t>(),
                               tq.lo.as<uint16_t>(), nq, tx.hi.as<uint16_t>(), tx.lo.as<uint16_t>(),
                               nx, Kp, tq.norm2.as<float>(), tx.norm2.as<float>(), thr.as<float>(),
                               (int)metric, cq.as<int32_t>(), cx.as<int32_t>(), cap,
                               ctr.as<unsigned long long>());
        else
            hipLaunchKernelGGL(k_range_tiles<1>, grid, dim3(256), 0, s, tq.hi.as<uint16_t>(),
                               nullptr, nq, tx.hi.as<uint16_t>(), nullptr, nx, Kp,
                               tq.norm2.as<float>(), tx.norm2.as<float>(), thr.as<float>(),
                               (int)metric, cq.as<int32_t>(), cx.as<int32_t>(), cap,
                               ctr.as<unsigned long long>());
        VJ_HIP(hipGetLastError());
        VJ_HIP(hipMemcpyAsync(&ncand, ctr.p, 8, hipMemcpyDeviceToHost, s));
        VJ_HIP(hipStreamSynchronize(s));
        if ((int64_t)ncand <= cap) break;
        VJ_CHECK(!fixed, VJ_ERR_UNSUPPORTED,
                 "the candidate pairs exceed the fixed scratch region (" + std::to_string(ncand) +
                     " candidates, room for " + std::to_string(cap) + ")");
        cap = (int64_t)ncand + (int64_t)ncand / 8 + 1024;
        VJ_CHECK(attempt < 2, VJ_ERR_INTERNAL, "candidate capacity did not converge");
    }
    *ncand_out = (int64_t)ncand;
    const PairSink o = sink((int64_t)ncand);
    if (ncand > 0)
        hipLaunchKernelGGL(k_recheck, dim3(g1((int64_t)ncand * 8, 256)), dim3(256), 0, s, Q, X, d,
                           (int)metric, (double)eps, cq.as<int32_t>(), cx.as<int32_t>(),
                           (int64_t)ncand, o.q, o.x, o.stride, o.dist, o.cap,
                           ctr.as<unsigned long long>() + 1);
    VJ_HIP(hipGetLastError());
    unsigned long long kept = 0;
    VJ_HIP(hipMemcpyAsync(&kept, ctr.as<char>() + 8, 8, hipMemcpyDeviceToHost, s));
    VJ_HIP(hipStreamSynchronize(s));
    return (int64_t)kept;
}

}  // namespace

// The fixed scratch region of the allocation-free entry point: one copy per
// device, reached through its address on that device (looked up once per
// device with the device current; host code never uses the symbol itself
// as an address).  Calls that overlap on one device race on it.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

char *noalloc_scratch() {
    static std::mutex mu;
    static void *addr[64] = {};
    int dev = 0;
    VJ_HIP(hipGetDevice(&dev));
    VJ_CHECK(dev >= 0 && dev < 64, VJ_ERR_UNSUPPORTED, "device index >= 64");
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        VJ_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        VJ_CHECK(p != nullptr, VJ_ERR_HIP, "no device address for the scratch region");
        addr[dev] = p;
    }
    return static_cast<char *>(addr[dev]);
}

}  // namespace

void bruteforce_join(const float *Q, int64_t nq, const float *X, int64_t nx, int d, float eps,
                     vj_metric metric, vj_precision prec, hipStream_t s, Pairs &out) {
    out.n_queries = 0;
    out.count = 0;
    Arena A;  // fresh allocations
    auto sink = [&](int64_t ncand) {
        const size_t n = (size_t)std::max<int64_t>(ncand, 1);
        out.q.alloc(n * sizeof(int32_t));
        out.x.alloc(n * sizeof(int32_t));
        out.dist.alloc(n * sizeof(float));
        return PairSink{out.q.as<int32_t>(), out.x.as<int32_t>(), 1, out.dist.as<float>(), ncand};
    };
    int64_t ncand = 0;
    out.count = bruteforce_core(Q, nq, X, nx, d, eps, metric, prec, s, A, sink, &ncand);
    out.n_candidates = ncand;
}

void exact_top1(const float *Q, int64_t nq, const float *X, int64_t nx, int d, vj_metric metric,
                int32_t *w, double *dist, hipStream_t s) {
    if (nq == 0) return;
    const int Kp = ((d + 31) / 32) * 32;
    TileRows tq, tx;
    prepare_rows(Q, nq, d, Kp, true, tq, s);
    prepare_rows(X, nx, d, Kp, true, tx, s);
    double e_dot, e_fin;
    tile_error_bounds(tq, tx, 3, e_dot, e_fin);
    const int nsplit = e_dot == 0.0 && e_fin == 0.0 ? 1 : 3;
    if (nsplit == 1) tile_error_bounds(tq, tx, 1, e_dot, e_fin);
    const dim3 grid(g1(nx, 128), g1(nq, 64));
    VJ_CHECK(grid.y <= 65535u, VJ_ERR_UNSUPPORTED, "too many query rows for one call");
    DevBuf minkey((size_t)nq * sizeof(unsigned)), thr((size_t)nq * sizeof(float));
    hipLaunchKernelGGL(k_fill_u32, dim3(g1(nq, 256)), dim3(256), 0, s, minkey.as<unsigned>(), nq,
                       0xffffffffu);
    const uint16_t *ql = nsplit == 3 ? tq.lo.as<uint16_t>() : nullptr;
    const uint16_t *xl = nsplit == 3 ? tx.lo.as<uint16_t>() : nullptr;
    if (nsplit == 3)
        hipLaunchKernelGGL(k_top1_min<3>, grid, dim3(256), 0, s, tq.hi.as<uint16_t>(), ql, nq,
                           tx.hi.as<uint16_t>(), xl, nx, Kp, tq.norm2.as<float>(),
                           tx.norm2.as<float>(), (int)metric, minkey.as<unsigned>());
    else
        hipLaunchKernelGGL(k_top1_min<1>, grid, dim3(256), 0, s, tq.hi.as<uint16_t>(), ql, nq,
                           tx.hi.as<uint16_t>(), xl, nx, Kp, tq.norm2.as<float>(),
                           tx.norm2.as<float>(), (int)metric, minkey.as<unsigned>());
    hipLaunchKernelGGL(k_top1_thr, dim3(g1(nq, 256)), dim3(256), 0, s, minkey.as<unsigned>(),
                       tq.norm2.as<float>(), nq, (int)metric, e_dot, e_fin, tx.maxnorm,
                       thr.as<float>());
    VJ_HIP(hipGetLastError());
    DevBuf ctr(16);
    int64_t cap = std::max<int64_t>(1 << 20, nq * 8);
    DevBuf cq, cx;
    unsigned long long ncand = 0;
    for (int attempt = 0; attempt < 3; ++attempt) {
        cq.alloc((size_t)cap * sizeof(int32_t));
        cx.alloc((size_t)cap * sizeof(int32_t));
        hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, ctr.as<unsigned long long>(), 2);
        if (nsplit == 3)
            hipLaunchKernelGGL(k_top1_cand<3>, grid, dim3(256), 0, s, tq.hi.as<uint16_t>(), ql, nq,
                               tx.hi.as<uint16_t>(), xl, nx, Kp, tq.norm2.as<float>(),
                               tx.norm2.as<float>(), thr.as<float>(), (int)metric,
                               cq.as<int32_t>(), cx.as<int32_t>(), cap,
                               ctr.as<unsigned long long>());
        else
            hipLaunchKernelGGL(k_top1_cand<1>, grid, dim3(256), 0, s, tq.hi.as<uint16_t>(), ql, nq,
                               tx.hi.as<uint16_t>(), xl, nx, Kp, tq.norm2.as<float>(),
                               tx.norm2.as<float>(), thr.as<float>(), (int)metric,
                               cq.as<int32_t>(), cx.as<int32_t>(), cap,
                               ctr.as<unsigned long long>());
        VJ_HIP(hipGetLastError());
        VJ_HIP(hipMemcpyAsync(&ncand, ctr.p, 8, hipMemcpyDeviceToHost, s));
        VJ_HIP(hipStreamSynchronize(s));
        if ((int64_t)ncand <= cap) break;
        cap = (int64_t)ncand + (int64_t)ncand / 8 + 1024;
        VJ_CHECK(attempt < 2, VJ_ERR_INTERNAL, "candidate capacity did not converge");
    }
    // every row has at least its tile minimum as a candidate
    DevBuf key((size_t)std::max<unsigned long long>(ncand, 1) * sizeof(double));
    DevBuf min64((size_t)nq * sizeof(unsigned long long)), wid((size_t)nq * sizeof(int32_t));
    hipLaunchKernelGGL(k_fill_u64, dim3(g1(nq, 256)), dim3(256), 0, s,
                       min64.as<unsigned long long>(), nq, ~0ull);
    hipLaunchKernelGGL(k_fill_u32, dim3(g1(nq, 256)), dim3(256), 0, s, wid.as<unsigned>(), nq,
                       0x7fffffffu);
    if (ncand > 0) {
        hipLaunchKernelGGL(k_top1_recheck, dim3(g1((int64_t)ncand * 8, 256)), dim3(256), 0, s, Q, X,
                           d, (int)metric, cq.as<int32_t>(), cx.as<int32_t>(), (int64_t)ncand,
                           key.as<double>(), min64.as<unsigned long long>());
        hipLaunchKernelGGL(k_top1_tie, dim3(g1((int64_t)ncand, 256)), dim3(256), 0, s,
                           cq.as<int32_t>(), cx.as<int32_t>(), (int64_t)ncand, key.as<double>(),
                           min64.as<unsigned long long>(), wid.as<int32_t>());
    }
    hipLaunchKernelGGL(k_top1_out, dim3(g1(nq, 256)), dim3(256), 0, s,
                       min64.as<unsigned long long>(), wid.as<int32_t>(), nq, (int)metric, w, dist);
    VJ_HIP(hipGetLastError());
    VJ_HIP(hipStreamSynchronize(s));
}

int64_t bruteforce_join_noalloc(const float *Q, int64_t nq, const float *X, int64_t nx, int d,
                                float eps, vj_metric metric, vj_precision prec, int32_t *qx,
                                float *dist, int64_t cap, hipStream_t s) {
    Arena A;
    A.base = noalloc_scratch();
    A.cap = kNoAllocScratchBytes;
    auto sink = [&](int64_t) { return PairSink{qx, qx + 1, 2, dist, cap}; };
    int64_t ncand = 0;
    return bruteforce_core(Q, nq, X, nx, d, eps, metric, prec, s, A, sink, &ncand);
}

}  // namespace vj
