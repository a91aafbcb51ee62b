// Dot-product tiles on gfx950 matrix cores: v_mfma_f32_16x16x32_bf16.
//
// A wave computes a 64 x 32 block of <a_i, b_j> for 64 rows of A and 32 rows
// of B (both row-major bf16, rows padded with zeros to Kp, a multiple of 32),
// accumulating in fp32.  With NSPLIT = 3 each fp32 value is carried as
// hi + lo bf16 terms and the product as hi*hi + hi*lo + lo*hi (the lo*lo term
// is dropped), which brings the input rounding error from ~2^-8 to ~2^-16.
//
// Lane layout of one 16x16x32 step: lane l supplies row (l % 16) of its
// 16-row A slice and of its 16-row B slice, each with the 8 consecutive k of
// group (l / 16); lane l receives D[4 (l / 16) + i][l % 16], i = 0..3.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vj {
namespace mt {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bf16x8 load8(const uint16_t *base, int64_t row, int64_t nrows, int Kp,
                                        int k) {
    if (row < nrows) return *reinterpret_cast<const bf16x8 *>(base + row * Kp + k);
    bf16x8 z;
#pragma unroll
    for (int i = 0; i < 8; ++i) z[i] = (__bf16)0.0f;
    return z;
}

template <int NSPLIT>
__device__ __forceinline__ void tile_64x32(const uint16_t *Ah, const uint16_t *Al, int64_t a0,
                                           int64_t na, const uint16_t *Bh, const uint16_t *Bl,
                                           int64_t b0, int64_t nb, int Kp, int lane,
                                           floatx4 acc[4][2]) {
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) acc[rt][ct] = floatx4{0.f, 0.f, 0.f, 0.f};
    const int r16 = lane & 15, kq = (lane >> 4) * 8;
    for (int k0 = 0; k0 < Kp; k0 += 32) {
        bf16x8 a[4], b[2];
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) a[rt] = load8(Ah, a0 + rt * 16 + r16, na, Kp, k0 + kq);
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) b[ct] = load8(Bh, b0 + ct * 16 + r16, nb, Kp, k0 + kq);
#pragma unroll
        for (int rt = 0; rt < 4; ++rt)
#pragma unroll
            for (int ct = 0; ct < 2; ++ct)
                acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[rt], b[ct], acc[rt][ct], 0, 0, 0);
        if (NSPLIT == 3) {
            bf16x8 al[4], bl[2];
#pragma unroll
            for (int rt = 0; rt < 4; ++rt) al[rt] = load8(Al, a0 + rt * 16 + r16, na, Kp, k0 + kq);
#pragma unroll
            for (int ct = 0; ct < 2; ++ct) bl[ct] = load8(Bl, b0 + ct * 16 + r16, nb, Kp, k0 + kq);
#pragma unroll
            for (int rt = 0; rt < 4; ++rt)
#pragma unroll
                for (int ct = 0; ct < 2; ++ct) {
                    acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[rt], bl[ct], acc[rt][ct], 0, 0, 0);
                    acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[rt], b[ct], acc[rt][ct], 0, 0, 0);
                }
        }
    }
}

// A wave's 16 x 128 block: 16 rows of A against 8 slices of 16 rows of B.
template <int NSPLIT>
__device__ __forceinline__ void tile_16x128(const uint16_t *Ah, const uint16_t *Al, int64_t a0,
                                            int64_t na, const uint16_t *Bh, const uint16_t *Bl,
                                            int64_t b0, int64_t nb, int Kp, int lane,
                                            floatx4 acc[8]) {
#pragma unroll
    for (int ct = 0; ct < 8; ++ct) acc[ct] = floatx4{0.f, 0.f, 0.f, 0.f};
    const int r16 = lane & 15, kq = (lane >> 4) * 8;
    for (int k0 = 0; k0 < Kp; k0 += 32) {
        const bf16x8 a = load8(Ah, a0 + r16, na, Kp, k0 + kq);
        bf16x8 b[8];
#pragma unroll
        for (int ct = 0; ct < 8; ++ct) b[ct] = load8(Bh, b0 + ct * 16 + r16, nb, Kp, k0 + kq);
#pragma unroll
        for (int ct = 0; ct < 8; ++ct)
            acc[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[ct], acc[ct], 0, 0, 0);
        if (NSPLIT == 3) {
            const bf16x8 al = load8(Al, a0 + r16, na, Kp, k0 + kq);
#pragma unroll
            for (int ct = 0; ct < 8; ++ct) {
                const bf16x8 bl = load8(Bl, b0 + ct * 16 + r16, nb, Kp, k0 + kq);
                acc[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bl, acc[ct], 0, 0, 0);
                acc[ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, b[ct], acc[ct], 0, 0, 0);
            }
        }
    }
}

// row of A / row of B of accumulator element (rt, ct, i) for this lane
__device__ __forceinline__ int tile_arow(int rt, int i, int lane) { return rt * 16 + (lane >> 4) * 4 + i; }
__device__ __forceinline__ int tile_brow(int ct, int lane) { return ct * 16 + (lane & 15); }

// (key, id) order: smaller key first, then smaller id
__device__ __forceinline__ bool kless(float ka, int ia, float kb, int ib) {
    return ka < kb || (ka == kb && ia < ib);
}

// Bitonic sort, ascending by (key, id), of 64*E elements held E per lane
// (element e = j*64 + lane lives in register j of that lane).
template <int E>
__device__ __forceinline__ void wave_sort(float *key, int *id, int lane) {
#pragma unroll
    for (int size = 2; size <= 64 * E; size <<= 1) {
#pragma unroll
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            if (stride >= 64) {
                const int s = stride >> 6;
#pragma unroll
                for (int j = 0; j < E; ++j) {
                    if (j & s) continue;
                    const int j2 = j | s;
                    const bool asc = (((j << 6) | lane) & size) == 0;
                    const bool sw = asc ? kless(key[j2], id[j2], key[j], id[j])
                                        : kless(key[j], id[j], key[j2], id[j2]);
                    if (sw) {
                        const float tk = key[j]; key[j] = key[j2]; key[j2] = tk;
                        const int ti = id[j]; id[j] = id[j2]; id[j2] = ti;
                    }
                }
            } else {
#pragma unroll
                for (int j = 0; j < E; ++j) {
                    const float pk = __shfl_xor(key[j], stride);
                    const int pi = __shfl_xor(id[j], stride);
                    const bool lower = (lane & stride) == 0;
                    const bool asc = (((j << 6) | lane) & size) == 0;
                    const bool want_min = lower == asc;
                    const bool take = want_min ? kless(pk, pi, key[j], id[j]) : kless(key[j], id[j], pk, pi);
                    if (take) { key[j] = pk; id[j] = pi; }
                }
            }
        }
    }
}

// exclusive prefix sum of per-lane counts over the wave; returns the total
__device__ __forceinline__ int wave_scan(int c, int lane, int &excl) {
    int incl = c;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int t = __shfl_up(incl, off);
        if (lane >= off) incl += t;
    }
    excl = incl - c;
    return __shfl(incl, 63);
}

}  // namespace mt
}  // namespace vj
