// Small device helpers of the index and the result: padded copies, exact u8
// and bf16 copies, edge lengths, id bookkeeping and the pair export.
#include <cstring>
#include <mutex>
#include <vector>

#include <rocprim/rocprim.hpp>

#include "vj_internal.h"
#include "util.h"

namespace vj {

namespace {

__global__ void k_pad_rows(const float *src, int64_t rows, int d, float *dst, int dp) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = rows * (int64_t)dp;
    if (i >= total) return;
    const int64_t r = i / dp;
    const int c = (int)(i - r * dp);
    dst[i] = c < d ? src[r * d + c] : 0.0f;
}

// bf16 by round-to-nearest-even of the fp32 bits
__device__ __forceinline__ uint16_t to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// u8 and bf16 copies of n values, grid-stride.  flag bit 0: a value is not
// an integer in [0, 255]; bit 1: a value is not exact in bf16.  One atomic
// per workgroup (same-address atomics serialise).
__global__ void __launch_bounds__(256)
k_quantize(const float *vec, int64_t n, uint8_t *u8, uint16_t *bf, int32_t *flag) {
    __shared__ int s_bits[4];
    bool bad_u8 = false, bad_bf = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float f = vec[i];
        if (u8) {
            const float r = rintf(f);
            const bool ok = r == f && f >= 0.0f && f <= 255.0f;
            bad_u8 |= !ok;
            u8[i] = ok ? (uint8_t)r : 0;
        }
        if (bf) {
            const uint16_t h = to_bf16(f);
            bf[i] = h;
            bad_bf |= __uint_as_float((uint32_t)h << 16) != f;
        }
    }
    const int bits = (__ballot(bad_u8) ? 1 : 0) | (__ballot(bad_bf) ? 2 : 0);
    if ((threadIdx.x & 63) == 0) s_bits[threadIdx.x >> 6] = bits;
    __syncthreads();
    if (threadIdx.x == 0 && flag) {
        const int b = s_bits[0] | s_bits[1] | s_bits[2] | s_bits[3];
        if (b) atomicOr(flag, b);
    }
}

// one 64-thread block per node (node rows[block] when rows is given); thread
// j handles edge j (R <= 64)
__global__ void k_edge_lengths(const float *vec, int dp, const int32_t *adj, int64_t N, int R,
                               float *elen, const int32_t *rows) {
    const int64_t u = rows ? (int64_t)rows[blockIdx.x] : (int64_t)blockIdx.x;
    const int j = threadIdx.x;
    if (u >= N || j >= R) return;
    const int32_t v = adj[u * R + j];
    if (v < 0 || v >= N) { elen[u * R + j] = INFINITY; return; }
    const float4 *a = reinterpret_cast<const float4 *>(vec + u * dp);
    const float4 *b = reinterpret_cast<const float4 *>(vec + (int64_t)v * dp);
    float acc = 0.f;
    for (int c = 0; c < dp / 4; ++c) {
        const float4 x = a[c], y = b[c];
        float t;
        t = x.x - y.x; acc = fmaf(t, t, acc);
        t = x.y - y.y; acc = fmaf(t, t, acc);
        t = x.z - y.z; acc = fmaf(t, t, acc);
        t = x.w - y.w; acc = fmaf(t, t, acc);
    }
    elen[u * R + j] = sqrtf(acc);
}

// L2 distance of rows [first, first+n) to row `node`
__global__ void k_dist_to_node(const float *vec, int dp, int64_t first, int64_t n, int32_t node,
                               float *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float4 *a = reinterpret_cast<const float4 *>(vec + (first + i) * dp);
    const float4 *b = reinterpret_cast<const float4 *>(vec + (int64_t)node * dp);
    float acc = 0.f;
    for (int c = 0; c < dp / 4; ++c) {
        const float4 x = a[c], y = b[c];
        float t;
        t = x.x - y.x; acc = fmaf(t, t, acc);
        t = x.y - y.y; acc = fmaf(t, t, acc);
        t = x.z - y.z; acc = fmaf(t, t, acc);
        t = x.w - y.w; acc = fmaf(t, t, acc);
    }
    out[i] = sqrtf(acc);
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// OCP fp8 e4m3: 1 sign, 4 exponent (bias 7), 3 mantissa bits; largest
// finite 448, subnormal step 2^-9, code 0x7f (and 0xff) NaN, never produced.
__device__ __forceinline__ uint32_t f8_encode(float v) {
    const uint32_t sign = v < 0.f ? 0x80u : 0u;
    const float a = fabsf(v);
    uint32_t code;
    if (!(a < 448.f)) {
        code = 0x7eu;  // saturate (also NaN input: never produced by finite rows)
    } else if (a < 0.015625f) {  // below 2^-6: subnormal, step 2^-9
        code = (uint32_t)rintf(a * 512.f);  // 0..8; 8 is the smallest normal
    } else {
        int e;
        const float f = frexpf(a, &e);  // a = f 2^e, f in [0.5, 1)
        int E = e - 1;
        uint32_t m = (uint32_t)rintf((2.f * f - 1.f) * 8.f);
        if (m == 8u) { m = 0u; E += 1; }
        const int field = E + 7;
        code = (field > 15 || (field == 15 && m == 7u)) ? 0x7eu : ((uint32_t)field << 3) | m;
    }
    return sign | code;
}

// one wave per row: scale, codes and the fp64 bound of the rounding error
__global__ void k_quantize_f8(const float *vec, int64_t rows, int dp, uint8_t *codes, float2 *meta) {
    const int lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (r >= rows) return;
    const float *x = vec + r * dp;
    float amax = 0.f;
    for (int k = lane; k < dp; k += 64) amax = fmaxf(amax, fabsf(x[k]));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) amax = fmaxf(amax, __shfl_xor(amax, off));
    // smallest power of two s with amax / s <= 448
    float sc = 1.f;
    if (amax > 0.f) {
        int e;
        frexpf(amax / 448.f, &e);  // amax / 448 < 2^e
        sc = ldexpf(1.f, e);
        if (amax / ldexpf(1.f, e - 1) <= 448.f) sc = ldexpf(1.f, e - 1);
    }
    const float inv = 1.f / sc;  // exact: a power of two
    double err = 0.0;
    for (int k = lane; k < dp; k += 64) {
        const uint32_t c = f8_encode(x[k] * inv);
        codes[r * dp + k] = (uint8_t)c;
        const double t = (double)x[k] - (double)sc * (double)f8_value(c);
        err += t * t;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) err += __shfl_xor(err, off);
    if (lane == 0) meta[r] = make_float2(sc, __double2float_ru(sqrt(err) * (1.0 + 1e-12)));
}

// NN-Map OOD bit, one wave per query (fp64 sums of the fp32 rows): d1 =
// |q - w|, d2 = mean |w - z| over w's data neighbours z; OOD iff d1 / d2 >
// ratio (no such z: not OOD)
__global__ void k_nn_ood(const float *vec, int dp, int64_t nx, int64_t nq, const int32_t *adj,
                         int R, const int32_t *w, double ratio, uint8_t *ood) {
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (i >= nq) return;
    const int32_t y = w[i];
    auto l2 = [&](int64_t a, int64_t b) {
        double acc = 0.0;
        for (int k = lane; k < dp; k += 64) {
            const double t = (double)vec[a * dp + k] - (double)vec[b * dp + k];
            acc += t * t;
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
        return sqrt(acc);
    };
    if (y < 0 || y >= nx) {
        if (lane == 0) ood[i] = 0;
        return;
    }
    const double d1 = l2(nx + i, y);
    double s2 = 0.0;
    int c2 = 0;
    for (int k = 0; k < R; ++k) {
        const int32_t z = adj[(int64_t)y * R + k];
        if (z < 0 || z >= nx) continue;
        s2 += l2(y, z);
        ++c2;
    }
    if (lane == 0) ood[i] = c2 > 0 && d1 / (s2 / (double)c2) > ratio;
}

// role switch of a merged index: data id v < nx becomes nq + v, query node
// id v >= nx becomes v - nx (-1 padding stays)
__global__ void k_swap_ids(int32_t *p, int64_t n, int32_t nx, int32_t nq) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t v = p[i];
    if (v >= 0) p[i] = v < nx ? v + nq : v - nx;
}

__global__ void k_offset_ids(int32_t *p, int64_t n, int32_t off) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && p[i] >= 0) p[i] += off;
}

__global__ void k_iota(int32_t *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = (int32_t)i;
}

__global__ void k_stamp(int32_t *inb, int64_t nq, const int32_t *ids, int64_t n, int32_t gen,
                        int32_t *err) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t q = ids ? ids[i] : (int32_t)i;
    if (q < 0 || q >= nq) { atomicOr(err, 8); return; }
    inb[q] = gen;
}

__global__ void k_depth_keys(const int32_t *depth, int64_t nq, const int32_t *ids, int64_t n,
                             int32_t *keys, int32_t *pos) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t q = ids ? ids[i] : (int32_t)i;
    keys[i] = (q >= 0 && q < nq) ? depth[q] : 0;
    pos[i] = (int32_t)i;
}

__global__ void k_gather_ids(const int32_t *ids, const int32_t *pos, int64_t n, int32_t *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = ids ? ids[pos[i]] : pos[i];
}

__global__ void k_gather_slots(const int32_t *qlist, const int32_t *qpos, const int32_t *slots,
                               int64_t n, int32_t *q2, int32_t *p2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    q2[i] = qlist[slots[i]];
    p2[i] = qpos[slots[i]];
}

// densest first without a sort: slot i goes to the bucket of its d1 (the
// top 12 bits below the sign of the float: exponent and 4 mantissa bits, so
// buckets are ordered by d1 and 6 % wide), the buckets are counted, scanned
// and scattered
__device__ __forceinline__ int density_bucket(const int32_t *adj, const float *elen, int R,
                                              int64_t nx, int64_t nq, int32_t q) {
    if (q < 0 || q >= nq) return kOrderBuckets - 1;
    const int64_t u = nx + q;
    float sum = 0.f;
    int c = 0;
    for (int j = 0; j < R; ++j) {
        const int32_t y = adj[u * R + j];
        if (y >= 0 && y < nx) { sum += elen[u * R + j]; ++c; }
    }
    const float d1 = c ? sum / (float)c : INFINITY;
    return min((int)(__float_as_uint(d1) >> 19), kOrderBuckets - 1);
}

// first kernel of a replayed batch step.  Workgroup 0 sets up batch b =
// ctr[kBatchCursor]: its eps and stats rows in the join arguments, the
// per-batch counters cleared, where its pairs begin and the clock.  Every
// thread i < count writes the batch's query id i to qlist and, when ordering
// densest first, its d1 bucket (counted in hist).
__global__ void __launch_bounds__(256)
k_batch_start(const BatchDesc *desc, JoinArgs *args, int32_t *ctr, uint64_t *rec, int64_t nmax,
              const int32_t *adj, const float *elen, int R, int64_t nx, int64_t nq,
              int32_t *qlist, int32_t *bucket, uint32_t *hist) {
    __shared__ uint32_t lh[kOrderBuckets];
    const int b = ctr[kBatchCursor];
    const BatchDesc d = desc[b];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        args->eps = d.eps;
        args->eps2 = d.eps2;
        args->stats = d.stats;
        ctr[kBatchCount] = d.count;
        ctr[2] = 0;  // first overflow list
        ctr[4] = 0;  // global regions taken by promotion
        ctr[kBatchOvf2] = 0;
        ctr[kBatchOvf3] = 0;
        rec[kBatchRec * b + 0] = *reinterpret_cast<const unsigned long long *>(ctr);
        rec[kBatchRec * b + 4] = *reinterpret_cast<const unsigned long long *>(ctr + 6);
        rec[kBatchRec * b + 6] = (uint64_t)wall_clock64();
    }
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool ok = i < nmax && i < d.count;
    int32_t q = 0;
    if (ok) {
        q = d.ids ? d.ids[d.start + i] : (int32_t)(d.start + i);
        qlist[i] = q;
    }
    if (bucket == nullptr) return;  // the same for every thread
    // bucket counts: per workgroup in LDS, then one global atomic per bucket
    for (int k = threadIdx.x; k < kOrderBuckets; k += blockDim.x) lh[k] = 0u;
    __syncthreads();
    if (ok) {
        const int k = density_bucket(adj, elen, R, nx, nq, q);
        bucket[i] = k;
        atomicAdd(&lh[k], 1u);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kOrderBuckets; k += blockDim.x)
        if (lh[k]) atomicAdd(&hist[k], lh[k]);
}

// one workgroup of 1024 threads, 4 buckets each: off = exclusive scan of
// hist; hist is cleared for the next batch
__global__ void __launch_bounds__(1024) k_batch_scan(uint32_t *hist, uint32_t *off) {
    __shared__ uint32_t part[1024];
    const int t = threadIdx.x;
    uint32_t c[4], sum = 0;
    for (int j = 0; j < 4; ++j) {
        c[j] = hist[4 * t + j];
        sum += c[j];
    }
    part[t] = sum;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {  // inclusive Hillis-Steele scan
        const uint32_t v = t >= d ? part[t - d] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint32_t run = part[t] - sum;
    for (int j = 0; j < 4; ++j) {
        off[4 * t + j] = run;
        run += c[j];
        hist[4 * t + j] = 0u;
    }
}

// slot i goes to off[bucket] + its rank: each workgroup reserves one range
// per bucket (one global atomic per bucket), ranks come from LDS counters
__device__ __forceinline__ void scatter_ranked(bool ok, int k, uint32_t *off, uint32_t *lh,
                                               uint32_t *lb, uint32_t &p) {
    for (int j = threadIdx.x; j < kOrderBuckets; j += blockDim.x) lh[j] = 0u;
    __syncthreads();
    uint32_t r = 0;
    if (ok) r = atomicAdd(&lh[k], 1u);
    __syncthreads();
    for (int j = threadIdx.x; j < kOrderBuckets; j += blockDim.x)
        if (lh[j]) lb[j] = atomicAdd(&off[j], lh[j]);
    __syncthreads();
    if (ok) p = lb[k] + r;
}

__global__ void __launch_bounds__(256)
k_batch_scatter(const int32_t *qlist, const int32_t *ctr, int64_t nmax, const int32_t *bucket,
                uint32_t *off, int32_t *q2, int32_t *p2) {
    __shared__ uint32_t lh[kOrderBuckets], lb[kOrderBuckets];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool ok = i < nmax && i < ctr[kBatchCount];
    const int k = ok ? bucket[i] : 0;
    uint32_t p = 0;
    scatter_ranked(ok, k, off, lh, lb, p);
    if (ok) {
        q2[p] = qlist[i];
        p2[p] = (int32_t)i;
    }
}

// densest first for one join: the d1 bucket of each slot, counted per
// workgroup in LDS (one global atomic per bucket and workgroup)
__global__ void __launch_bounds__(256)
k_density_buckets(const int32_t *adj, const float *elen, int R, int64_t nx, int64_t nq,
                  const int32_t *ids, int64_t n, int32_t *bucket, uint32_t *hist) {
    __shared__ uint32_t lh[kOrderBuckets];
    for (int k = threadIdx.x; k < kOrderBuckets; k += blockDim.x) lh[k] = 0u;
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const int k = density_bucket(adj, elen, R, nx, nq, ids ? ids[i] : (int32_t)i);
        bucket[i] = k;
        atomicAdd(&lh[k], 1u);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < kOrderBuckets; k += blockDim.x)
        if (lh[k]) atomicAdd(&hist[k], lh[k]);
}

// ... and each slot placed after the slots of lower buckets
__global__ void __launch_bounds__(256)
k_bucket_scatter(const int32_t *ids, int64_t n, const int32_t *bucket, uint32_t *off,
                 int32_t *qlist, int32_t *qpos) {
    __shared__ uint32_t lh[kOrderBuckets], lb[kOrderBuckets];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool ok = i < n;
    const int k = ok ? bucket[i] : 0;
    uint32_t p = 0;
    scatter_ranked(ok, k, off, lh, lb, p);
    if (ok) {
        qlist[p] = ids ? ids[i] : (int32_t)i;
        qpos[p] = (int32_t)i;
    }
}

// end of the batch step: where its pairs end, how many queries each re-run
// took; the cursor moves to the next batch
__global__ void k_batch_end(int32_t *ctr, uint64_t *rec) {
    if (threadIdx.x != 0) return;
    const int b = ctr[kBatchCursor];
    rec[kBatchRec * b + 1] = *reinterpret_cast<const unsigned long long *>(ctr);
    rec[kBatchRec * b + 2] = (uint64_t)ctr[2];
    rec[kBatchRec * b + 3] = (uint64_t)ctr[kBatchOvf2];
    rec[kBatchRec * b + 5] = *reinterpret_cast<const unsigned long long *>(ctr + 6);
    rec[kBatchRec * b + 7] = (uint64_t)wall_clock64();
    if (ctr[kBatchOvf3] != 0) atomicOr(ctr + 3, 64);
    ctr[kBatchCursor] = b + 1;
}

__global__ void k_pack_keys(const int32_t *q, const int32_t *x, int64_t n, uint64_t *key) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) key[i] = ((uint64_t)(uint32_t)q[i] << 32) | (uint32_t)x[i];
}

__global__ void k_unpack_keys(const uint64_t *key, int64_t n, int32_t *qx) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    qx[2 * i] = (int32_t)(key[i] >> 32);
    qx[2 * i + 1] = (int32_t)(uint32_t)key[i];
}

__global__ void k_interleave(const int32_t *q, const int32_t *x, int64_t n, int32_t *qx) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    qx[2 * i] = q[i];
    qx[2 * i + 1] = x[i];
}

inline unsigned grid1(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

}  // namespace

int num_cus() {
    static int cached[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (dev < 0 || dev >= 64) return 256;
    if (!cached[dev]) {
        hipDeviceProp_t p;
        if (hipGetDeviceProperties(&p, dev) != hipSuccess) return 256;
        cached[dev] = p.multiProcessorCount;
    }
    return cached[dev];
}

void launch_pad_rows(const float *src, int64_t rows, int d, float *dst, int dp, hipStream_t s) {
    const int64_t n = rows * (int64_t)dp;
    if (n == 0) return;
    hipLaunchKernelGGL(k_pad_rows, dim3(grid1(n)), dim3(256), 0, s, src, rows, d, dst, dp);
}

void launch_quantize(const float *vec, int64_t rows, int dp, uint8_t *u8, uint16_t *bf16,
                     int32_t *flag, hipStream_t s) {
    const int64_t n = rows * (int64_t)dp;
    if (n == 0) return;
    hipLaunchKernelGGL(k_quantize, dim3(std::min<unsigned>(grid1(n), 8192)), dim3(256), 0, s, vec, n, u8,
                       bf16, flag);
}

void launch_edge_lengths(const float *vec, int dp, const int32_t *adj, int64_t N, int R,
                         float *elen, hipStream_t s) {
    if (N == 0) return;
    hipLaunchKernelGGL(k_edge_lengths, dim3((unsigned)N), dim3(64), 0, s, vec, dp, adj, N, R, elen,
                       nullptr);
}

void launch_edge_lengths_rows(const float *vec, int dp, const int32_t *adj, int64_t N, int R,
                              const int32_t *rows, int64_t M, float *elen, hipStream_t s) {
    if (M == 0) return;
    hipLaunchKernelGGL(k_edge_lengths, dim3((unsigned)M), dim3(64), 0, s, vec, dp, adj, N, R, elen,
                       rows);
}

void launch_dist_to_node(const float *vec, int dp, int64_t first, int64_t n, int32_t node,
                         float *out, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_dist_to_node, dim3(grid1(n)), dim3(256), 0, s, vec, dp, first, n, node, out);
}

// ----------------------------------------------------- upper layers --
// dst[i][:] = src[ids[i]][:] (rows of dp floats)
__global__ void k_gather_rows_f32(const float *src, int dp, const int32_t *ids, int64_t n,
                                  float *dst) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * (dp / 4)) return;
    const int64_t i = e / (dp / 4), c = e - i * (dp / 4);
    reinterpret_cast<float4 *>(dst + i * dp)[c] =
        reinterpret_cast<const float4 *>(src + (int64_t)ids[i] * dp)[c];
}

// adj[e] = ids[adj[e]] for every entry >= 0 (local row -> data id)
__global__ void k_map_ids(int32_t *adj, int64_t n, const int32_t *ids) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n && adj[e] >= 0) adj[e] = ids[adj[e]];
}

// pos[ids[i]] = i
__global__ void k_scatter_pos(int32_t *pos, const int32_t *ids, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) pos[ids[i]] = (int32_t)i;
}

// Greedy descent through the upper layers, one wave per query: from the top
// layer's entry, move to the neighbour smallest by (distance, id) while it
// is smaller than the current node, then one layer down; 8 lanes per
// neighbour row (16-byte loads), fp32 distances (squared for L2).  The
// moves of a layer are bounded by its node count (each move strictly
// decreases (distance, id)).
__global__ void __launch_bounds__(256)
k_descend(const float *vec, int dp, int64_t nx, int metric, int nl, const int64_t *loff,
          const int64_t *lcnt, const int32_t *lpos, const int32_t *ladj, int R, int32_t top,
          const int32_t *qids, int64_t n, int32_t *seed_i, int32_t *seed_q, int32_t *moves,
          int32_t *err) {
    const int lane = threadIdx.x & 63, g = lane >> 3, p = lane & 7;
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= n) return;
    const int32_t qi = qids ? qids[i] : (int32_t)i;
    const float4 *q = reinterpret_cast<const float4 *>(vec + (nx + qi) * dp);
    auto dist = [&](int32_t v) {  // every lane of the 8-lane group gets it
        const float4 *x = reinterpret_cast<const float4 *>(vec + (int64_t)v * dp);
        float acc = 0.f;
        for (int c = p; c < dp / 4; c += 8) {
            const float4 a = q[c], b = x[c];
            if (metric == VJ_L2) {
                float t = a.x - b.x; acc = fmaf(t, t, acc);
                t = a.y - b.y; acc = fmaf(t, t, acc);
                t = a.z - b.z; acc = fmaf(t, t, acc);
                t = a.w - b.w; acc = fmaf(t, t, acc);
            } else {
                acc = fmaf(a.x, b.x, acc); acc = fmaf(a.y, b.y, acc);
                acc = fmaf(a.z, b.z, acc); acc = fmaf(a.w, b.w, acc);
            }
        }
        acc += __shfl_xor(acc, 4);
        acc += __shfl_xor(acc, 2);
        acc += __shfl_xor(acc, 1);
        return metric == VJ_L2 ? acc : 1.f - acc;
    };
    int32_t c = top;
    float dc = dist(c);
    int32_t mv = 0;
    for (int j = nl - 1; j >= 0; --j) {
        for (int64_t it = 0; it < lcnt[j]; ++it) {
            const int32_t r = lpos[(int64_t)j * nx + c];
            if (r < 0) {  // the layers are nested: cannot happen
                if (lane == 0) atomicOr(err, 1);
                break;
            }
            const int32_t *row = ladj + (loff[j] + r) * R;
            float bd = dc;
            int32_t bv = c;
            for (int b0 = 0; b0 < R; b0 += 8) {
                const int k = b0 + g;
                const int32_t v = k < R ? row[k] : -1;
                // every lane of the group evaluates (a padding slot evaluates c)
                const bool ok = v >= 0 && v < nx;
                const float dv = dist(ok ? v : c);
                if (ok && (dv < bd || (dv == bd && v < bv))) { bd = dv; bv = v; }
            }
            // the smallest (distance, id) over the eight groups
#pragma unroll
            for (int off = 8; off < 64; off <<= 1) {
                const float od = __shfl_xor(bd, off);
                const int32_t ov = __shfl_xor(bv, off);
                if (od < bd || (od == bd && ov < bv)) { bd = od; bv = ov; }
            }
            if (bv == c) break;
            c = bv;
            dc = bd;
            ++mv;
        }
    }
    if (lane == 0) {
        if (seed_i) seed_i[i] = c;
        if (seed_q) seed_q[qi] = c;
        if (moves) moves[i] = mv;
    }
}

void gather_rows_f32(const float *src, int dp, const int32_t *ids, int64_t n, float *dst,
                     hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_gather_rows_f32, dim3(grid1(n * (dp / 4))), dim3(256), 0, s, src, dp, ids,
                       n, dst);
    VJ_HIP(hipGetLastError());
}

void map_ids(int32_t *adj, int64_t n, const int32_t *ids, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_map_ids, dim3(grid1(n)), dim3(256), 0, s, adj, n, ids);
    VJ_HIP(hipGetLastError());
}

void scatter_pos(int32_t *pos, const int32_t *ids, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_scatter_pos, dim3(grid1(n)), dim3(256), 0, s, pos, ids, n);
    VJ_HIP(hipGetLastError());
}

void descend(const float *vec, int dp, int64_t nx, int metric, int nl, const int64_t *loff,
             const int64_t *lcnt, const int32_t *lpos, const int32_t *ladj, int R, int32_t top,
             const int32_t *qids, int64_t n, int32_t *seed_i, int32_t *seed_q, int32_t *moves,
             int32_t *err, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_descend, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, vec, dp, nx,
                       metric, nl, loff, lcnt, lpos, ladj, R, top, qids, n, seed_i, seed_q, moves,
                       err);
    VJ_HIP(hipGetLastError());
}

// Counter calibration: out[i] = sum of row ids[i] of rows [nrows][dp]
// (fp32, dp a multiple of 32), read as the join reads a row: 8 lanes per
// row, 16 bytes per lane per load, each load of the 8-lane group covering
// whole 128-byte lines; 8 rows per wave.
__global__ void __launch_bounds__(256)
k_calib_gather(const float *rows, int64_t nrows, int dp, const int32_t *ids, int64_t n,
               float *out) {
    const int lane = threadIdx.x & 63, g = lane >> 3, p = lane & 7;
    const int64_t i = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 8 + g;
    const bool ok = i < n;
    const int32_t r = ok ? ids[i] : 0;
    const bool rok = ok && r >= 0 && r < nrows;
    const float4 *row = reinterpret_cast<const float4 *>(rows + (int64_t)(rok ? r : 0) * dp);
    float acc = 0.f;
    if (rok)
        for (int c = p; c < dp / 4; c += 8) {
            const float4 v = row[c];
            acc += (v.x + v.y) + (v.z + v.w);
        }
    acc += __shfl_xor(acc, 4);
    acc += __shfl_xor(acc, 2);
    acc += __shfl_xor(acc, 1);
    if (ok && p == 0) out[i] = acc;
}

void calib_gather(const float *rows, int64_t nrows, int dp, const int32_t *ids, int64_t n,
                  float *out, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_calib_gather, dim3((unsigned)((n + 31) / 32)), dim3(256), 0, s, rows,
                       nrows, dp, ids, n, out);
    VJ_HIP(hipGetLastError());
}

void fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_fill_i32, dim3(grid1(n)), dim3(256), 0, s, p, n, v);
}

void nn_ood(const float *vec, int dp, int64_t nx, int64_t nq, const int32_t *adj, int R,
            const int32_t *w, double ratio, uint8_t *ood, hipStream_t s) {
    if (nq <= 0) return;
    hipLaunchKernelGGL(k_nn_ood, dim3((unsigned)((nq + 3) / 4)), dim3(256), 0, s, vec, dp, nx, nq,
                       adj, R, w, ratio, ood);
    VJ_HIP(hipGetLastError());
}

void swap_ids(int32_t *p, int64_t n, int32_t nx, int32_t nq, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_swap_ids, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, nx, nq);
    VJ_HIP(hipGetLastError());
}

void launch_quantize_f8(const float *vec, int64_t rows, int dp, uint8_t *codes, float2 *meta,
                        hipStream_t s) {
    if (rows <= 0) return;
    hipLaunchKernelGGL(k_quantize_f8, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, s, vec, rows,
                       dp, codes, meta);
    VJ_HIP(hipGetLastError());
}

void offset_ids(int32_t *p, int64_t n, int32_t off, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_offset_ids, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, off);
    VJ_HIP(hipGetLastError());
}

void iota_i32(int32_t *p, int64_t n, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_iota, dim3(grid1(n)), dim3(256), 0, s, p, n);
}

void stamp_batch(int32_t *inb, int64_t nq, const int32_t *ids, int64_t n, int32_t gen,
                 int32_t *err, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_stamp, dim3(grid1(n)), dim3(256), 0, s, inb, nq, ids, n, gen, err);
}

void gather_slots(const int32_t *qlist, const int32_t *qpos, const int32_t *slots, int64_t n,
                  int32_t *q2, int32_t *p2, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_gather_slots, dim3(grid1(n)), dim3(256), 0, s, qlist, qpos, slots, n, q2, p2);
}

void batch_start(const BatchDesc *desc, JoinArgs *args, int32_t *ctr, uint64_t *rec, int64_t nmax,
                 const int32_t *adj, const float *elen, int R, int64_t nx, int64_t nq,
                 int32_t *qlist, int32_t *bucket, uint32_t *hist, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_start, dim3(std::max(1u, grid1(nmax))), dim3(256), 0, s, desc, args,
                       ctr, rec, nmax, adj, elen, R, nx, nq, qlist, bucket, hist);
}

void batch_order(const int32_t *qlist, const int32_t *ctr, int64_t nmax, const int32_t *bucket,
                 uint32_t *hist, uint32_t *off, int32_t *q2, int32_t *p2, hipStream_t s) {
    if (nmax == 0) return;
    hipLaunchKernelGGL(k_batch_scan, dim3(1), dim3(1024), 0, s, hist, off);
    hipLaunchKernelGGL(k_batch_scatter, dim3(grid1(nmax)), dim3(256), 0, s, qlist, ctr, nmax, bucket,
                       off, q2, p2);
}

void batch_end(int32_t *ctr, uint64_t *rec, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_end, dim3(1), dim3(64), 0, s, ctr, rec);
}

// processing order parents-first: stable sort of caller positions by MST depth
void sort_pairs_i32(const int32_t *keys_in, int32_t *keys_out, const int32_t *vals_in,
                    int32_t *vals_out, int64_t n, int end_bit, DevBuf &tmp, hipStream_t s) {
    if (n == 0) return;
    size_t bytes = 0;
    VJ_HIP(rocprim::radix_sort_pairs(nullptr, bytes, keys_in, keys_out, vals_in, vals_out,
                                     (size_t)n, 0, end_bit, s));
    tmp.reserve(bytes);
    VJ_HIP(rocprim::radix_sort_pairs(tmp.p, bytes, keys_in, keys_out, vals_in, vals_out,
                                     (size_t)n, 0, end_bit, s));
}

namespace {
struct CachedBlock {
    void *p;
    size_t n;
};
struct BlockCache {
    std::mutex mu;
    std::vector<CachedBlock> blocks[64];
    size_t held[64] = {};
};
// never destroyed: no HIP call runs during static destruction
BlockCache &block_cache() {
    static BlockCache *c = new BlockCache;
    return *c;
}
void drop_cached(BlockCache &c, int dev) {
    for (const CachedBlock &b : c.blocks[dev]) (void)hipFree(b.p);
    c.blocks[dev].clear();
    c.held[dev] = 0;
}
}  // namespace

void *dev_alloc(size_t n, int *dev, size_t *cap) {
    VJ_HIP(hipGetDevice(dev));
    BlockCache &c = block_cache();
    const int d = *dev;
    *cap = n;
    if (n >= kBlockCacheMin && d >= 0 && d < 64) {
        std::lock_guard<std::mutex> lk(c.mu);
        auto &v = c.blocks[d];
        int best = -1;
        for (int i = 0; i < (int)v.size(); ++i)
            if (v[i].n >= n && v[i].n / 2 <= n && (best < 0 || v[i].n < v[best].n)) best = i;
        if (best >= 0) {
            void *p = v[best].p;
            *cap = v[best].n;
            c.held[d] -= v[best].n;
            v.erase(v.begin() + best);
            return p;
        }
        // a new block: rounded up to an eighth of the request's power of two
        size_t g = (size_t)1 << 63;
        while (g > n) g >>= 1;
        g >>= 3;
        *cap = (n + g - 1) / g * g;
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, *cap);
    if (e == hipErrorOutOfMemory && d >= 0 && d < 64) {
        (void)hipGetLastError();
        {
            std::lock_guard<std::mutex> lk(c.mu);
            drop_cached(c, d);
        }
        e = hipMalloc(&p, *cap);
    }
    VJ_HIP(e);
    return p;
}

size_t trim_block_cache() {
    int d = -1;
    VJ_HIP(hipGetDevice(&d));
    if (d < 0 || d >= 64) return 0;
    BlockCache &c = block_cache();
    std::lock_guard<std::mutex> lk(c.mu);
    const size_t n = c.held[d];
    drop_cached(c, d);
    return n;
}

void dev_free(void *p, size_t n, int dev) {
    // a freed buffer may still be read by work in flight on any stream, as
    // with hipFree: wait for the device before the block can be reused
    BlockCache &c = block_cache();
    if (n >= kBlockCacheMin && dev >= 0 && dev < 64) {
        int cur = -1;
        if (hipGetDevice(&cur) == hipSuccess && cur == dev && hipDeviceSynchronize() == hipSuccess) {
            std::lock_guard<std::mutex> lk(c.mu);
            c.blocks[dev].push_back({p, n});
            c.held[dev] += n;
            while (c.held[dev] > kBlockCacheMax && !c.blocks[dev].empty()) {
                (void)hipFree(c.blocks[dev].front().p);
                c.held[dev] -= c.blocks[dev].front().n;
                c.blocks[dev].erase(c.blocks[dev].begin());
            }
            return;
        }
    }
    (void)hipFree(p);
}

__global__ void k_scan_tail(const int32_t *in, int64_t *out, int64_t n) {
    out[n] = n > 0 ? out[n - 1] + in[n - 1] : 0;
}

void exclusive_scan_i32_i64(const int32_t *in, int64_t *out, int64_t n, DevBuf &tmp,
                            hipStream_t s) {
    if (n > 0) {
        size_t bytes = 0;
        VJ_HIP(rocprim::exclusive_scan(nullptr, bytes, in, out, (int64_t)0, (size_t)n,
                                       rocprim::plus<int64_t>(), s));
        tmp.reserve(bytes);
        VJ_HIP(rocprim::exclusive_scan(tmp.p, bytes, in, out, (int64_t)0, (size_t)n,
                                       rocprim::plus<int64_t>(), s));
    }
    hipLaunchKernelGGL(k_scan_tail, dim3(1), dim3(1), 0, s, in, out, n);
}

void order_by_depth(const int32_t *depth, int64_t nq, const int32_t *ids, int64_t n,
                    int32_t *qlist, int32_t *qpos, DevBuf &tmp, hipStream_t s) {
    if (n == 0) return;
    DevBuf keys(n * sizeof(int32_t)), keys2(n * sizeof(int32_t)), pos(n * sizeof(int32_t));
    hipLaunchKernelGGL(k_depth_keys, dim3(grid1(n)), dim3(256), 0, s, depth, nq, ids, n,
                       keys.as<int32_t>(), pos.as<int32_t>());
    size_t bytes = 0;
    VJ_HIP(rocprim::radix_sort_pairs(nullptr, bytes, keys.as<int32_t>(), keys2.as<int32_t>(),
                                     pos.as<int32_t>(), qpos, (size_t)n, 0, 31, s));
    tmp.reserve(bytes);
    VJ_HIP(rocprim::radix_sort_pairs(tmp.p, bytes, keys.as<int32_t>(), keys2.as<int32_t>(),
                                     pos.as<int32_t>(), qpos, (size_t)n, 0, 31, s));
    hipLaunchKernelGGL(k_gather_ids, dim3(grid1(n)), dim3(256), 0, s, ids, qpos, n, qlist);
    VJ_HIP(hipStreamSynchronize(s));  // the temporaries above are freed on return
}

void order_by_density(const int32_t *adj, const float *elen, int R, int64_t nx, int64_t nq,
                      const int32_t *ids, int64_t n, int32_t *qlist, int32_t *qpos, DevBuf &keys,
                      DevBuf &tmp, hipStream_t s) {
    if (n == 0) return;
    // d1 buckets (4,096, about 6 % wide) counted, scanned and scattered: the
    // order only has to start dense neighbourhoods first, and three small
    // kernels cost less than a radix sort
    keys.reserve(n * sizeof(int32_t));
    tmp.reserve(2 * kOrderBuckets * sizeof(uint32_t));
    uint32_t *hist = tmp.as<uint32_t>(), *off = hist + kOrderBuckets;
    VJ_HIP(hipMemsetAsync(hist, 0, kOrderBuckets * sizeof(uint32_t), s));
    hipLaunchKernelGGL(k_density_buckets, dim3(grid1(n)), dim3(256), 0, s, adj, elen, R, nx, nq, ids,
                       n, keys.as<int32_t>(), hist);
    hipLaunchKernelGGL(k_batch_scan, dim3(1), dim3(1024), 0, s, hist, off);
    hipLaunchKernelGGL(k_bucket_scatter, dim3(grid1(n)), dim3(256), 0, s, ids, n, keys.as<int32_t>(),
                       off, qlist, qpos);
    VJ_HIP(hipGetLastError());
}

void export_pairs(const Pairs &r, int32_t *qx, float *dist, bool sorted, hipStream_t s) {
    const int64_t n = r.count;
    if (n == 0) return;
    if (!sorted) {
        hipLaunchKernelGGL(k_interleave, dim3(grid1(n)), dim3(256), 0, s, r.q.as<int32_t>(),
                           r.x.as<int32_t>(), n, qx);
        if (dist) VJ_HIP(hipMemcpyAsync(dist, r.dist.p, n * sizeof(float), hipMemcpyDeviceToDevice, s));
        return;
    }
    DevBuf k1(n * 8), k2(n * 8), v2(n * sizeof(float)), tmp;
    hipLaunchKernelGGL(k_pack_keys, dim3(grid1(n)), dim3(256), 0, s, r.q.as<int32_t>(),
                       r.x.as<int32_t>(), n, k1.as<uint64_t>());
    size_t bytes = 0;
    VJ_HIP(rocprim::radix_sort_pairs(nullptr, bytes, k1.as<uint64_t>(), k2.as<uint64_t>(),
                                     r.dist.as<float>(), v2.as<float>(), (size_t)n, 0, 64, s));
    tmp.alloc(bytes);
    VJ_HIP(rocprim::radix_sort_pairs(tmp.p, bytes, k1.as<uint64_t>(), k2.as<uint64_t>(),
                                     r.dist.as<float>(), v2.as<float>(), (size_t)n, 0, 64, s));
    hipLaunchKernelGGL(k_unpack_keys, dim3(grid1(n)), dim3(256), 0, s, k2.as<uint64_t>(), n, qx);
    if (dist) VJ_HIP(hipMemcpyAsync(dist, v2.p, n * sizeof(float), hipMemcpyDeviceToDevice, s));
    VJ_HIP(hipStreamSynchronize(s));  // temporaries are freed on return
}

}  // namespace vj
