// Difficulty predictor on the GPU: the post-probe features of a query (the
// d1/d2 signal of CheckHybrid, Section 4.4, extended), and an MLP that maps
// them to the predicted recall under a few out-range pop budgets; training
// (mean BCE, Adam) runs on the device.  The dense layers are fp32 tiled
// GEMMs on the vector ALUs (64x64 output tile per workgroup, k-steps of 16
// staged through LDS); at 776 -> 256 -> 256 -> 4 they are small and bound by
// launch latency, not by MFMA throughput.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <random>
#include <vector>

#include "predictor.h"

namespace vj {
namespace {

inline unsigned g1p(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// ------------------------------------------------------------- features --
// One wave per query.  Distances in the join metric (L2: |q - y|; IP:
// 1 - <q, y>); d1 and d2 in L2 units (|q - y| from the vectors, stored edge
// lengths for d2).  Row layout: q[0..d), f0..f7.  The neighbours of q are
// evaluated 8 at a time (8 lanes per row) and the R x R second-hop entries
// are spread over the lanes, so the loads of a query are independent.
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fminf(v, __shfl_xor(v, off));
    return v;
}

__device__ __forceinline__ float group8_sum(float v) {
#pragma unroll
    for (int off = 4; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

__global__ void __launch_bounds__(256)
k_features(const float *vec, int dp, int d, int64_t nx, const int32_t *adj, const float *elen,
           int R, int32_t entry, int metric, float eps, const int32_t *qlist, int64_t n,
           float *out) {
    const int lane = threadIdx.x & 63;
    const int g = lane >> 3, p = lane & 7;
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= n) return;
    const int64_t q = nx + qlist[i];
    const float *qv = vec + q * dp;
    float *o = out + i * (int64_t)(d + kFeatures);
    for (int c = lane; c < d; c += 64) o[c] = qv[c];
    const bool l2 = metric == VJ_L2;
    // f1: the entry, one whole-wave dot
    float f1;
    {
        const float *ev = vec + (int64_t)entry * dp;
        float acc = 0.f;
        for (int c = lane; c < dp; c += 64) {
            if (l2) { const float t = qv[c] - ev[c]; acc = fmaf(t, t, acc); }
            else acc = fmaf(qv[c], ev[c], acc);
        }
        acc = wave_sum(acc);
        f1 = l2 ? sqrtf(acc) : 1.0f - acc;
    }
    // A = N(q) among the data nodes: group g takes neighbours g, g + 8, ...
    float mn = INFINITY, s1 = 0.f;
    int na = 0, nin = 0;
    for (int j0 = 0; j0 < R; j0 += 8) {
        const int j = j0 + g;
        const int32_t y = j < R ? adj[q * R + j] : -1;
        const bool ok = y >= 0 && y < nx;
        float sq = 0.f, dt = 0.f;
        if (ok) {
            const float *yv = vec + (int64_t)y * dp;
            for (int c = p; c < dp; c += 8) {
                const float a = qv[c], b = yv[c];
                const float t = a - b;
                sq = fmaf(t, t, sq);
                dt = fmaf(a, b, dt);
            }
        }
        sq = group8_sum(sq);
        dt = group8_sum(dt);
        if (ok && p == 0) {
            const float dy = l2 ? sqrtf(sq) : 1.0f - dt;
            mn = fminf(mn, dy);
            if (dy < eps) ++nin;
            s1 += sqrtf(sq);
            ++na;
        }
    }
    // d2: stored edge lengths of N(y) for y in A, z a data node other than q
    float s2 = 0.f;
    int c2 = 0;
    for (int e = lane; e < R * R; e += 64) {
        const int yj = e / R, zj = e - yj * R;
        const int32_t y = adj[q * R + yj];
        if (y < 0 || y >= nx) continue;
        const int32_t z = adj[(int64_t)y * R + zj];
        if (z >= 0 && z < nx && z != q) {
            s2 += elen[(int64_t)y * R + zj];
            ++c2;
        }
    }
    mn = wave_min(mn);
    s1 = wave_sum(s1);
    s2 = wave_sum(s2);
    na = (int)wave_sum((float)na);
    nin = (int)wave_sum((float)nin);
    c2 = (int)wave_sum((float)c2);
    if (lane == 0) {
        const float d1 = na ? s1 / (float)na : 0.f;
        const float d2 = c2 ? s2 / (float)c2 : 0.f;
        float *f = o + d;
        f[0] = eps;
        f[1] = f1;
        f[2] = na ? mn : 0.f;
        f[3] = d1;
        f[4] = d2;
        f[5] = d2 > 0.f ? d1 / d2 : 0.f;
        f[6] = (float)na / (float)R;
        f[7] = (float)nin / (float)R;
    }
}

// ----------------------------------------------------------------- GEMM --
// C[m][n] = sum_k A'[m][k] B'[k][n] (+ bias[n]) (ReLU) (masked by M[m][n] > 0)
// A' = TA ? A^T : A (A row-major, leading dimension lda); B' likewise.
template <bool TA, bool TB>
__global__ void __launch_bounds__(256)
k_gemm(int M, int N, int K, const float *A, int lda, const float *B, int ldb, float *C, int ldc,
       const float *bias, int relu, const float *mask, int ldm) {
    constexpr int BM = 64, BN = 64, BK = 16;
    __shared__ float As[BK][BM + 4];
    __shared__ float Bs[BK][BN + 4];
    const int t = threadIdx.x;
    const int tx = t & 15, ty = t >> 4;
    const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    float acc[4][4] = {};
    for (int k0 = 0; k0 < K; k0 += BK) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            // 1024 elements of each tile; consecutive threads walk the operand's
            // contiguous dimension
            const int e = t + 256 * r;
            {
                const int kk = TA ? e / BM : e % BK, mm = TA ? e % BM : e / BK;
                const int gm = m0 + mm, gk = k0 + kk;
                float va = 0.f;
                if (gm < M && gk < K) va = TA ? A[(size_t)gk * lda + gm] : A[(size_t)gm * lda + gk];
                As[kk][mm] = va;
            }
            {
                const int kk = TB ? e % BK : e / BN, nn = TB ? e / BK : e % BN;
                const int gn = n0 + nn, gk = k0 + kk;
                float vb = 0.f;
                if (gn < N && gk < K) vb = TB ? B[(size_t)gn * ldb + gk] : B[(size_t)gk * ldb + gn];
                Bs[kk][nn] = vb;
            }
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < BK; ++kk) {
            float a[4], b[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) a[i] = As[kk][ty * 4 + i];
#pragma unroll
            for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx * 4 + j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(a[i], b[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int gm = m0 + ty * 4 + i;
        if (gm >= M) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int gn = n0 + tx * 4 + j;
            if (gn >= N) continue;
            float v = acc[i][j] + (bias ? bias[gn] : 0.f);
            if (relu) v = fmaxf(v, 0.f);
            if (mask && !(mask[(size_t)gm * ldm + gn] > 0.f)) v = 0.f;
            C[(size_t)gm * ldc + gn] = v;
        }
    }
}

template <bool TA, bool TB>
void gemm(int M, int N, int K, const float *A, int lda, const float *B, int ldb, float *C, int ldc,
          const float *bias, bool relu, const float *mask, int ldm, hipStream_t s) {
    if (M <= 0 || N <= 0) return;
    hipLaunchKernelGGL((k_gemm<TA, TB>), dim3(g1p(N, 64), g1p(M, 64)), dim3(256), 0, s, M, N, K, A,
                       lda, B, ldb, C, ldc, bias, relu ? 1 : 0, mask, ldm);
}

// ------------------------------------------------------ elementwise parts --
__global__ void k_normalize(const float *X, int64_t n, int din, const float *mu,
                            const float *inv_sigma, float *Y) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * din) return;
    const int c = (int)(e % din);
    Y[e] = (X[e] - mu[c]) * inv_sigma[c];
}

// G = mask (sigmoid(Z) - Y) / cnt; loss += mask BCE(Z, Y)
__global__ void k_bce(const float *Z, const float *Y, const float *mask, int64_t total, float inv_cnt,
                      float *G, double *loss) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double l = 0.0;
    if (e < total) {
        const float m = mask ? (mask[e] != 0.f ? 1.f : 0.f) : 1.f;
        const float z = Z[e], y = Y[e];
        const float sg = 1.f / (1.f + expf(-z));
        G[e] = m * (sg - y) * inv_cnt;
        l = (double)m * ((double)fmaxf(z, 0.f) - (double)z * y + (double)log1pf(expf(-fabsf(z))));
    }
    l = (double)wave_sum((float)l);
    if ((threadIdx.x & 63) == 0 && l != 0.0) atomicAdd(loss, l);
}

__global__ void k_mask_count(const float *mask, int64_t total, unsigned long long *cnt) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool on = e < total && mask[e] != 0.f;
    const int c = __popcll(__ballot(on));
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(cnt, (unsigned long long)c);
}

// column sums of G [n][k] into out [k]; one block per column
__global__ void k_colsum(const float *G, int64_t n, int k, float *out) {
    const int col = blockIdx.x;
    float acc = 0.f;
    for (int64_t r = threadIdx.x; r < n; r += blockDim.x) acc += G[r * k + col];
    __shared__ float part[4];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) out[col] = part[0] + part[1] + part[2] + part[3];
}

// omb1 = 1 - b1 and omb2 = 1 - b2 come from the host in double: 1 - 0.999f in
// fp32 is off by 1.3e-5 relative (0.999 is not a float)
__global__ void k_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1,
                       float omb1, float b2, float omb2, float c1, float c2) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const float gg = g[e];
    const float mm = b1 * m[e] + omb1 * gg;
    const float vv = b2 * v[e] + omb2 * gg * gg;
    m[e] = mm;
    v[e] = vv;
    p[e] -= lr * (mm * c1) / (sqrtf(vv * c2) + 1e-8f);
}

// column mean and 1 / std of X [n][din] (fp64 sums); one block per column
__global__ void k_col_stats(const float *X, int64_t n, int din, float *mu, float *inv_sigma) {
    const int c = blockIdx.x;
    double s = 0.0, s2 = 0.0;
    for (int64_t r = threadIdx.x; r < n; r += blockDim.x) {
        const double x = X[r * din + c];
        s += x;
        s2 += x * x;
    }
    __shared__ double ps[256], ps2[256];
    ps[threadIdx.x] = s;
    ps2[threadIdx.x] = s2;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            ps[threadIdx.x] += ps[threadIdx.x + w];
            ps2[threadIdx.x] += ps2[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double mean = n ? ps[0] / (double)n : 0.0;
        const double var = n ? ps2[0] / (double)n - mean * mean : 0.0;
        mu[c] = (float)mean;
        inv_sigma[c] = var > 1e-12 ? (float)(1.0 / sqrt(var)) : 1.f;
    }
}

__global__ void k_select(const float *logits, int64_t n, int k, const int32_t *budgets, float target,
                         int32_t *budget) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t b = -1;
    for (int j = 0; j < k; ++j) {
        const float r = 1.f / (1.f + expf(-logits[i * k + j]));
        if (r >= target) { b = budgets[j]; break; }
    }
    budget[i] = b;
}

__global__ void k_gather_rows(const float *src, int ld, const int32_t *rows, int64_t n, float *dst) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * ld) return;
    const int64_t r = e / ld;
    dst[e] = src[(int64_t)rows[r] * ld + (e % ld)];
}

__global__ void k_remap(int32_t *v, int64_t n, const int32_t *list) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = list[v[i]];
}

void forward_acts(const Predictor &p, const float *X, int64_t n, Acts &t, hipStream_t s) {
    t.xn.reserve((size_t)n * p.din * sizeof(float));
    t.a1.reserve((size_t)n * p.h1 * sizeof(float));
    t.a2.reserve((size_t)n * p.h2 * sizeof(float));
    t.z3.reserve((size_t)n * p.k * sizeof(float));
    hipLaunchKernelGGL(k_normalize, dim3(g1p(n * p.din, 256)), dim3(256), 0, s, X, n, p.din,
                       p.mu.as<float>(), p.inv_sigma.as<float>(), t.xn.as<float>());
    gemm<false, true>((int)n, p.h1, p.din, t.xn.as<float>(), p.din, p.W1.as<float>(), p.din,
                      t.a1.as<float>(), p.h1, p.b1.as<float>(), true, nullptr, 0, s);
    gemm<false, true>((int)n, p.h2, p.h1, t.a1.as<float>(), p.h1, p.W2.as<float>(), p.h1,
                      t.a2.as<float>(), p.h2, p.b2.as<float>(), true, nullptr, 0, s);
    gemm<false, true>((int)n, p.k, p.h2, t.a2.as<float>(), p.h2, p.W3.as<float>(), p.h2,
                      t.z3.as<float>(), p.k, p.b3.as<float>(), false, nullptr, 0, s);
}

// loss and gradients into g (parameter layout of Predictor::n_params)
double backward(const Predictor &p, const float *X, const float *Y, const float *mask, int64_t n,
                Acts &t, float *g, hipStream_t s) {
    forward_acts(p, X, n, t, s);
    const int64_t tot = n * p.k;
    double cnt = (double)tot;
    t.aux.reserve(16);
    DevBuf &aux = t.aux;
    VJ_HIP(hipMemsetAsync(aux.p, 0, 16, s));
    if (mask) {
        hipLaunchKernelGGL(k_mask_count, dim3(g1p(tot, 256)), dim3(256), 0, s, mask, tot,
                           aux.as<unsigned long long>() + 1);
        unsigned long long c = 0;
        VJ_HIP(hipMemcpyAsync(&c, aux.as<unsigned long long>() + 1, 8, hipMemcpyDeviceToHost, s));
        VJ_HIP(hipStreamSynchronize(s));
        cnt = c ? (double)c : 1.0;
    }
    t.g3.reserve((size_t)tot * sizeof(float));
    t.g2.reserve((size_t)n * p.h2 * sizeof(float));
    t.g1.reserve((size_t)n * p.h1 * sizeof(float));
    DevBuf &g3 = t.g3, &g2 = t.g2, &g1b = t.g1;
    hipLaunchKernelGGL(k_bce, dim3(g1p(tot, 256)), dim3(256), 0, s, t.z3.as<float>(), Y, mask, tot,
                       (float)(1.0 / cnt), g3.as<float>(), aux.as<double>());
    float *gW1 = g, *gb1 = gW1 + (size_t)p.h1 * p.din, *gW2 = gb1 + p.h1,
          *gb2 = gW2 + (size_t)p.h2 * p.h1, *gW3 = gb2 + p.h2, *gb3 = gW3 + (size_t)p.k * p.h2;
    const int N = (int)n;
    // layer 3
    gemm<true, false>(p.k, p.h2, N, g3.as<float>(), p.k, t.a2.as<float>(), p.h2, gW3, p.h2, nullptr,
                      false, nullptr, 0, s);
    hipLaunchKernelGGL(k_colsum, dim3(p.k), dim3(256), 0, s, g3.as<float>(), n, p.k, gb3);
    gemm<false, false>(N, p.h2, p.k, g3.as<float>(), p.k, p.W3.as<float>(), p.h2, g2.as<float>(),
                       p.h2, nullptr, false, t.a2.as<float>(), p.h2, s);
    // layer 2
    gemm<true, false>(p.h2, p.h1, N, g2.as<float>(), p.h2, t.a1.as<float>(), p.h1, gW2, p.h1,
                      nullptr, false, nullptr, 0, s);
    hipLaunchKernelGGL(k_colsum, dim3(p.h2), dim3(256), 0, s, g2.as<float>(), n, p.h2, gb2);
    gemm<false, false>(N, p.h1, p.h2, g2.as<float>(), p.h2, p.W2.as<float>(), p.h1,
                       g1b.as<float>(), p.h1, nullptr, false, t.a1.as<float>(), p.h1, s);
    // layer 1
    gemm<true, false>(p.h1, p.din, N, g1b.as<float>(), p.h1, t.xn.as<float>(), p.din, gW1, p.din,
                      nullptr, false, nullptr, 0, s);
    hipLaunchKernelGGL(k_colsum, dim3(p.h1), dim3(256), 0, s, g1b.as<float>(), n, p.h1, gb1);
    VJ_HIP(hipGetLastError());
    double loss = 0.0;
    VJ_HIP(hipMemcpyAsync(&loss, aux.p, 8, hipMemcpyDeviceToHost, s));
    VJ_HIP(hipStreamSynchronize(s));
    return loss / cnt;
}

}  // namespace

void compute_features(const Index &ix, const int32_t *qlist, int64_t n, float eps, int ld,
                      float *out, hipStream_t s) {
    (void)ld;
    if (n == 0) return;
    hipLaunchKernelGGL(k_features, dim3(g1p(n, 4)), dim3(256), 0, s, ix.vec.as<float>(), ix.dp, ix.d,
                       ix.nx, ix.adj.as<int32_t>(), ix.elen.as<float>(), ix.R, ix.entry,
                       (int)ix.metric, eps, qlist, n, out);
    VJ_HIP(hipGetLastError());
}

void predictor_init(Predictor &p, int din, int h1, int h2, int k, uint64_t seed, hipStream_t s) {
    p.din = din;
    p.h1 = h1;
    p.h2 = h2;
    p.k = k;
    // He-uniform weights, zero biases, from a seeded host generator
    std::mt19937_64 rng(seed);
    auto layer = [&](DevBuf &W, DevBuf &b, int out, int in) {
        std::vector<float> w((size_t)out * in);
        const double lim = std::sqrt(6.0 / in);
        std::uniform_real_distribution<double> u(-lim, lim);
        for (auto &x : w) x = (float)u(rng);
        W.alloc(w.size() * sizeof(float));
        VJ_HIP(hipMemcpyAsync(W.p, w.data(), W.bytes, hipMemcpyHostToDevice, s));
        b.alloc((size_t)out * sizeof(float));
        VJ_HIP(hipMemsetAsync(b.p, 0, b.bytes, s));
        VJ_HIP(hipStreamSynchronize(s));
    };
    layer(p.W1, p.b1, h1, din);
    layer(p.W2, p.b2, h2, h1);
    layer(p.W3, p.b3, k, h2);
    std::vector<float> mu((size_t)din, 0.f), is((size_t)din, 1.f);
    p.mu.alloc(din * sizeof(float));
    p.inv_sigma.alloc(din * sizeof(float));
    VJ_HIP(hipMemcpyAsync(p.mu.p, mu.data(), p.mu.bytes, hipMemcpyHostToDevice, s));
    VJ_HIP(hipMemcpyAsync(p.inv_sigma.p, is.data(), p.inv_sigma.bytes, hipMemcpyHostToDevice, s));
    p.m.alloc(p.n_params() * sizeof(float));
    p.v.alloc(p.n_params() * sizeof(float));
    VJ_HIP(hipMemsetAsync(p.m.p, 0, p.m.bytes, s));
    VJ_HIP(hipMemsetAsync(p.v.p, 0, p.v.bytes, s));
    VJ_HIP(hipStreamSynchronize(s));
    p.steps = 0;
}

void predictor_forward(const Predictor &p, const float *X, int64_t n, float *logits,
                       hipStream_t s) {
    if (n == 0) return;
    Acts &t = p.scratch;
    forward_acts(p, X, n, t, s);
    VJ_HIP(hipMemcpyAsync(logits, t.z3.p, (size_t)n * p.k * sizeof(float), hipMemcpyDeviceToDevice, s));
    VJ_HIP(hipGetLastError());
    VJ_HIP(hipStreamSynchronize(s));
}

double predictor_loss_grad(const Predictor &p, const float *X, const float *Y, const float *mask,
                           int64_t n, float *gW1, float *gb1, float *gW2, float *gb2, float *gW3,
                           float *gb3, hipStream_t s) {
    DevBuf g(p.n_params() * sizeof(float));
    Acts &t = p.scratch;
    const double loss = n ? backward(p, X, Y, mask, n, t, g.as<float>(), s) : 0.0;
    float *dst[6] = {gW1, gb1, gW2, gb2, gW3, gb3};
    const size_t len[6] = {(size_t)p.h1 * p.din, (size_t)p.h1, (size_t)p.h2 * p.h1, (size_t)p.h2,
                           (size_t)p.k * p.h2, (size_t)p.k};
    size_t off = 0;
    for (int i = 0; i < 6; ++i) {
        if (dst[i] && n)
            VJ_HIP(hipMemcpyAsync(dst[i], g.as<float>() + off, len[i] * sizeof(float),
                                  hipMemcpyDeviceToDevice, s));
        off += len[i];
    }
    VJ_HIP(hipStreamSynchronize(s));
    return loss;
}

void predictor_fit_normalization(Predictor &p, const float *X, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_col_stats, dim3(p.din), dim3(256), 0, s, X, n, p.din, p.mu.as<float>(),
                       p.inv_sigma.as<float>());
    VJ_HIP(hipGetLastError());
    VJ_HIP(hipStreamSynchronize(s));
}

void predictor_adam(Predictor &p, const float *g, float lr, hipStream_t s) {
    // parameters are separate buffers; Adam runs per buffer over its slice of
    // g, m and v (all parameters back to back in the order W1 b1 W2 b2 W3 b3)
    DevBuf *par[6] = {&p.W1, &p.b1, &p.W2, &p.b2, &p.W3, &p.b3};
    const double b1 = 0.9, b2 = 0.999;
    p.steps += 1;
    const float c1 = (float)(1.0 / (1.0 - std::pow(b1, (double)p.steps)));
    const float c2 = (float)(1.0 / (1.0 - std::pow(b2, (double)p.steps)));
    size_t off = 0;
    for (int i = 0; i < 6; ++i) {
        const int64_t len = (int64_t)(par[i]->bytes / sizeof(float));
        hipLaunchKernelGGL(k_adam, dim3(g1p(len, 256)), dim3(256), 0, s, par[i]->as<float>(),
                           g + off, p.m.as<float>() + off, p.v.as<float>() + off, len, lr,
                           (float)b1, (float)(1.0 - b1), (float)b2, (float)(1.0 - b2), c1, c2);
        off += (size_t)len;
    }
    VJ_HIP(hipGetLastError());
}

void predictor_train(Predictor &p, const float *X, const float *Y, int64_t n, int epochs,
                     int batch, float lr, uint64_t seed, float *loss_per_epoch, hipStream_t s) {
    if (n == 0 || epochs <= 0) return;
    batch = (int)std::max<int64_t>(1, std::min<int64_t>(batch, n));
    std::mt19937_64 rng(seed);
    std::vector<int32_t> perm((size_t)n);
    std::iota(perm.begin(), perm.end(), 0);
    DevBuf idx((size_t)batch * sizeof(int32_t)), xb((size_t)batch * p.din * sizeof(float)),
        yb((size_t)batch * p.k * sizeof(float)), g(p.n_params() * sizeof(float));
    Acts &t = p.scratch;
    for (int e = 0; e < epochs; ++e) {
        std::shuffle(perm.begin(), perm.end(), rng);
        double sum = 0.0;
        int64_t seen = 0;
        for (int64_t r0 = 0; r0 < n; r0 += batch) {
            const int nb = (int)std::min<int64_t>(batch, n - r0);
            VJ_HIP(hipMemcpyAsync(idx.p, perm.data() + r0, nb * sizeof(int32_t), hipMemcpyHostToDevice, s));
            hipLaunchKernelGGL(k_gather_rows, dim3(g1p((int64_t)nb * p.din, 256)), dim3(256), 0, s, X,
                               p.din, idx.as<int32_t>(), (int64_t)nb, xb.as<float>());
            hipLaunchKernelGGL(k_gather_rows, dim3(g1p((int64_t)nb * p.k, 256)), dim3(256), 0, s, Y,
                               p.k, idx.as<int32_t>(), (int64_t)nb, yb.as<float>());
            const double loss = backward(p, xb.as<float>(), yb.as<float>(), nullptr, nb, t,
                                         g.as<float>(), s);
            sum += loss * nb;
            seen += nb;
            predictor_adam(p, g.as<float>(), lr, s);
        }
        if (loss_per_epoch) loss_per_epoch[e] = (float)(sum / (double)seen);
    }
    VJ_HIP(hipStreamSynchronize(s));
}

void select_budgets(const float *logits, int64_t n, int k, const int32_t *budgets_dev,
                    float target, int32_t *budget, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_select, dim3(g1p(n, 256)), dim3(256), 0, s, logits, n, k, budgets_dev,
                       target, budget);
    VJ_HIP(hipGetLastError());
}

void gather_rows(const float *src, int ld, const int32_t *rows, int64_t n, float *dst,
                 hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_gather_rows, dim3(g1p(n * ld, 256)), dim3(256), 0, s, src, ld, rows, n, dst);
    VJ_HIP(hipGetLastError());
}

void remap_ids(int32_t *v, int64_t n, const int32_t *list, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_remap, dim3(g1p(n, 256)), dim3(256), 0, s, v, n, list);
    VJ_HIP(hipGetLastError());
}

}  // namespace vj
