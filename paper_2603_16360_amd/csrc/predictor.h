// Difficulty predictor: per-query features after the probe, and a small MLP
// (din -> h1 -> h2 -> k, ReLU, k sigmoid heads) that predicts a query's
// recall under k out-range pop budgets (defined in predictor.hip).
#pragma once

#include "vj_internal.h"

namespace vj {

constexpr int kFeatures = 8;  // features after the query vector

// activations and backward scratch of the MLP (kept between calls)
struct Acts {
    DevBuf xn, a1, a2, z3;   // forward activations
    DevBuf g3, g2, g1, aux;  // backward scratch
};

struct Predictor {
    int din = 0, h1 = 0, h2 = 0, k = 0;
    DevBuf W1, b1, W2, b2, W3, b3;  // float, row-major W[out][in]
    DevBuf mu, inv_sigma;           // float [din] input normalisation (x - mu) * inv_sigma
    DevBuf m, v;                    // Adam moments, all parameters back to back
    int64_t steps = 0;
    mutable Acts scratch;             // calls on one predictor must not overlap
    size_t n_params() const {
        return (size_t)h1 * din + h1 + (size_t)h2 * h1 + h2 + (size_t)k * h2 + k;
    }
};

// features [n][dp_q + 8] of the queries qlist[0..n) (indices into Q): the
// query's padded row (d values then zeros up to ld - 8) and f0..f7
void compute_features(const Index &ix, const int32_t *qlist, int64_t n, float eps, int ld,
                      float *out, hipStream_t s);

void predictor_init(Predictor &p, int din, int h1, int h2, int k, uint64_t seed, hipStream_t s);
void predictor_forward(const Predictor &p, const float *X, int64_t n, float *logits,
                       hipStream_t s);
// mean BCE-with-logits over the entries with mask != 0 (mask may be null)
// and the gradients of every parameter (device buffers of the parameters'
// shapes, any may be null); returns the loss
double predictor_loss_grad(const Predictor &p, const float *X, const float *Y, const float *mask,
                           int64_t n, float *gW1, float *gb1, float *gW2, float *gb2, float *gW3,
                           float *gb3, hipStream_t s);
// one Adam step (beta 0.9 / 0.999, eps 1e-8, bias-corrected) with the
// gradient g of every parameter, back to back in the order W1 b1 W2 b2 W3 b3
void predictor_adam(Predictor &p, const float *g, float lr, hipStream_t s);
// Adam over shuffled minibatches; loss_per_epoch (host, may be null)
void predictor_train(Predictor &p, const float *X, const float *Y, int64_t n, int epochs,
                     int batch, float lr, uint64_t seed, float *loss_per_epoch, hipStream_t s);
// predictor files: parameters, normalisation, Adam moments and step count
void predictor_save(const Predictor &p, const char *path);
void predictor_load(Predictor &p, const char *path, hipStream_t s);
// mu / inv_sigma from the columns of X (constant columns get inv_sigma 1)
void predictor_fit_normalization(Predictor &p, const float *X, int64_t n, hipStream_t s);
// budget[i] = budgets[j] for the smallest j whose predicted recall
// sigmoid(logit[i][j]) >= target, else -1 (route to brute force)
void select_budgets(const float *logits, int64_t n, int k, const int32_t *budgets_dev,
                    float target, int32_t *budget, hipStream_t s);
// dst[r][.] = src[rows[r]][.] for rows of ld floats
void gather_rows(const float *src, int ld, const int32_t *rows, int64_t n, float *dst,
                 hipStream_t s);
// v[i] = list[v[i]]
void remap_ids(int32_t *v, int64_t n, const int32_t *list, hipStream_t s);

}  // namespace vj
