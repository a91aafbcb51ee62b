// MFMA distance tiles (defined in tiles.hip).
#pragma once

#include "vj_internal.h"

namespace vj {

// bf16 copies of a row set, padded to Kp (a multiple of 32), for MFMA tiles
struct TileRows {
    int64_t rows = 0;
    int Kp = 0;
    DevBuf hi, lo;        // bf16 hi / lo parts [rows][Kp] (lo only in split mode)
    DevBuf norm2;         // float [rows] squared norms of the fp32 rows
    float maxabs = 0.f;   // largest |value|
    float maxnorm = 0.f;  // largest row norm
    bool small_int = false;  // every value an integer with |v| <= 256
};

// Device memory for one call's temporaries: fresh allocations (base null),
// or 256-byte aligned slices of a fixed region that is never grown, so a
// call on a region allocates nothing.
struct Arena {
    char *base = nullptr;
    size_t cap = 0, used = 0;
    DevBuf take(size_t bytes) {
        if (!base) return DevBuf(bytes);
        const size_t at = (used + 255) & ~(size_t)255;
        VJ_CHECK(at <= cap && bytes <= cap - at, VJ_ERR_UNSUPPORTED,
                 "the call's temporaries exceed the fixed scratch region");
        used = at + bytes;
        return DevBuf::view(base + at, bytes);
    }
    size_t left() const {
        const size_t at = (used + 255) & ~(size_t)255;
        return at < cap ? cap - at : 0;
    }
};

void prepare_rows(const float *src, int64_t rows, int d, int Kp, bool split, TileRows &t,
                  hipStream_t s, Arena *arena = nullptr);

// Bounds of the tile value's error: |dot~ - dot| <= e_dot |a||b| and the
// remaining fp32 operations add at most e_fin (|a| + |b|)^2 (0 and 0 when the
// tiles are exact).
void tile_error_bounds(const TileRows &a, const TileRows &b, int nsplit, double &e_dot,
                       double &e_fin);

// Exact epsilon-join of Q against X on MFMA tiles with an fp64 re-check of
// every pair whose tile value lies inside the rounding-error bound of eps.
void bruteforce_join(const float *Q, int64_t nq, const float *X, int64_t nx, int d, float eps,
                     vj_metric metric, vj_precision prec, hipStream_t s, Pairs &out);

// Exact nearest row of X for every row of Q by the metric (L2 distance, or
// 1 - <q, x>), ties to the smaller index: tile minima on MFMA, then every
// pair within twice the tiles' proven error bound of its row's minimum
// re-decided in fp64.  w [nq] int32, dist [nq] float64 (device).
void exact_top1(const float *Q, int64_t nq, const float *X, int64_t nx, int d, vj_metric metric,
                int32_t *w, double *dist, hipStream_t s);

// The same join with every temporary in the library's fixed device scratch
// region (kNoAllocScratchBytes per device; no allocation of any kind) and
// the pairs written to the caller's qx [cap][2] (query, data) and dist
// [cap] (may be null), in no particular order.  Returns the number of pairs
// (if it exceeds cap, cap of them were written).
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
int64_t bruteforce_join_noalloc(const float *Q, int64_t nq, const float *X, int64_t nx, int d,
                                float eps, vj_metric metric, vj_precision prec, int32_t *qx,
                                float *dist, int64_t cap, hipStream_t s);

}  // namespace vj
