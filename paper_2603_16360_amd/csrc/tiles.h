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

void prepare_rows(const float *src, int64_t rows, int d, int Kp, bool split, TileRows &t,
                  hipStream_t s);

// Bounds of the tile value's error: |dot~ - dot| <= e_dot |a||b| and the
// remaining fp32 operations add at most e_fin (|a| + |b|)^2 (0 and 0 when the
// tiles are exact).
void tile_error_bounds(const TileRows &a, const TileRows &b, int nsplit, double &e_dot,
                       double &e_fin);

// Exact epsilon-join of Q against X on MFMA tiles with an fp64 re-check of
// every pair whose tile value lies inside the rounding-error bound of eps.
void bruteforce_join(const float *Q, int64_t nq, const float *X, int64_t nx, int d, float eps,
                     vj_metric metric, vj_precision prec, hipStream_t s, Pairs &out);

}  // namespace vj
