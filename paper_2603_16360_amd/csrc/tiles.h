// MFMA distance tiles (defined in tiles.hip).
#pragma once

#include "vj_internal.h"

namespace vj {

// Exact epsilon-join of Q against X on MFMA tiles with an fp64 re-check of
// every pair whose tile value lies inside the rounding-error bound of eps.
void bruteforce_join(const float *Q, int64_t nq, const float *X, int64_t nx, int d, float eps,
                     vj_metric metric, vj_precision prec, hipStream_t s, Pairs &out);

}  // namespace vj
