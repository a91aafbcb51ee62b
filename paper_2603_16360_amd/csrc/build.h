// Merged-graph construction (defined in build.hip).
#pragma once

#include "vj_internal.h"

namespace vj {

// Build adj / elen / entry of `ix` from its vectors: exact kNN candidates
// (MFMA tiles), RNG prune, reverse edges, entry, connectivity repair.
void build_graph(Index &ix, int kc, hipStream_t s);
void ensure_bf16(Index &ix, hipStream_t s);
void ensure_f8(Index &ix, hipStream_t s);
void compute_mst(Index &ix, hipStream_t s);

}  // namespace vj
