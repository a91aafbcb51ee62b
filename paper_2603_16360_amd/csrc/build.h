// Merged-graph construction (defined in build.hip).
#pragma once

#include "vj_internal.h"

namespace vj {

// Build adj / elen / entry of `ix` from its vectors: exact kNN candidates
// (MFMA tiles), RNG prune, reverse edges, entry, connectivity repair.
void build_graph(Index &ix, int kc, hipStream_t s);
// Insert rows [n_old, ix.N) of ix.vec as new nodes into the graph of rows
// [0, n_old) (ix.adj and ix.elen hold N rows, the old ones filled): exact kNN
// of the new nodes among all nodes, forward RNG prune, the new nodes' edges
// offered as reverse edges, every row that receives offers re-pruned over
// its current row plus the offers (kept whole if they fit in R), then the
// connectivity repair from the unchanged entry and the lengths of the rows
// that changed.
void insert_graph(Index &ix, int64_t n_old, int kc, hipStream_t s);
void ensure_bf16(Index &ix, hipStream_t s);
void ensure_f8(Index &ix, hipStream_t s);
void compute_mst(Index &ix, hipStream_t s);

}  // namespace vj
