// Traversal kernels over uint16_t rows (see traverse_impl.h).
#include "traverse_impl.h"

namespace vj {
int launch_traverse_bf16(const TraverseLaunch &a, bool spill, int max_blocks, int wpb, hipStream_t s) {
    return trav::launch_elem<uint16_t>(a, spill, max_blocks, wpb, s);
}
}  // namespace vj
