// Traversal kernels over float rows (see traverse_impl.h).
#include "traverse_impl.h"

namespace vj {
int launch_traverse_f32(const TraverseLaunch &a, bool spill, int max_blocks, int wpb, hipStream_t s) {
    return trav::launch_elem<float>(a, spill, max_blocks, wpb, s);
}
}  // namespace vj
