#include "build.h"

namespace vj {
void build_graph(Index &, int, hipStream_t) {
    VJ_CHECK(false, VJ_ERR_UNSUPPORTED, "graph build not available");
}
}  // namespace vj
