#include "tiles.h"

namespace vj {
void bruteforce_join(const float *, int64_t, const float *, int64_t, int, float, vj_metric,
                     vj_precision, hipStream_t, Pairs &) {
    VJ_CHECK(false, VJ_ERR_UNSUPPORTED, "brute force not available");
}
}  // namespace vj
