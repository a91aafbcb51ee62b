// One row-width instantiation of the graph-build row kernels (see
// build_rows.h); the build compiles this file once per width VJ_BUILD_DP.
// Defines build_rows_<DP> and build_rev_<DP>.
#include "build_rows.h"

#ifndef VJ_BUILD_DP
#error "build with -DVJ_BUILD_DP=<width>"
#endif

#define VJ_CAT2(a, b) a##b
#define VJ_CAT(a, b) VJ_CAT2(a, b)

namespace vj {

void VJ_CAT(build_rows_, VJ_BUILD_DP)(const float *vec, int64_t N, int R, int K, int Kc,
                                      const int32_t *bid, int32_t *kid, float *kd2,
                                      int32_t *fwd, float *fwd_d2, int32_t *fdeg,
                                      int32_t *indeg, hipStream_t s) {
    brow::launch_rows<VJ_BUILD_DP>(vec, N, R, K, Kc, bid, kid, kd2, fwd, fwd_d2, fdeg, indeg, s);
}

void VJ_CAT(build_rev_, VJ_BUILD_DP)(const float *vec, int64_t N, int R, const int32_t *fwd,
                                     const float *fwd_d2, const int32_t *fdeg,
                                     const int64_t *roff, const int32_t *rid,
                                     const float *rd2, int32_t *adj, hipStream_t s) {
    brow::launch_rev<VJ_BUILD_DP>(vec, N, R, fwd, fwd_d2, fdeg, roff, rid, rd2, adj, s);
}

}  // namespace vj
