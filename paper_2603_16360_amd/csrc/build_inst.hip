// One row-width instantiation of the graph-build row kernels (see
// build_rows.h); the build compiles this file once per width VJ_BUILD_DP.
// Defines build_rows_<DP>, build_rev_<DP> and build_gather_<DP>.
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
                                      int32_t *indeg, int64_t rb, int64_t M, hipStream_t s) {
    brow::launch_rows<VJ_BUILD_DP>(vec, N, R, K, Kc, bid, kid, kd2, fwd, fwd_d2, fdeg, indeg, rb,
                                   M, s);
}

void VJ_CAT(build_rev_, VJ_BUILD_DP)(const float *vec, int64_t M, int R, const int32_t *fwd,
                                     const float *fwd_d2, const int32_t *fdeg,
                                     const int64_t *roff, const int32_t *rid,
                                     const float *rd2, int32_t *adj, const int32_t *rows,
                                     hipStream_t s) {
    brow::launch_rev<VJ_BUILD_DP>(vec, M, R, fwd, fwd_d2, fdeg, roff, rid, rd2, adj, rows, s);
}

void VJ_CAT(build_gather_, VJ_BUILD_DP)(const float *vec, int R, const int32_t *adj,
                                        const int32_t *fwd_new, const int32_t *fdeg_new,
                                        int64_t n_old, const int32_t *rows, int64_t M,
                                        int32_t *fwd, float *fwd_d2, int32_t *fdeg,
                                        hipStream_t s) {
    brow::launch_gather<VJ_BUILD_DP>(vec, R, adj, fwd_new, fdeg_new, n_old, rows, M, fwd, fwd_d2,
                                     fdeg, s);
}

}  // namespace vj
