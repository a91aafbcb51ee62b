// Device helpers defined in util.hip.
#pragma once

#include "vj_internal.h"

namespace vj {

void launch_dist_to_node(const float *vec, int dp, int64_t first, int64_t n, int32_t node,
                         float *out, hipStream_t s);
void fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);
void iota_i32(int32_t *p, int64_t n, hipStream_t s);
void stamp_batch(int32_t *inb, int64_t nq, const int32_t *ids, int64_t n, int32_t gen,
                 int32_t *err, hipStream_t s);
void gather_slots(const int32_t *qlist, const int32_t *qpos, const int32_t *slots, int64_t n,
                  int32_t *q2, int32_t *p2, hipStream_t s);
// self mode: slots ordered by d1 of the query (mean edge length to its data
// neighbours) ascending -- densest neighbourhoods, the longest queries,
// first; the buffers are caller-owned scratch
void order_by_density(const int32_t *adj, const float *elen, int R, int64_t nx, int64_t nq,
                      const int32_t *ids, int64_t n, int32_t *qlist, int32_t *qpos, DevBuf &keys,
                      DevBuf &keys2, DevBuf &pos, DevBuf &tmp, hipStream_t s);
void order_by_depth(const int32_t *depth, int64_t nq, const int32_t *ids, int64_t n,
                    int32_t *qlist, int32_t *qpos, DevBuf &tmp, hipStream_t s);

}  // namespace vj
