// Device helpers defined in util.hip.
#pragma once

#include "vj_internal.h"

namespace vj {

void launch_dist_to_node(const float *vec, int dp, int64_t first, int64_t n, int32_t node,
                         float *out, hipStream_t s);
void fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);
// upper layers: row gather, local -> data ids, positions, greedy descent
// (see k_descend)
void gather_rows_f32(const float *src, int dp, const int32_t *ids, int64_t n, float *dst,
                     hipStream_t s);
void map_ids(int32_t *adj, int64_t n, const int32_t *ids, hipStream_t s);
void scatter_pos(int32_t *pos, const int32_t *ids, int64_t n, hipStream_t s);
void descend(const float *vec, int dp, int64_t nx, int metric, int nl, const int64_t *loff,
             const int64_t *lcnt, const int32_t *lpos, const int32_t *ladj, int R, int32_t top,
             const int32_t *qids, int64_t n, int32_t *seed_i, int32_t *seed_q, int32_t *moves,
             int32_t *err, hipStream_t s);
// counter calibration gather (the join's row-read layout); see vj_calib_gather
void calib_gather(const float *rows, int64_t nrows, int dp, const int32_t *ids, int64_t n,
                  float *out, hipStream_t s);
void iota_i32(int32_t *p, int64_t n, hipStream_t s);
// NN-Map OOD bits of the queries from their witnesses w (see k_nn_ood)
void nn_ood(const float *vec, int dp, int64_t nx, int64_t nq, const int32_t *adj, int R,
            const int32_t *w, double ratio, uint8_t *ood, hipStream_t s);
// role switch of a merged index's node ids (data v -> nq + v, query v -> v - nx)
void swap_ids(int32_t *p, int64_t n, int32_t nx, int32_t nq, hipStream_t s);
// p[i] += off for every id >= 0 (-1 padding stays)
void offset_ids(int32_t *p, int64_t n, int32_t off, hipStream_t s);
void stamp_batch(int32_t *inb, int64_t nq, const int32_t *ids, int64_t n, int32_t gen,
                 int32_t *err, hipStream_t s);
void gather_slots(const int32_t *qlist, const int32_t *qpos, const int32_t *slots, int64_t n,
                  int32_t *q2, int32_t *p2, hipStream_t s);

// Batch steps replayed from captured graphs: the batch descriptors sit in
// device memory and a cursor in the join counters selects the batch.
struct BatchDesc {
    const int32_t *ids;  // id list of the batch (null: the ids start, start + 1, ...)
    int32_t *stats;      // the batch's rows of per-query counters
    int64_t start;       // first entry of the batch in the id list
    int32_t count;       // queries (0: the batch runs nothing)
    float eps, eps2;
    int32_t pad;
};
// join counters the batch steps use beyond those of a single join
constexpr int kBatchCount = 5;    // slots of the current batch (first launch)
constexpr int kBatchOvf2 = 8;     // queries left for the full-size tables
constexpr int kBatchOvf3 = 9;     // queries no table held (must stay 0)
constexpr int kBatchCursor = 10;  // batch the next step runs
// per batch record: pairs before and after it, queries re-run on global
// tables and on full-size tables, bf16 re-checks before and after it, device
// wall clock at its start and end
constexpr int kBatchRec = 8;
constexpr int kOrderBuckets = 4096;
// the step's first kernel: set-up, the batch's query list, and (bucket
// non-null) the d1 bucket of each query counted in hist
void batch_start(const BatchDesc *desc, JoinArgs *args, int32_t *ctr, uint64_t *rec, int64_t nmax,
                 const int32_t *adj, const float *elen, int R, int64_t nx, int64_t nq,
                 int32_t *qlist, int32_t *bucket, uint32_t *hist, hipStream_t s);
// densest neighbourhoods first (4,096 d1 buckets): q2 / p2 get the ids of
// qlist and their positions; hist is zero again on return
void batch_order(const int32_t *qlist, const int32_t *ctr, int64_t nmax, const int32_t *bucket,
                 uint32_t *hist, uint32_t *off, int32_t *q2, int32_t *p2, hipStream_t s);
void batch_end(int32_t *ctr, uint64_t *rec, hipStream_t s);

// self mode: slots ordered by d1 of the query (mean edge length to its data
// neighbours) ascending, in 4,096 buckets about 6 % wide -- densest
// neighbourhoods, the longest queries, first; keys and tmp are caller-owned
// scratch
void order_by_density(const int32_t *adj, const float *elen, int R, int64_t nx, int64_t nq,
                      const int32_t *ids, int64_t n, int32_t *qlist, int32_t *qpos, DevBuf &keys,
                      DevBuf &tmp, hipStream_t s);
// stable radix sort of (key, value) int32 pairs on key bits [0, end_bit);
// keys must be non-negative; tmp is grown as needed
void sort_pairs_i32(const int32_t *keys_in, int32_t *keys_out, const int32_t *vals_in,
                    int32_t *vals_out, int64_t n, int end_bit, DevBuf &tmp, hipStream_t s);
void order_by_depth(const int32_t *depth, int64_t nq, const int32_t *ids, int64_t n,
                    int32_t *qlist, int32_t *qpos, DevBuf &tmp, hipStream_t s);
// out[i] = in[0] + ... + in[i - 1] for i = 0 .. n (n + 1 entries; out[n] is
// the total); tmp is grown as needed
void exclusive_scan_i32_i64(const int32_t *in, int64_t *out, int64_t n, DevBuf &tmp,
                            hipStream_t s);

}  // namespace vj
