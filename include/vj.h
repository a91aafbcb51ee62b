/*
 * vj.h -- C ABI of the MI355X merged-index vector-join library (libvj.so).
 *
 * Problem (paper, Definition 1): given a query set Q, a data set X, a
 * distance dist and a threshold eps, the vector join is the set of pairs
 * (q, x) with dist(q, x) < eps.  The approximate join of the paper (Section
 * 4) indexes Q and X together in ONE proximity graph (the merged index,
 * Section 4.3) and answers every query by probing its own neighbourhood and
 * expanding in-range neighbours (Algorithms 1-8).
 *
 * Conventions for every call:
 *  - Array arguments are DEVICE pointers (HIP device memory of the current
 *    device, e.g. torch CUDA tensors) unless the name ends in _host.
 *    Vectors are float32, row-major [rows][d].
 *  - `stream` is a hipStream_t (NULL = the default stream).  Work is queued
 *    on it; calls that must return a size to the host (the pair count)
 *    synchronise that stream before returning.
 *  - Node ids of an index: data rows are 0..nx-1, query rows nx..nx+nq-1.
 *    Pairs are reported as (query index 0..nq-1, data index 0..nx-1).
 *  - Metrics: VJ_L2 is the unsquared Euclidean distance ||q - x||;
 *    VJ_IP is 1 - <q, x>.  The predicate is strict: dist < eps.
 *  - Errors: every call returns a vj_status; on error nothing is written to
 *    the outputs and vj_last_error() (per thread) describes the failure.
 *    No C++ exception crosses this boundary.
 *  - Ownership: objects returned through vj_index ** / vj_pairs ** belong
 *    to the caller and are released with vj_index_free / vj_pairs_free.
 *    Indexes copy their inputs; the caller may free them on return.
 *  - Every call works on the device that is current on the calling thread.
 */
#ifndef VJ_H
#define VJ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    VJ_OK = 0,
    VJ_ERR_INVALID_ARG = 1,     /* null pointer, negative size, d <= 0, eps NaN, ids out of range */
    VJ_ERR_METRIC_MISMATCH = 2, /* join metric differs from the index metric */
    VJ_ERR_OOM = 3,             /* device allocation failed */
    VJ_ERR_HIP = 4,             /* a HIP runtime call failed */
    VJ_ERR_INTERNAL = 5,        /* a kernel reported an inconsistency */
    VJ_ERR_UNSUPPORTED = 6,     /* shape outside the supported range (see each call) */
    VJ_ERR_IO = 7               /* a file could not be written or read, or is not a valid file */
} vj_status;

typedef enum { VJ_L2 = 0, VJ_IP = 1 } vj_metric;

/* Work-sharing mode (cfg.work_sharing, Algorithms 3 and 8). */
typedef enum {
    VJ_WS_SELF = 0, /* seeds {s, q}: the merged-index default (MI) */
    VJ_WS_SOFT = 1, /* + the parent query's closest visited data node (SWS) */
    VJ_WS_HARD = 2, /* + every in-range node the parent found (HWS) */
    VJ_WS_NNMAP = 3 /* separate indexes with an NN-Map (Section 6, vj_build_nnmap): a query
                       whose nearest data node lies at dist >= eps is certified empty,
                       otherwise that node is the only seed and the greedy phase is
                       skipped; VJ_HYB_ADAPT takes the map's OOD bit */
} vj_work_sharing;

/* Expansion mode (cfg.force_hybrid / cfg.adapt_hybrid, Algorithms 6-7). */
typedef enum {
    VJ_HYB_OFF = 0,    /* BFS over in-range data nodes only */
    VJ_HYB_FORCE = 1,  /* hybrid search for every query */
    VJ_HYB_ADAPT = 2,  /* hybrid only for queries predicted OOD (d1/d2 > ratio) */
    VJ_HYB_BUDGET = 3, /* hybrid with a per-query cap on out-range pops (budget[]) */
    VJ_HYB_LEARNED = 4 /* budgets chosen by the index's attached predictor; queries no
                          budget satisfies are joined exactly on MFMA tiles */
} vj_hybrid;

/* Arithmetic of the distance evaluations. */
typedef enum {
    VJ_PREC_FP32 = 0, /* fp32 inputs, fp32 accumulation */
    VJ_PREC_BF16 = 1, /* bf16 rows, fp32 query and accumulation; a candidate within the
                         proven error margin of eps is re-decided from the fp32 rows in the
                         fp32 kernels' arithmetic, so in/out decisions equal VJ_PREC_FP32's
                         (join: workgroup tiers only) */
    VJ_PREC_FP8 = 2,  /* OCP e4m3 rows with a power-of-two scale per row and a stored
                         bound on |x - x~| (fp64, rounded up); fp32 query and accumulation; a
                         candidate within that margin of eps (triangle inequality) is
                         re-decided from the fp32 rows in the fp32 kernels' arithmetic, so
                         in/out decisions equal VJ_PREC_FP32's (join: workgroup tiers only) */
    VJ_PREC_U8 = 3,   /* exact u8 copy (integer data in [0, 255] only) */
    VJ_PREC_AUTO = 4  /* u8 if the index data is exactly u8, else fp32 */
} vj_precision;

typedef struct vj_index vj_index;
typedef struct vj_pairs vj_pairs;
typedef struct vj_predictor vj_predictor;

typedef struct {
    int32_t R;           /* max out-degree, 1..64 */
    int32_t K_cand;      /* exact-kNN candidates per node before pruning, <= 112 (0: min(2R, 112)) */
    int32_t build_mst;   /* 1: compute the query MST (needed for SOFT/HARD) */
    int32_t copies;      /* low-precision copies made at build (else on first use): 1 bf16,
                            2 fp8; exact u8 rows are made whenever the data allows them */
} vj_build_params;

typedef struct {
    int32_t work_sharing;   /* vj_work_sharing */
    int32_t hybrid;         /* vj_hybrid */
    int32_t hybrid_beam;    /* bound on the out-range queue (default 256) */
    int32_t conv_threshold; /* stop after this many unproductive out-range pops (10; <=0: none) */
    float ood_ratio;        /* d1/d2 threshold of VJ_HYB_ADAPT (1.5) */
    int32_t precision;      /* vj_precision */
    const int32_t *budget;  /* device [n]: out-range pops allowed (VJ_HYB_BUDGET); <0: brute force */
    int32_t start_tier;     /* first storage tier of every query (1): 0 one wave per query,
                               1 one workgroup per query, 2 one workgroup per query with its
                               tables in global memory; a query
                               that outgrows a tier re-runs on the next.  Callers that know
                               their queries are large (high eps) skip the small tiers. */
    int32_t coop_tables;    /* LDS tables of the workgroup tier (0): 0 large (8192 visited
                               slots, 768 pairs), 1 small (4096 slots, 1024 pairs); both
                               run 4 workgroups per CU; same results either way */
    int64_t pair_capacity;  /* initial result capacity hint (0: auto) */
    int32_t dense_first;    /* self mode (1): launch queries in ascending order of d1, the mean
                               stored length of their edges to data nodes -- dense
                               neighbourhoods, whose joins run longest, start first, which
                               shortens the tail of uneven query costs; 0: the given order.
                               Results are the same either way.  Merged indexes only. */
    int32_t greedy_beam;    /* separate indexes: bound on the best-first greedy queue
                               (cfg.greedy_beam_size, default 256, at most 256) */
    int32_t persistent;     /* 0 (default, and the only value accepted at present: others
                               return VJ_ERR_UNSUPPORTED): one workgroup per query, one launch
                               per MST level in SOFT / HARD mode.  1 would run the workgroup
                               tier as ONE launch of resident workgroups claiming queries in
                               processing order, children waiting on the device for their MST
                               parent; it is switched off while a GPU fault seen with it is
                               investigated. */
    int32_t layer_seeds;    /* separate indexes with upper layers (vj_index_build_layers): 1
                               seeds each query's greedy phase with the node its greedy
                               descent through the layers reaches, in place of the data
                               graph's entry; 0 (default): the entry */
} vj_join_params;

void vj_default_build_params(vj_build_params *p);
void vj_default_join_params(vj_join_params *p);

/*
 * Build the merged index over Q and X (Section 4.3: one graph over both
 * sets, per-node set label = id < nx).  Q: [nq][d], X: [nx][d] float32.
 * Graph: exact kNN candidates (MFMA tiles) -> RNG edge rule (Appendix C) ->
 * reverse edges -> entry nearest the centroid -> connectivity repair ->
 * edge lengths -> query MST (Section 3.2).  The graph is always built on L2
 * geometry; `metric` is the metric joins must use (for VJ_IP the rows
 * should be unit-norm, where L2 and IP orders coincide).
 * Limits: 1 <= d <= 1024, nq + nx < 2^30, 1 <= R <= 64 (VJ_ERR_UNSUPPORTED).
 * With the environment variable VJ_LOG set, the build (and an insertion's
 * kNN sweep) prints its progress on stderr, synchronising the stream at each
 * step; builds over millions of nodes take tens of seconds.
 */
vj_status vj_build_merged_index(const float *Q, int64_t nq, const float *X, int64_t nx,
                                int32_t d, vj_metric metric, const vj_build_params *p,
                                void *stream, vj_index **out);

/*
 * Wrap a graph built elsewhere (the paper treats the index as a black box,
 * e.g. NSG or HNSW) as a merged index.  adj: [nq+nx][R] int32 node ids,
 * -1 padded; entry: entry node id.  parent: [nq] MST parent node ids (-1 =
 * the entry is the parent) or NULL to compute the MST here.  Edge lengths
 * are computed here.  Same limits as vj_build_merged_index.
 */
vj_status vj_index_from_graph(const float *Q, int64_t nq, const float *X, int64_t nx,
                              int32_t d, vj_metric metric, const int32_t *adj, int32_t R,
                              int32_t entry, const int32_t *parent, void *stream,
                              vj_index **out);

/*
 * Separate indexes (cfg.merged = false, Section 2.2 and Algorithms 1-8):
 * the data graph G_X over X alone and the query graph G_Q over Q alone,
 * each built by the merged build's recipe over its own set.  Joins on such
 * an index seed each query with the entry of G_X (plus the parent's cache
 * under SOFT / HARD work sharing; VJ_WS_SELF means no sharing, the INLJ of
 * Section 2.2), run the best-first greedy phase of Algorithms 4-5 (queue
 * bound greedy_beam, stop rules 1 and 2 with conv_threshold), then the same
 * expansion as the merged index.  The query MST (SOFT / HARD order) uses the
 * edges of G_Q plus an (entry, q) edge per query, rooted at the entry.
 * VJ_HYB_ADAPT behaves as VJ_HYB_OFF there (Algorithm 6: the OOD test needs
 * the merged index); VJ_HYB_LEARNED, vj_join_features and the device batch
 * runner are refused.  Stats column 4 holds the greedy pops.  The graph is
 * exported as for a merged index: rows 0..nx-1 = G_X (data ids), rows
 * nx.. = G_Q (query node ids nx + j).
 */
vj_status vj_build_separate_index(const float *Q, int64_t nq, const float *X, int64_t nx,
                                  int32_t d, vj_metric metric, const vj_build_params *p,
                                  void *stream, vj_index **out);
/* Separate indexes around graphs built elsewhere: adj [nq + nx][R] in the
 * layout above (a data row may hold only data ids, a query row only query
 * node ids; VJ_ERR_INVALID_ARG otherwise); entry: a data node. */
vj_status vj_index_from_separate_graphs(const float *Q, int64_t nq, const float *X, int64_t nx,
                                        int32_t d, vj_metric metric, const int32_t *adj,
                                        int32_t R, int32_t entry, const int32_t *parent,
                                        void *stream, vj_index **out);

/*
 * Incremental insertion of a query batch into a merged index (Section 4.3:
 * updating a merged graph needs only the set label of each node, and the
 * graph's own update rules apply).  Q: device fp32 [n][d] row-major (d of
 * the index), copied; the new queries get query indexes nq_old .. nq_old+n-1
 * (node ids nx + nq_old + i); existing ids do not change.  The update:
 * exact K_cand nearest neighbours of each new node among all nodes (ties by
 * smaller id), RNG prune to R; each kept edge (u, v) is offered to v as a
 * reverse edge; every node that receives offers takes its current row (a
 * new node: its pruned list) plus the offers, whole if they fit in R, else
 * RNG-pruned; rows without offers do not change; then the build's
 * connectivity repair from the (unchanged) entry.  K_cand <= 0: min(2R,
 * 112), the build's default.  The index's MST, if it has one, and its
 * low-precision copies are recomputed.  n == 0 is a no-op.  Separate
 * indexes: VJ_ERR_UNSUPPORTED.  Must not overlap a join on the same index.
 * On an error after the argument checks the index keeps its old graph.
 */
vj_status vj_index_insert_queries(vj_index *idx, const float *Q, int64_t n, int32_t K_cand,
                                  void *stream);

/*
 * Query-data role switch of a merged index (Appendix E: the join is
 * symmetric, and for large thresholds iterating over the larger set while
 * traversing the smaller set's part of the graph avoids most random
 * accesses).  The new index has the same graph and vectors with the roles
 * exchanged: its queries are the old data rows (query index j = old data
 * index j) and its data are the old queries (data index i = old query index
 * i); node ids are relabelled (data first), the entry follows its node.  A
 * join on it returns pairs (old data index, old query index): the
 * role-switched join, to be read transposed.  build_mst != 0 computes the
 * MST of the new query set (needed only for SOFT / HARD).  Merged indexes
 * only (VJ_ERR_INVALID_ARG otherwise).
 */
vj_status vj_index_swap_roles(const vj_index *idx, int32_t build_mst, void *stream,
                              vj_index **out);

/*
 * NN-Map (Section 6): for every query of a separate index its nearest data
 * node w (exact by the index metric: MFMA tile minima, then every candidate
 * within twice the tiles' proven error bound re-decided in fp64; ties to the
 * smaller id), that distance (fp64) and an OOD bit.  Reading of the OOD bit:
 * the d1/d2 rule of Section 4.4 with the witness as the only neighbour, d1 =
 * |q - w| and d2 = the mean L2 length of w's edges to data nodes in the data
 * graph; OOD iff d1 / d2 > ood_ratio (1.5).  Joins with VJ_WS_NNMAP use it.
 */
vj_status vj_build_nnmap(vj_index *idx, float ood_ratio, void *stream);
/* Copy the map out: w [nq] int32, dist [nq] float64, ood [nq] uint8 (device;
 * any may be NULL). */
vj_status vj_index_export_nnmap(const vj_index *idx, int32_t *w, double *dist, uint8_t *ood,
                                void *stream);

/* Copy the graph out: adj [N][R] int32, elen [N][R] float32 (either may be
 * NULL), parent [nq] int32 (may be NULL; -1 = entry).  Device pointers. */
vj_status vj_index_export_graph(const vj_index *idx, int32_t *adj, float *elen,
                                int32_t *parent, void *stream);

/* Scalar facts of an index (any pointer may be NULL). */
vj_status vj_index_info(const vj_index *idx, int64_t *nq, int64_t *nx, int32_t *d,
                        int32_t *R, int32_t *entry, int32_t *metric);

/*
 * Work counters of the index's last build or insertion (any pointer may be
 * NULL).  The kNN sweep (Section 4.3's graph, built here by exact kNN on
 * MFMA tiles) groups the nodes around centres and sweeps, per block of rows,
 * first the tiles of the block's own groups, then only the groups a
 * triangle-inequality bound cannot rule out; tiles_first and tiles_second
 * count those (row blocks x column tiles), tiles_all what a sweep of all
 * pairs would take (all three 0 where the sweep for rows wider than 256
 * floats ran).  repairs: connectivity-repair edges; repairs_listed: repair
 * steps answered from the unreachable node's own kNN list (which the index
 * keeps from its build and insertions), with at most a scan of the nodes
 * added since that list was made instead of all nodes.  Host pointers.
 */
vj_status vj_index_build_stats(const vj_index *idx, int64_t *tiles_first, int64_t *tiles_second,
                               int64_t *tiles_all, int64_t *repairs, int64_t *repairs_listed);

void vj_index_free(vj_index *idx);

/*
 * Index files.  The paper builds the merged index once, offline, and reuses
 * it for every later join and threshold (Section 4.3); a file keeps it
 * across processes.  vj_index_save writes the vectors (padded fp32 rows),
 * the graph, its edge lengths, the entry node and the query MST to `path`
 * (host string; the file is overwritten) and synchronises the device.
 * vj_index_load reads such a file into a new index on the current device
 * (exact low-precision copies and the join state are rebuilt there); joins
 * on it give the same results as on the saved index.  A missing,
 * truncated or corrupt file (checked by a hash of its bytes) returns
 * VJ_ERR_IO.  An attached predictor is not part of the index file.
 */
vj_status vj_index_save(const vj_index *idx, const char *path);
vj_status vj_index_load(const char *path, void *stream, vj_index **out);

/*
 * The merged-index join (Algorithm 1 with cfg.merged = true) of the queries
 * query_ids[0..n) (indices into Q; NULL = all nq queries in order) at
 * threshold eps.  In SOFT/HARD mode queries are processed parents-first
 * along the MST; a query whose MST parent is not in this call gets no
 * cached seed.  eps <= 0 (L2) returns an empty result.  By default
 * (start_tier = 1) each query runs on one workgroup of four waves with its
 * visited set, in-range list and out-range queue in LDS (8192 visited slots
 * and 768 pairs, or 4096 and 1024 with coop_tables = 1); start_tier = 0
 * starts every query on one wavefront (1024 slots, 512 pairs, four queries
 * per workgroup).  A query that outgrows its tier re-runs on the next: one
 * workgroup on tables in global memory (2^16 slots and 32768 pairs: within
 * the same launch while the index's regions last, else in a re-run
 * launch), then on tables as large as the data set.  Calls on one index
 * must not overlap (they share the index's per-query cache).
 * Limits: hybrid_beam <= 256.
 */
vj_status vj_join(vj_index *idx, const int32_t *query_ids, int64_t n, float eps,
                  vj_metric metric, const vj_join_params *p, void *stream,
                  vj_pairs **out);

/*
 * Exact nested-loop join (the NLJ of Section 2.2) on MFMA tiles: every
 * pair with dist < eps.  Distances are evaluated in bf16 (one term, or a
 * three-term hi/lo split for prec = VJ_PREC_FP32) with fp32 accumulation;
 * every pair whose tile value lies within a proven error bound of eps is
 * re-decided from the fp32 inputs in fp64, so the result equals the exact
 * fp64 decision.  Limits: 1 <= d <= 1024.
 */
vj_status vj_bruteforce_join(const float *Q, int64_t nq, const float *X, int64_t nx,
                             int32_t d, float eps, vj_metric metric, vj_precision prec,
                             void *stream, vj_pairs **out);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture of the surrounding work, tight serving loops, harnesses that
 * forbid hipMalloc): vj_bruteforce_join with no allocation of any kind.
 * Its temporaries (bf16 tile rows and norms of Q and X, thresholds,
 * candidate pairs, counters) live in one fixed device region of 64 MiB per
 * device, held by the library until the process ends; the pairs go to the
 * caller's qx [cap][2] int32 (query index, data index) and dist [cap]
 * float32 (may be NULL), in no particular order.  *count_host receives the
 * number of pairs; if it exceeds cap only cap of them were written (which
 * ones is unspecified) and the call must be repeated with a larger buffer.
 * Inputs whose temporaries do not fit (about (nq + nx) * (4 Kp + 4) bytes
 * for VJ_PREC_FP32, Kp = d rounded up to 32, plus 8 bytes per candidate
 * pair) return VJ_ERR_UNSUPPORTED.  The call synchronises `stream`.
 * Calls that overlap on one device race on the region: serialise them.
 */
vj_status vj_bruteforce_join_noalloc(const float *Q, int64_t nq, const float *X, int64_t nx,
                                     int32_t d, float eps, vj_metric metric, vj_precision prec,
                                     int32_t *qx, float *dist, int64_t cap, int64_t *count_host,
                                     void *stream);

/*
 * Batches (a stream of joins on one index): batch b joins the queries
 * query_ids[start[b] .. start[b] + count[b]) (indices into Q; query_ids NULL:
 * the ids start[b] .. start[b] + count[b] - 1 themselves) at eps_host[b],
 * with the parameters p, one after the other on `stream`, reusing the
 * index's join buffers.  out[n_batches] receives the results (on error none
 * is kept); batch_ms_host[b] (may be NULL) the wall time of batch b, from
 * its submission to its result being complete.
 */
vj_status vj_join_batches(vj_index *idx, const int32_t *query_ids, const int64_t *batch_start_host,
                          const int64_t *batch_count_host, const float *eps_host,
                          int32_t n_batches, vj_metric metric, const vj_join_params *p,
                          void *stream, vj_pairs **out, float *batch_ms_host);

/* How vj_join_batches_device submits its batch steps. */
typedef enum {
    VJ_SUBMIT_DIRECT = 0, /* each step's kernels launched on the slot streams */
    VJ_SUBMIT_GRAPH = 1   /* steps captured as HIP graphs (16 steps each) and replayed */
} vj_submit;

/*
 * Batches driven from the device: the same arguments and results as
 * vj_join_batches, but with no host synchronisation between batches.  The
 * batch descriptors (range, eps) sit in device memory and each batch step
 * reads its own; a query that outgrows the workgroup tier's tables is
 * re-run within the step on global tables, then on tables as large as the
 * data set, from counts kept on the device.  Two slots with their own
 * state and stream take the even and the odd batches, so one batch's tail
 * overlaps the next batch's start.  submit chooses direct launches or HIP
 * graph replay (the graphs are kept in the index for the next call of the
 * same shape).
 * Differences from vj_join_batches: self mode only (work_sharing =
 * VJ_WS_SELF) and hybrid OFF, FORCE or ADAPT; dense_first orders each batch
 * by buckets of d1 (4,096 buckets, about 6 % wide) instead of a sort;
 * start_tier is not used (the workgroup tier runs first); batch_ms_host[b] is
 * the device time of batch b (device wall clock at its first and last
 * kernel), not the wall time.  The results of one call share one device
 * allocation, freed with the last of them.  Pair sets are those of vj_join
 * on the same queries.  Calls on one index must not overlap.
 */
vj_status vj_join_batches_device(vj_index *idx, const int32_t *query_ids,
                                 const int64_t *batch_start_host, const int64_t *batch_count_host,
                                 const float *eps_host, int32_t n_batches, vj_metric metric,
                                 const vj_join_params *p, vj_submit submit, void *stream,
                                 vj_pairs **out, float *batch_ms_host);

/*
 * Autotuning: time vj_join on the sample query_ids[0..n) at eps for each
 * candidate launch configuration (first storage tier 0 or 1; large or small
 * workgroup-tier tables; fp32 rows, or
 * exact u8 rows when the index data allows them -- every candidate gives
 * the same decisions) and write the fastest into *p, keeping its other
 * fields.  best_ms_host (may be NULL): the device time of the pick.
 */
vj_status vj_autotune_join(vj_index *idx, const int32_t *query_ids, int64_t n, float eps,
                           vj_metric metric, vj_join_params *p, float *best_ms_host, void *stream);

/* Number of pairs held by a result. */
int64_t vj_pairs_count(const vj_pairs *r);

/* Write the pairs: qx [count][2] int32 (query index, data index), dist
 * [count] float32 (may be NULL).  sorted != 0 orders by (query, data). */
vj_status vj_pairs_export(const vj_pairs *r, int32_t *qx, float *dist, int sorted,
                          void *stream);

/* Per-query counters of a vj_join result, [n][8] int32 in the order of
 * query_ids: pairs, distance evaluations, expanded nodes, out-range pops,
 * predicted OOD, hybrid used, distinct data nodes visited, flags
 * (bit 0: ran on the workgroup tier, bit 1: routed to brute force, bit 3:
 * finished on global tables, bit 4: finished in a separate re-run launch). */
vj_status vj_pairs_stats(const vj_pairs *r, int32_t *stats, void *stream);

/* Device time of a vj_join result's traversal launches, measured with HIP
 * events recorded on the call's stream around them: kernel_ms for the
 * small-LDS-tier launches, spill_ms for the re-runs of queries that outgrew
 * that tier, n_spilled the number of such queries.  Any pointer may be NULL. */
vj_status vj_pairs_timing(const vj_pairs *r, float *kernel_ms, float *spill_ms,
                          int64_t *n_spilled);

/* Candidates whose low-precision value fell inside the proven error margin
 * of eps and were re-decided at full precision: from the fp32 rows, in the
 * fp32 kernels' arithmetic (vj_join with VJ_PREC_BF16), or in fp64
 * (vj_bruteforce_join). */
vj_status vj_pairs_rechecked(const vj_pairs *r, int64_t *n);

/* Per-tier breakdown of a vj_join result's traversal, for the storage tiers
 * 0 (one wave per query, LDS), 1 (one workgroup per query, LDS), 2 (one
 * workgroup per query, global tables of 2^16 slots) and 3 (the same with
 * tables as large as the data set): ms[t] the device time of the tier's launches (HIP events on the
 * call's stream), launches[t] their number and queries[t] the queries
 * launched on the tier, re-runs included.  Arrays of 4; any may be NULL. */
vj_status vj_pairs_tiers(const vj_pairs *r, float *ms, int32_t *launches, int64_t *queries);

void vj_pairs_free(vj_pairs *r);

/* ---------------------------------------------------------------------------
 * Difficulty predictor (VJ_HYB_LEARNED).  The paper's OOD test (Section 4.4)
 * predicts, from d1/d2 after the probe, whether a query needs hybrid
 * search.  The learned form extends that signal: an MLP over the query
 * vector and 8 post-probe features predicts the query's recall under k
 * out-range pop budgets; the join gives each query the smallest budget whose
 * predicted recall reaches a target and joins the rest exactly.
 * ------------------------------------------------------------------------- */

/* Features of the queries query_ids[0..n) (NULL = all, n == nq): row i,
 * [d + 8] float32, is the query vector then f0..f7 = eps, dist(q, s),
 * min over A of dist(q, y), d1, d2, d1 / d2, |A| / R, |{y in A: dist < eps}| / R
 * with A = the data nodes among N(q), dist the join metric, d1 (mean |q - y|
 * over A) and d2 (mean edge length |y - z|, z a data neighbour of y other
 * than q) in L2 units; A-based values are 0 when A is empty. */
vj_status vj_join_features(vj_index *idx, const int32_t *query_ids, int64_t n, float eps,
                           vj_metric metric, float *features, void *stream);

/* An MLP din -> h1 -> h2 -> k (ReLU hidden layers, k logits, sigmoid
 * heads), He-uniform weights from `seed`, zero biases, identity input
 * normalisation.  Weights are row-major W[out][in]; the input is normalised
 * as (x - mu) * inv_sigma per column before the first layer. */
vj_status vj_predictor_create(int32_t din, int32_t h1, int32_t h2, int32_t k, uint64_t seed,
                              void *stream, vj_predictor **out);
void vj_predictor_free(vj_predictor *p);
/* Copy parameters in / out (device pointers of the shapes above; NULL
 * skips that parameter). */
vj_status vj_predictor_set_params(vj_predictor *p, const float *W1, const float *b1,
                                  const float *W2, const float *b2, const float *W3,
                                  const float *b3, const float *mu, const float *inv_sigma,
                                  void *stream);
vj_status vj_predictor_get_params(const vj_predictor *p, float *W1, float *b1, float *W2,
                                  float *b2, float *W3, float *b3, float *mu, float *inv_sigma,
                                  void *stream);
/* mu / inv_sigma from the columns of X [n][din] (constant columns: 1). */
vj_status vj_predictor_fit_normalization(vj_predictor *p, const float *X, int64_t n, void *stream);
/* logits [n][k] of X [n][din]. */
vj_status vj_predictor_forward(const vj_predictor *p, const float *X, int64_t n, float *logits,
                               void *stream);
/* Mean binary cross-entropy of sigmoid(logits) against Y [n][k] in [0, 1]
 * over the entries with mask != 0 (mask NULL: all), into *loss (host), and
 * its gradient for each parameter (device, parameter shapes; NULL skips). */
vj_status vj_predictor_loss_grad(const vj_predictor *p, const float *X, const float *Y,
                                 const float *mask, int64_t n, double *loss, float *gW1,
                                 float *gb1, float *gW2, float *gb2, float *gW3, float *gb3,
                                 void *stream);
/* Adam (beta 0.9 / 0.999) on the mean BCE over minibatches of `batch` rows
 * of a seeded shuffle, for `epochs` passes; the mean loss of each epoch goes
 * to loss_per_epoch_host (may be NULL). */
vj_status vj_predictor_train(vj_predictor *p, const float *X, const float *Y, int64_t n,
                             int32_t epochs, int32_t batch, float lr, uint64_t seed,
                             float *loss_per_epoch_host, void *stream);
/* One Adam step (Kingma and Ba 2015, Algorithm 1: beta 0.9 / 0.999, eps
 * 1e-8 outside the square root, bias-corrected moments; the step counter is
 * the predictor's, shared with vj_predictor_train) with the caller's
 * gradient: grad, device, n_params floats = every parameter back to back in
 * the order W1 b1 W2 b2 W3 b3 (the shapes above), with n_params = h1*din +
 * h1 + h2*h1 + h2 + k*h2 + k. */
vj_status vj_predictor_adam_step(vj_predictor *p, const float *grad, float lr, void *stream);
/* The optimizer state: first and second moments (device, n_params floats
 * each, layout of vj_predictor_adam_step's grad; either may be NULL) and the
 * number of steps taken (host, may be NULL). */
vj_status vj_predictor_get_adam_state(const vj_predictor *p, float *m, float *v, int64_t *steps,
                                      void *stream);
/* Layer widths of a predictor (host; any pointer may be NULL). */
vj_status vj_predictor_info(const vj_predictor *p, int32_t *din, int32_t *h1, int32_t *h2,
                            int32_t *k);
/* Predictor files (host path string): parameters, input normalisation, the
 * optimizer's moments and step count, so training can resume.  Errors as
 * for vj_index_save / vj_index_load. */
vj_status vj_predictor_save(const vj_predictor *p, const char *path);
vj_status vj_predictor_load(const char *path, void *stream, vj_predictor **out);
/* Attach a predictor to an index for VJ_HYB_LEARNED joins (NULL detaches):
 * head j predicts the recall under budgets_host[j] out-range pops (k values,
 * ascending, >= 0).  The predictor must outlive its use by the index. */
vj_status vj_index_attach_predictor(vj_index *idx, const vj_predictor *p, float recall_target,
                                    const int32_t *budgets_host);

/*
 * HNSW-style upper layers over the data nodes of an index (the paper
 * evaluates the method on HNSW as well as NSG, Section 5; the index is a
 * black box to the join).  Data node v gets level L(v) = the number of
 * trailing zero 4-bit digits of output v + 1 of SplitMix64 seeded with
 * `seed`, capped at max_levels (1..16), so P(L >= l) = 16^-l and the layers
 * are nested.  Layer l (l >= 1) holds the nodes with L >= l and its graph is
 * this library's build recipe (exact kNN, RNG prune to R, reverse edges,
 * connectivity repair, entry nearest to the centroid) over those nodes
 * alone; layers stop before the first with fewer than two nodes.  Replaces
 * any layers the index had.  A separate-index join with
 * vj_join_params.layer_seeds = 1 seeds each query's greedy phase with the
 * node a greedy descent reaches: from the top layer's entry, repeatedly
 * move to the neighbour in that layer smallest by (dist(q, .), id) while it
 * is smaller than the current node, then continue one layer down; the node
 * reached in layer 1 is the seed.  Layers are not stored by vj_index_save.
 * R in [1, 64].  Errors: VJ_ERR_INVALID_ARG (null index, R or max_levels
 * out of range).
 */
vj_status vj_index_build_layers(vj_index *idx, int32_t R, uint64_t seed, int32_t max_levels,
                                void *stream);
/* Number of layers and their out-degree R (host int32, R may be NULL) and,
 * for each layer (layer 1 first), its node count and entry (host arrays of
 * at least *n_layers entries, or NULL). */
vj_status vj_index_layers_info(const vj_index *idx, int32_t *n_layers, int32_t *R,
                               int64_t *counts, int32_t *entries);
/* Layer `layer` (1-based): its data ids, ascending ([count] int32, device)
 * and its adjacency ([count][R] int32 data ids, -1 padded, device). */
vj_status vj_index_export_layer(const vj_index *idx, int32_t layer, int32_t *ids, int32_t *adj,
                                void *stream);
/* The descent's seed of each listed query (query_ids: device [n] query
 * indexes, NULL = all; seeds: device [n] data ids; moves: device [n] or
 * NULL, the number of moves).  Errors: VJ_ERR_INVALID_ARG (no layers). */
vj_status vj_index_descend(vj_index *idx, const int32_t *query_ids, int64_t n, int32_t *seeds,
                           int32_t *moves, void *stream);

/* Text of the last error on the calling thread ("" if none). */
const char *vj_last_error(void);

/*
 * Device memory kept by the library: a freed temporary of 16 MB or more is
 * not returned to the runtime but kept for a later request of between half
 * its size and its size (the device is synchronised first, as hipFree
 * would), at most 32 GB per device; such blocks are allocated rounded up to
 * an eighth of their power of two (at most 12.5 % more), and a failed
 * allocation empties the device's cache and retries.  vj_trim_memory returns every kept block of the current
 * device to the runtime.  bytes_freed (host, may be NULL): the bytes
 * returned.
 */
vj_status vj_trim_memory(int64_t *bytes_freed);

/*
 * Hardware-counter calibration (not part of the method): out[i] = the sum
 * of row ids[i] of rows, for i < n.  rows: [nrows][dp] fp32 on the device,
 * dp a positive multiple of 32; ids: [n] int32 (an id outside [0, nrows)
 * gives 0); out: [n] fp32.  A row is read exactly as the join reads one
 * (8 lanes, 16 bytes per lane per load, whole 128-byte lines per load), so
 * with n distinct ids over a set far larger than the caches the kernel
 * moves n * dp * 4 bytes of rows plus 8 n bytes of ids and output; the
 * memory counters' reading for it calibrates theirs for the join's gathers.
 * Errors: VJ_ERR_INVALID_ARG (n or nrows < 0, dp not a positive multiple of
 * 32, a null pointer with n > 0).
 */
vj_status vj_calib_gather(const float *rows, int64_t nrows, int32_t dp, const int32_t *ids,
                          int64_t n, float *out, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* VJ_H */
