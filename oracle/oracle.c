/*
 * Plain, slow FP64 CPU oracle for the merged-index epsilon-join.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may call, link or
 * load this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code, header or table with the HIP
 * library.
 *
 * Every distance is computed in double precision from the float inputs.
 * Each function names the passage of the paper it follows:
 *   - Definition 1 (vector join):      or_nlj, or_pooled_kth
 *   - Section 4.3 + Appendix C (RNG):  or_knn, or_rng_prune, or_build_merged
 *   - Section 3.2 (work sharing, MST): or_mst_parents
 *   - Algorithms 1-8:                  or_join
 *   - Section 5, varying index type (HNSW-style upper layers):
 *                                      or_splitmix64, or_levels, or_descend
 *   - difficulty MLP (not in the paper; fp64 reference):
 *                                      or_features, or_mlp_forward,
 *                                      or_mlp_bce_backward, or_adam_step
 *
 * Readings of points the paper leaves open are marked "reading:".
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_L2 0
#define OR_IP 1

/* dist(a,b): L2 is the unsquared Euclidean distance; IP is 1 - <a,b>
 * (reading: the paper only defines dist abstractly in Definition 1). */
static double dist64(const float *a, const float *b, int d, int metric)
{
    double s = 0.0;
    if (metric == OR_L2) {
        for (int k = 0; k < d; ++k) {
            double t = (double)a[k] - (double)b[k];
            s += t * t;
        }
        return sqrt(s);
    }
    for (int k = 0; k < d; ++k)
        s += (double)a[k] * (double)b[k];
    return 1.0 - s;
}

static double l2_64(const float *a, const float *b, int d)
{
    return dist64(a, b, d, OR_L2);
}

/* ------------------------------------------------------------------------
 * O1: exact nested-loop join, Definition 1: all (i, j) with dist < eps.
 * Emits pairs in (i, j) order.  Returns the total count; writes at most cap.
 * ---------------------------------------------------------------------- */
int64_t or_nlj(const float *Q, int64_t nq, const float *X, int64_t nx, int d,
               int metric, double eps, int64_t cap, int32_t *oq, int32_t *ox,
               double *od)
{
    int64_t cnt = 0;
    for (int64_t i = 0; i < nq; ++i) {
        for (int64_t j = 0; j < nx; ++j) {
            double t = dist64(Q + i * d, X + j * d, d, metric);
            if (t < eps) {
                if (cnt < cap) {
                    oq[cnt] = (int32_t)i;
                    ox[cnt] = (int32_t)j;
                    od[cnt] = t;
                }
                ++cnt;
            }
        }
    }
    return cnt;
}

/* Per-query match counts of the exact join (same predicate as or_nlj). */
void or_nlj_counts(const float *Q, int64_t nq, const float *X, int64_t nx,
                   int d, int metric, double eps, int64_t *counts)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < nq; ++i) {
        int64_t c = 0;
        for (int64_t j = 0; j < nx; ++j)
            if (dist64(Q + i * d, X + j * d, d, metric) < eps)
                ++c;
        counts[i] = c;
    }
}

/* Exact distances of a list of (q, x) pairs. */
void or_pair_dists(const float *Q, const float *X, int d, int metric,
                   int64_t n, const int32_t *pq, const int32_t *px, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        out[i] = dist64(Q + (int64_t)pq[i] * d, X + (int64_t)px[i] * d, d, metric);
}

/* Dense distance matrix (small inputs only). */
void or_dist_matrix(const float *A, int64_t na, const float *B, int64_t nb,
                    int d, int metric, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < na; ++i)
        for (int64_t j = 0; j < nb; ++j)
            out[i * nb + j] = dist64(A + i * d, B + j * d, d, metric);
}

/* ---- max-heap on doubles (for the per-query M smallest) ---------------- */
static void heap_sift_down(double *h, int64_t n, int64_t i)
{
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, m = i;
        if (l < n && h[l] > h[m]) m = l;
        if (r < n && h[r] > h[m]) m = r;
        if (m == i) return;
        double t = h[i]; h[i] = h[m]; h[m] = t;
        i = m;
    }
}

static void heap_push_bounded(double *h, int64_t *n, int64_t cap, double v)
{
    if (*n < cap) {
        int64_t i = (*n)++;
        h[i] = v;
        while (i > 0) {
            int64_t p = (i - 1) / 2;
            if (h[p] >= h[i]) break;
            double t = h[p]; h[p] = h[i]; h[i] = t;
            i = p;
        }
    } else if (v < h[0]) {
        h[0] = v;
        heap_sift_down(h, *n, 0);
    }
}

static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* k-th and (k+1)-th smallest pooled distance over all (q, x) pairs of a
 * query sample (1-based k).  Used to calibrate eps for a target mean match
 * count.  Each query keeps its M smallest distances; if some query's M-th
 * smallest is <= the pooled (k+1)-th value the cap was too small and the
 * function returns 1 (the caller retries with a larger M). */
int or_pooled_kth(const float *Q, int64_t nq, const float *X, int64_t nx, int d,
                  int metric, int64_t k, int64_t M, double *vk, double *vk1)
{
    double *pool = (double *)malloc(sizeof(double) * (size_t)(nq * M));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)nq);
    double *top = (double *)malloc(sizeof(double) * (size_t)nq);
    if (!pool || !fill || !top) { free(pool); free(fill); free(top); return 2; }
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < nq; ++i) {
        double *h = pool + i * M;
        int64_t n = 0;
        for (int64_t j = 0; j < nx; ++j)
            heap_push_bounded(h, &n, M, dist64(Q + i * d, X + j * d, d, metric));
        fill[i] = n;
        top[i] = n ? h[0] : INFINITY;
        for (int64_t t = n; t < M; ++t) h[t] = INFINITY;
    }
    qsort(pool, (size_t)(nq * M), sizeof(double), cmp_double);
    *vk = pool[k - 1];
    *vk1 = pool[k];
    int bad = 0;
    for (int64_t i = 0; i < nq; ++i)
        if (fill[i] == M && top[i] <= *vk1) bad = 1;
    free(pool); free(fill); free(top);
    return bad;
}

/* ------------------------------------------------------------------------
 * O2: deterministic merged-graph build.  The paper treats the graph index as
 * a black box (NSG, max degree 70) and does not specify it; this build uses
 * exact kNN candidates + the RNG edge rule of Appendix C (keep v unless an
 * already-kept w is closer to v than u is), reverse edges, an entry point
 * nearest to the centroid and a connectivity repair.  Ties: smaller id.
 * ---------------------------------------------------------------------- */

/* (d, id) lexicographic "less than" */
static int lt_pair(double da, int32_t ia, double db, int32_t ib)
{
    return da < db || (da == db && ia < ib);
}

/* Exact K nearest neighbours of every node (self excluded), by L2. */
void or_knn(const float *V, int64_t n, int d, int K, int32_t *ids, double *dd)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t u = 0; u < n; ++u) {
        int32_t *ri = ids + u * K;
        double *rd = dd + u * K;
        int cnt = 0;
        for (int64_t v = 0; v < n; ++v) {
            if (v == u) continue;
            double t = l2_64(V + u * d, V + v * d, d);
            if (cnt == K && !lt_pair(t, (int32_t)v, rd[K - 1], ri[K - 1]))
                continue;
            int p = cnt < K ? cnt++ : K - 1;
            while (p > 0 && lt_pair(t, (int32_t)v, rd[p - 1], ri[p - 1])) {
                rd[p] = rd[p - 1];
                ri[p] = ri[p - 1];
                --p;
            }
            rd[p] = t;
            ri[p] = (int32_t)v;
        }
        for (int p = cnt; p < K; ++p) { ri[p] = -1; rd[p] = INFINITY; }
    }
}

/* RNG prune of node u over candidates sorted by (dist, id).  Keeps v unless a
 * previously kept w satisfies dist(w, v) < dist(u, v); stops at R kept.
 * Returns the number kept; out receives the kept ids in scan order. */
int or_rng_prune(const float *V, int d, int64_t u, const int32_t *cand,
                 const double *cd, int m, int R, int32_t *out)
{
    (void)u;
    int kept = 0;
    for (int i = 0; i < m && kept < R; ++i) {
        int32_t v = cand[i];
        if (v < 0) continue;
        int ok = 1;
        for (int j = 0; j < kept && ok; ++j)
            if (l2_64(V + (int64_t)out[j] * d, V + (int64_t)v * d, d) < cd[i])
                ok = 0;
        if (ok) out[kept++] = v;
    }
    return kept;
}

typedef struct { double d; int32_t id; } or_cand;

static int cmp_cand(const void *a, const void *b)
{
    const or_cand *x = (const or_cand *)a, *y = (const or_cand *)b;
    if (x->d < y->d) return -1;
    if (x->d > y->d) return 1;
    return (x->id > y->id) - (x->id < y->id);
}

static void bfs_reach(const int32_t *adj, int64_t n, int R, int32_t s, uint8_t *reach,
                      int32_t *queue)
{
    memset(reach, 0, (size_t)n);
    int64_t h = 0, t = 0;
    reach[s] = 1;
    queue[t++] = s;
    while (h < t) {
        int32_t u = queue[h++];
        for (int j = 0; j < R; ++j) {
            int32_t v = adj[(int64_t)u * R + j];
            if (v >= 0 && !reach[v]) { reach[v] = 1; queue[t++] = v; }
        }
    }
}

static int row_degree(const int32_t *row, int R)
{
    int c = 0;
    while (c < R && row[c] >= 0) ++c;
    return c;
}

/* Re-sort one adjacency row by (dist to owner, id). */
static void sort_row(const float *V, int d, int64_t u, int32_t *row, int R)
{
    or_cand tmp[1024];
    int m = row_degree(row, R);
    for (int j = 0; j < m; ++j) {
        tmp[j].id = row[j];
        tmp[j].d = l2_64(V + u * d, V + (int64_t)row[j] * d, d);
    }
    qsort(tmp, (size_t)m, sizeof(or_cand), cmp_cand);
    for (int j = 0; j < m; ++j) row[j] = tmp[j].id;
}

/* Full merged-graph build over V = [X; Q] (n = nx + nq rows).
 * adj: [n][R], -1 padded, rows sorted by (dist, id).  elen: [n][R] lengths.
 * Returns the number of connectivity-repair edges added. */
int64_t or_build_merged(const float *V, int64_t n, int d, int R, int Kc,
                        int32_t *adj, double *elen, int32_t *entry)
{
    int32_t *knn = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n * Kc));
    double *kd = (double *)malloc(sizeof(double) * (size_t)(n * Kc));
    int32_t *fwd = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n * R));
    int *fdeg = (int *)calloc((size_t)n, sizeof(int));
    or_knn(V, n, d, Kc, knn, kd);

    /* step 3: forward RNG prune of each node's kNN list */
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t u = 0; u < n; ++u)
        fdeg[u] = or_rng_prune(V, d, u, knn + u * Kc, kd + u * Kc, Kc, R, fwd + u * R);

    /* step 4 (reading: batched): cand(v) = fwd(v) + {u : v in fwd(u)};
     * if |cand(v)| <= R keep all, else RNG-prune cand(v) to R. */
    int64_t *rcnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t u = 0; u < n; ++u)
        for (int j = 0; j < fdeg[u]; ++j) rcnt[fwd[u * R + j] + 1]++;
    for (int64_t v = 0; v < n; ++v) rcnt[v + 1] += rcnt[v];
    int32_t *rev = (int32_t *)malloc(sizeof(int32_t) * (size_t)(rcnt[n] + 1));
    int64_t *rpos = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t v = 0; v < n; ++v) rpos[v] = rcnt[v];
    for (int64_t u = 0; u < n; ++u)
        for (int j = 0; j < fdeg[u]; ++j) rev[rpos[fwd[u * R + j]]++] = (int32_t)u;

#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t v = 0; v < n; ++v) {
        int64_t m0 = fdeg[v] + (rcnt[v + 1] - rcnt[v]);
        or_cand *c = (or_cand *)malloc(sizeof(or_cand) * (size_t)(m0 + 1));
        int m = 0;
        for (int j = 0; j < fdeg[v]; ++j) c[m++].id = fwd[v * R + j];
        for (int64_t t = rcnt[v]; t < rcnt[v + 1]; ++t) {
            int32_t u = rev[t];
            int dup = 0;
            for (int j = 0; j < m; ++j) if (c[j].id == u) { dup = 1; break; }
            if (!dup) c[m++].id = u;
        }
        for (int j = 0; j < m; ++j)
            c[j].d = l2_64(V + v * d, V + (int64_t)c[j].id * d, d);
        qsort(c, (size_t)m, sizeof(or_cand), cmp_cand);
        int32_t *row = adj + v * R;
        for (int j = 0; j < R; ++j) row[j] = -1;
        if (m <= R) {
            for (int j = 0; j < m; ++j) row[j] = c[j].id;
        } else {
            int32_t *ci = (int32_t *)malloc(sizeof(int32_t) * (size_t)m);
            double *cdd = (double *)malloc(sizeof(double) * (size_t)m);
            for (int j = 0; j < m; ++j) { ci[j] = c[j].id; cdd[j] = c[j].d; }
            or_rng_prune(V, d, v, ci, cdd, m, R, row);
            free(ci); free(cdd);
        }
        free(c);
    }

    /* step 5: entry = node nearest to the fp64 centroid */
    double *cen = (double *)calloc((size_t)d, sizeof(double));
    for (int64_t u = 0; u < n; ++u)
        for (int k = 0; k < d; ++k) cen[k] += (double)V[u * d + k];
    for (int k = 0; k < d; ++k) cen[k] /= (double)n;
    int32_t s = 0;
    double best = INFINITY;
    for (int64_t u = 0; u < n; ++u) {
        double acc = 0.0;
        for (int k = 0; k < d; ++k) {
            double t = (double)V[u * d + k] - cen[k];
            acc += t * t;
        }
        if (acc < best) { best = acc; s = (int32_t)u; }
    }
    *entry = s;

    /* step 6: connectivity repair from s */
    uint8_t *reach = (uint8_t *)malloc((size_t)n);
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int64_t added = 0;
    for (;;) {
        bfs_reach(adj, n, R, s, reach, queue);
        int64_t w = -1;
        for (int64_t u = 0; u < n; ++u) if (!reach[u]) { w = u; break; }
        if (w < 0) break;
        int64_t pf = -1, pa = -1;
        double df = INFINITY, da = INFINITY;
        for (int64_t p = 0; p < n; ++p) {
            if (!reach[p]) continue;
            double t = l2_64(V + p * d, V + w * d, d);
            if (lt_pair(t, (int32_t)p, da, (int32_t)pa)) { da = t; pa = p; }
            if (row_degree(adj + p * R, R) < R && lt_pair(t, (int32_t)p, df, (int32_t)pf)) {
                df = t; pf = p;
            }
        }
        if (pf >= 0) {
            int32_t *row = adj + pf * R;
            row[row_degree(row, R)] = (int32_t)w;
            sort_row(V, d, pf, row, R);
        } else {
            /* no reachable node has a free slot: overwrite the longest edge
             * (largest (dist, id)) of the nearest reachable node; rows are
             * sorted, so that is the last slot */
            int32_t *row = adj + pa * R;
            row[R - 1] = (int32_t)w;
            sort_row(V, d, pa, row, R);
        }
        ++added;
    }

    /* step 7: edge lengths */
    for (int64_t u = 0; u < n; ++u)
        for (int j = 0; j < R; ++j) {
            int32_t v = adj[u * R + j];
            elen[u * R + j] = v >= 0 ? l2_64(V + u * d, V + (int64_t)v * d, d) : INFINITY;
        }

    free(knn); free(kd); free(fwd); free(fdeg); free(rcnt); free(rev); free(rpos);
    free(cen); free(reach); free(queue);
    return added;
}

/* ------------------------------------------------------------------------
 * MST over the query nodes, rooted at the entry s (Section 3.2, the
 * work-sharing paragraph: query-graph edges plus an (s, q) edge for every
 * query; s is the root).  In the merged index the query graph is the set of
 * G edges whose both ends are query nodes (reading).  Kruskal with ties on
 * (w, min id, max id).  parent[qi] = node id of the parent, -1 if it is s.
 * order receives the query indices in BFS order from s (parents first).
 * Returns the total tree weight.
 * ---------------------------------------------------------------------- */
typedef struct { double w; int32_t a, b; } or_edge;

static int cmp_edge(const void *x, const void *y)
{
    const or_edge *e = (const or_edge *)x, *f = (const or_edge *)y;
    if (e->w < f->w) return -1;
    if (e->w > f->w) return 1;
    if (e->a != f->a) return (e->a > f->a) - (e->a < f->a);
    return (e->b > f->b) - (e->b < f->b);
}

static int32_t uf_find(int32_t *p, int32_t x)
{
    while (p[x] != x) { p[x] = p[p[x]]; x = p[x]; }
    return x;
}

double or_mst_parents(const float *V, int64_t nx, int64_t nq, int d,
                      const int32_t *adj, int R, int32_t s, int32_t *parent,
                      int32_t *order)
{
    int64_t n = nx + nq;
    /* local vertex ids: 0 = s (if s is a data node) or s's query index;
     * we use node ids and a map node->local */
    int64_t cap = nq * (int64_t)(R + 1) + 1;
    or_edge *E = (or_edge *)malloc(sizeof(or_edge) * (size_t)cap);
    int64_t m = 0;
    for (int64_t qi = 0; qi < nq; ++qi) {
        int32_t u = (int32_t)(nx + qi);
        for (int j = 0; j < R; ++j) {
            int32_t v = adj[(int64_t)u * R + j];
            if (v < nx) continue; /* -1 or a data node */
            if (v == u) continue;
            int32_t a = u < v ? u : v, b = u < v ? v : u;
            E[m].w = l2_64(V + (int64_t)a * d, V + (int64_t)b * d, d);
            E[m].a = a; E[m].b = b; ++m;
        }
        if (u != s) {
            int32_t a = u < s ? u : s, b = u < s ? s : u;
            E[m].w = l2_64(V + (int64_t)a * d, V + (int64_t)b * d, d);
            E[m].a = a; E[m].b = b; ++m;
        }
    }
    qsort(E, (size_t)m, sizeof(or_edge), cmp_edge);
    int32_t *uf = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) uf[i] = (int32_t)i;
    /* tree adjacency (each query node has <= its degree in tree) */
    int32_t *ta = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * (nq + 1)));
    int32_t *tb = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * (nq + 1)));
    int64_t te = 0;
    double total = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        int32_t ra = uf_find(uf, E[i].a), rb = uf_find(uf, E[i].b);
        if (ra == rb) continue;
        if (ra < rb) uf[rb] = ra; else uf[ra] = rb;
        total += E[i].w;
        ta[te] = E[i].a; tb[te] = E[i].b; ++te;
    }
    /* root at s: BFS over tree edges */
    int64_t *deg = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t i = 0; i < te; ++i) { deg[ta[i] + 1]++; deg[tb[i] + 1]++; }
    for (int64_t i = 0; i < n; ++i) deg[i + 1] += deg[i];
    int32_t *nb = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * te + 1));
    int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) pos[i] = deg[i];
    for (int64_t i = 0; i < te; ++i) { nb[pos[ta[i]]++] = tb[i]; nb[pos[tb[i]]++] = ta[i]; }
    uint8_t *seen = (uint8_t *)calloc((size_t)n, 1);
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nq + 2));
    int64_t h = 0, t = 0, no = 0;
    for (int64_t qi = 0; qi < nq; ++qi) parent[qi] = -1;
    queue[t++] = s; seen[s] = 1;
    while (h < t) {
        int32_t u = queue[h++];
        if (u >= nx) order[no++] = u - (int32_t)nx;
        /* children in ascending node id for a deterministic order */
        int64_t lo = deg[u], hi = deg[u + 1];
        int32_t *kids = nb + lo;
        int64_t nk = hi - lo;
        for (int64_t a = 1; a < nk; ++a) {
            int32_t key = kids[a]; int64_t b = a - 1;
            while (b >= 0 && kids[b] > key) { kids[b + 1] = kids[b]; --b; }
            kids[b + 1] = key;
        }
        for (int64_t k = 0; k < nk; ++k) {
            int32_t v = kids[k];
            if (seen[v]) continue;
            seen[v] = 1;
            parent[v - nx] = (u == s) ? -1 : u;
            queue[t++] = v;
        }
    }
    free(E); free(uf); free(ta); free(tb); free(deg); free(nb); free(pos);
    free(seen); free(queue);
    return total;
}

/* ------------------------------------------------------------------------
 * O3: the join of Algorithm 1 with Algorithms 3-8, for cfg.merged = true (one
 * graph over X and Q) and for cfg.merged = false (separate indexes: adj rows
 * 0..nx-1 are the data graph G_X with entry s, rows nx.. the query graph,
 * read only by the MST).  Readings (documented with the design):
 *   - seeds are {s, q} plus the parent's cache in soft/hard mode (q is always
 *     a seed on the merged index, so the probe of N(q) always runs);
 *   - the greedy phase on the merged index pops q (distance 0, first) and
 *     stops: stop rule 3 fires once the front is no longer q;
 *   - the initial in-range set counts data nodes only;
 *   - expansion skips query nodes without marking them visited;
 *   - in-range nodes form a worklist that is processed to closure before any
 *     out-range node is popped (a min-queue keyed on distance pops every
 *     in-range node before any out-range one); out-range nodes go to a heap
 *     bounded to hybrid_beam entries, dropping the largest (dist, id);
 *   - hybrid stops after conv_threshold consecutive heap pops that added no
 *     in-range node (<= 0: no stop rule), or after budget[i] heap pops in
 *     the per-query budget mode;
 *   - OOD test d1/d2 > ratio with d1 = mean dist(q, y), y in N(q) cap X,
 *     d2 = mean dist(y, z), z in N(y) cap X, z != q; N(q) cap X empty =>
 *     OOD; no (y, z) pair => not OOD.  Distances in L2 units; for the inner
 *     product metric d1 uses sqrt(2 (1 - <q, y>)).
 * Separate indexes (cfg.merged = 0):
 *   - seeds are {s} plus the parent's cache (q is not a node of G_X);
 *   - the greedy phase is best-first search over a queue initialised with
 *     the seeds, keyed by (dist, id): before each pop, stop if the front is
 *     in range (rule 1) or if the front distance has not fallen below the
 *     smallest front distance seen for conv_threshold consecutive checks
 *     (rule 2; <= 0: no rule 2); pop the front, visit its unvisited
 *     neighbours (into the queue, and into I when in range), then trim the
 *     queue to its greedy_beam smallest entries (trimmed nodes stay
 *     visited);
 *   - CheckHybrid is force_hybrid (adapt needs the merged index);
 *   - the expansion starts from I with the visited set of the greedy
 *     phase, as in the merged case.
 *   Stats column 4 (OOD in the merged case) counts the greedy pops.
 * NN-Map (Section 6; work_sharing = 3, separate indexes, arrays nn_w, nn_d,
 * nn_ood from or_nnmap): if nn_d[q] >= eps the result is empty without a
 * distance evaluation (the witness certificate); otherwise the seed is the
 * witness nn_w[q] alone, the greedy phase is skipped, and adapt mode takes
 * the stored OOD bit as CheckHybrid's prediction.
 * ---------------------------------------------------------------------- */
typedef struct {
    int32_t work_sharing;     /* 0 self, 1 soft, 2 hard */
    int32_t hybrid;           /* 0 off, 1 force, 2 adapt, 3 per-query budget */
    int32_t hybrid_beam;      /* bound on out-range heap entries */
    int32_t conv_threshold;   /* unproductive heap pops before stopping */
    double ood_ratio;         /* 1.5 */
    int32_t uncertain_policy; /* 0 plain, 1 band counts as out, 2 as in */
    double uncertain_rel;     /* band half-width relative to eps */
    uint64_t shuffle_seed;    /* 0: FIFO worklist; else random pops */
    double fragile_rel;       /* relative gap under which an order is fragile */
    int32_t merged;           /* cfg.merged: 1 merged index, 0 separate indexes */
    int32_t greedy_beam;      /* cfg.greedy_beam_size (separate indexes) */
} or_cfg;

enum { ST_PAIRS, ST_NDIST, ST_NEXP, ST_HPOPS, ST_OOD, ST_HYB, ST_VDATA, ST_FRAGILE, ST_N };

typedef struct {
    double d;
    int32_t id;
} hent;

static uint64_t lcg_next(uint64_t *s)
{
    *s = *s * 6364136223846793005ULL + 1442695040888963407ULL;
    return *s >> 33;
}

int64_t or_join(const float *V, int64_t nx, int64_t nq, int d, int metric,
                const int32_t *adj, int R, int32_t s, const int32_t *parent,
                const int32_t *qidx, int64_t n, double eps, const or_cfg *cfg,
                const int32_t *budget, const int32_t *nn_w, const double *nn_d,
                const uint8_t *nn_ood, const int32_t *qseed, int64_t cap, int32_t *oq, int32_t *ox,
                double *od, int32_t *stats)
{
    int64_t N = nx + nq;
    int64_t *stamp = (int64_t *)malloc(sizeof(int64_t) * (size_t)N);
    double *dq = (double *)malloc(sizeof(double) * (size_t)N);
    int32_t *I = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    int32_t *W = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    int hcap = cfg->hybrid_beam > 0 ? cfg->hybrid_beam : 0;
    hent *H = (hent *)malloc(sizeof(hent) * (size_t)(hcap + 2));
    /* greedy queue of the separate-index mode: <= beam + R entries after a
     * pop, or every seed before the first */
    hent *G = (hent *)malloc(sizeof(hent) * (size_t)(N + cfg->greedy_beam + R + 4));
    /* cache: soft -> one node id per query; hard -> a list per query */
    int32_t *soft = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nq + 1));
    int64_t *hoff = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nq + 1));
    int64_t *hlen = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nq + 1));
    int32_t *hpool = NULL;
    int64_t hpool_n = 0, hpool_cap = 0;
    uint8_t *inbatch = (uint8_t *)calloc((size_t)nq + 1, 1);
    int64_t *ordr = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    for (int64_t i = 0; i < N; ++i) stamp[i] = -1;
    for (int64_t i = 0; i < nq; ++i) { soft[i] = -1; hlen[i] = 0; hoff[i] = 0; }
    for (int64_t i = 0; i < n; ++i) inbatch[qidx[i]] = 1;

    /* processing order: given order for self mode; parents first otherwise
     * (any parent-before-child order gives the same result) */
    for (int64_t i = 0; i < n; ++i) ordr[i] = i;
    if (cfg->work_sharing == 1 || cfg->work_sharing == 2) {
        int32_t *depth = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
        for (int64_t i = 0; i < n; ++i) {
            int32_t dd = 0, p = parent[qidx[i]];
            while (p >= 0) { ++dd; p = parent[p - nx]; }
            depth[i] = dd;
        }
        /* stable insertion-merge sort by depth (counting sort) */
        int32_t maxd = 0;
        for (int64_t i = 0; i < n; ++i) if (depth[i] > maxd) maxd = depth[i];
        int64_t *cnt = (int64_t *)calloc((size_t)maxd + 2, sizeof(int64_t));
        for (int64_t i = 0; i < n; ++i) cnt[depth[i] + 1]++;
        for (int32_t k = 0; k <= maxd; ++k) cnt[k + 1] += cnt[k];
        for (int64_t i = 0; i < n; ++i) ordr[cnt[depth[i]]++] = i;
        free(cnt); free(depth);
    }

    const double band = cfg->uncertain_rel * fabs(eps);
    const double frel = cfg->fragile_rel;
    int64_t npairs = 0;
    uint64_t rs = cfg->shuffle_seed;

    for (int64_t oi = 0; oi < n; ++oi) {
        int64_t i = ordr[oi];
        int64_t qi = qidx[i];
        int32_t q = (int32_t)(nx + qi);
        const float *qv = V + (int64_t)q * d;
        int64_t ni = 0, nw = 0, wh = 0, nh = 0;
        int32_t st[ST_N] = {0};
        int fragile = 0;

#define IN_RANGE(t) (fabs((t) - eps) <= band && cfg->uncertain_policy == 1 ? 0 \
                     : fabs((t) - eps) <= band && cfg->uncertain_policy == 2 ? 1 \
                     : ((t) < eps))
#define VISIT(v) do { stamp[v] = i; dq[v] = dist64(qv, V + (int64_t)(v) * d, d, metric); \
                      st[ST_NDIST]++; if ((v) < nx) st[ST_VDATA]++; \
                      if (fabs(dq[v] - eps) <= band) fragile |= (cfg->hybrid != 0 || cfg->work_sharing != 0); } while (0)

        /* expand node u: visit its unvisited data neighbours; in-range ones
         * join I and the worklist, out-range ones the bounded heap */
#define EXPAND(uu) do { \
            const int32_t *row_ = adj + (int64_t)(uu) * R; \
            st[ST_NEXP]++; \
            for (int j_ = 0; j_ < R; ++j_) { \
                int32_t v = row_[j_]; \
                if (v < 0 || v >= nx || stamp[v] == i) continue; \
                VISIT(v); \
                if (IN_RANGE(dq[v])) { I[ni++] = v; W[nw++] = v; } \
                else if (hyb && hcap > 0) { \
                    H[nh].d = dq[v]; H[nh].id = v; ++nh; \
                    if (nh > hcap) { \
                        int64_t mx = 0; \
                        for (int64_t k = 1; k < nh; ++k) \
                            if (lt_pair(H[mx].d, H[mx].id, H[k].d, H[k].id)) mx = k; \
                        for (int64_t k = 0; k < nh; ++k) \
                            if (k != mx && fabs(H[k].d - H[mx].d) <= frel * fabs(H[mx].d)) fragile = 1; \
                        H[mx] = H[--nh]; \
                    } \
                } \
            } } while (0)

        /* SeedPhase (Algorithm 3): S = {s} + cache of the parent (+ {q} on
         * the merged index) */
        int32_t seeds[4];
        int ns = 0;
        const int nnmap = cfg->work_sharing == 3;
        if (nnmap) {
            if (nn_d[qi] < eps) seeds[ns++] = nn_w[qi];
        } else {
            /* per-query seed (the node an upper-layer descent reached), else s */
            seeds[ns++] = qseed ? qseed[qi] : s;
        }
        if (cfg->merged) {
            stamp[q] = i; /* q is visited, at distance 0, and never in X */
            dq[q] = 0.0;
        }
        if (cfg->work_sharing == 1) {
            int32_t p = parent[qi];
            if (p >= 0 && inbatch[p - nx] && soft[p - nx] >= 0) seeds[ns++] = soft[p - nx];
        }
        for (int k = 0; k < ns; ++k) {
            int32_t u = seeds[k];
            if (stamp[u] == i) continue;
            VISIT(u);
            if (u < nx && IN_RANGE(dq[u])) I[ni++] = u;
        }
        if (cfg->work_sharing == 2) {
            int32_t p = parent[qi];
            if (p >= 0 && inbatch[p - nx]) {
                for (int64_t t = 0; t < hlen[p - nx]; ++t) {
                    int32_t u = hpool[hoff[p - nx] + t];
                    if (stamp[u] == i) continue;
                    VISIT(u);
                    if (u < nx && IN_RANGE(dq[u])) I[ni++] = u;
                }
            }
        }

        /* GreedySearchPhase (Algorithms 4, 5).  Merged: pop q and probe
         * N(q), then stop by rule 3.  Separate: best-first from the seeds,
         * stop rules 1 and 2. */
        const int32_t *nqrow = adj + (int64_t)q * R;
        int32_t gpops = 0;
        if (cfg->merged) {
            for (int j = 0; j < R; ++j) {
                int32_t v = nqrow[j];
                if (v < 0 || stamp[v] == i) continue;
                VISIT(v);
                if (v < nx && IN_RANGE(dq[v])) I[ni++] = v;
            }
        } else if (!nnmap) {
            /* the queue starts as every visited seed (all data nodes) */
            int64_t ng = 0;
            for (int k = 0; k < ns; ++k)
                if (seeds[k] >= 0 && stamp[seeds[k]] == i) {
                    int dup = 0;
                    for (int64_t t = 0; t < ng; ++t) if (G[t].id == seeds[k]) dup = 1;
                    if (!dup) { G[ng].d = dq[seeds[k]]; G[ng].id = seeds[k]; ++ng; }
                }
            if (cfg->work_sharing == 2) {
                int32_t p = parent[qi];
                if (p >= 0 && inbatch[p - nx])
                    for (int64_t t = 0; t < hlen[p - nx]; ++t) {
                        int32_t u = hpool[hoff[p - nx] + t];
                        int dup = 0;
                        for (int64_t k = 0; k < ng; ++k) if (G[k].id == u) dup = 1;
                        if (!dup) { G[ng].d = dq[u]; G[ng].id = u; ++ng; }
                    }
            }
            double best = INFINITY;
            int32_t stall = 0;
            for (;;) {
                if (ng == 0) break;
                int64_t mn = 0;
                for (int64_t k = 1; k < ng; ++k)
                    if (lt_pair(G[k].d, G[k].id, G[mn].d, G[mn].id)) mn = k;
                for (int64_t k = 0; k < ng; ++k)
                    if (k != mn && fabs(G[k].d - G[mn].d) <= frel * fabs(G[mn].d)) fragile = 1;
                if (fabs(G[mn].d - eps) <= band || fabs(G[mn].d - eps) <= frel * fabs(eps)) fragile = 1;
                if (G[mn].id < nx && IN_RANGE(G[mn].d)) break;               /* rule 1 */
                if (isfinite(best) && fabs(G[mn].d - best) <= frel * fabs(best)) fragile = 1;
                if (G[mn].d < best) { best = G[mn].d; stall = 0; }
                else ++stall;
                if (cfg->conv_threshold > 0 && stall >= cfg->conv_threshold) break; /* rule 2 */
                int32_t u = G[mn].id;
                G[mn] = G[--ng];
                ++gpops;
                const int32_t *row = adj + (int64_t)u * R;
                for (int j = 0; j < R; ++j) {
                    int32_t v = row[j];
                    if (v < 0 || v >= nx || stamp[v] == i) continue;
                    VISIT(v);
                    G[ng].d = dq[v]; G[ng].id = v; ++ng;
                    if (IN_RANGE(dq[v])) I[ni++] = v;
                }
                while (ng > cfg->greedy_beam) {
                    int64_t mx = 0;
                    for (int64_t k = 1; k < ng; ++k)
                        if (lt_pair(G[mx].d, G[mx].id, G[k].d, G[k].id)) mx = k;
                    for (int64_t k = 0; k < ng; ++k)
                        if (k != mx && fabs(G[k].d - G[mx].d) <= frel * fabs(G[mx].d)) fragile = 1;
                    G[mx] = G[--ng];
                }
            }
        }

        /* CheckHybrid (Algorithm 6): adapt only on the merged index */
        int hyb = 0;
        if (cfg->hybrid == 1) hyb = 1;
        else if (cfg->hybrid == 3) hyb = budget[i] > 0;
        else if (cfg->hybrid == 2 && nnmap) {
            hyb = nn_ood[qi] != 0;
            st[ST_OOD] = hyb;
        } else if (cfg->hybrid == 2 && cfg->merged) {
            double s1 = 0.0, s2 = 0.0;
            int64_t c1 = 0, c2 = 0;
            for (int j = 0; j < R; ++j) {
                int32_t y = nqrow[j];
                if (y < 0 || y >= nx) continue;
                double t = metric == OR_L2 ? l2_64(qv, V + (int64_t)y * d, d)
                                           : sqrt(fmax(0.0, 2.0 * dist64(qv, V + (int64_t)y * d, d, OR_IP)));
                s1 += t; ++c1;
                for (int k = 0; k < R; ++k) {
                    int32_t z = adj[(int64_t)y * R + k];
                    if (z < 0 || z >= nx || z == q) continue;
                    s2 += l2_64(V + (int64_t)y * d, V + (int64_t)z * d, d);
                    ++c2;
                }
            }
            if (c1 == 0) hyb = 1;
            else if (c2 == 0) hyb = 0;
            else {
                double r = (s1 / c1) / (s2 / c2);
                hyb = r > cfg->ood_ratio;
                if (fabs(r - cfg->ood_ratio) <= 1e-5 * cfg->ood_ratio) fragile = 1;
            }
            st[ST_OOD] = hyb;
        }
        st[ST_HYB] = hyb;

        /* ExpansionPhase (Algorithm 7) */
        for (int64_t t = 0; t < ni; ++t) W[nw++] = I[t];
        int64_t hpops = 0, unprod = 0, before = 0;
        int pending = 0;
        for (;;) {
            /* closure over the in-range worklist */
            while (wh < nw) {
                if (rs) {
                    int64_t pick = wh + (int64_t)(lcg_next(&rs) % (uint64_t)(nw - wh));
                    int32_t tmp = W[pick]; W[pick] = W[wh]; W[wh] = tmp;
                }
                EXPAND(W[wh]);
                ++wh;
            }
            if (pending) { if (ni == before) ++unprod; else unprod = 0; pending = 0; }
            /* best-first pop of an out-range bridge */
            if (!hyb || nh == 0) break;
            if (cfg->hybrid == 3) { if (hpops >= budget[i]) break; }
            else if (cfg->conv_threshold > 0 && unprod >= cfg->conv_threshold) break;
            int64_t mn = 0;
            for (int64_t k = 1; k < nh; ++k)
                if (lt_pair(H[k].d, H[k].id, H[mn].d, H[mn].id)) mn = k;
            for (int64_t k = 0; k < nh; ++k)
                if (k != mn && fabs(H[k].d - H[mn].d) <= frel * fabs(H[mn].d)) fragile = 1;
            int32_t b = H[mn].id;
            H[mn] = H[--nh];
            ++hpops;
            before = ni;
            pending = 1;
            EXPAND(b);
        }
        st[ST_HPOPS] = (int32_t)hpops;
        if (!cfg->merged && !nnmap) st[ST_OOD] = gpops;

        /* UpdateCache (Algorithm 8) */
        if (cfg->work_sharing == 1) {
            /* soft: the closest visited data node (reading: ties on id) */
            int32_t bi = -1, b2 = -1;
            for (int64_t v = 0; v < nx; ++v) {
                if (stamp[v] != i) continue;
                if (bi < 0 || lt_pair(dq[v], (int32_t)v, dq[bi], bi)) { b2 = bi; bi = (int32_t)v; }
                else if (b2 < 0 || lt_pair(dq[v], (int32_t)v, dq[b2], b2)) b2 = (int32_t)v;
            }
            soft[qi] = bi;
            if (bi >= 0 && b2 >= 0 && fabs(dq[b2] - dq[bi]) <= frel * fabs(dq[bi])) fragile = 1;
        } else if (cfg->work_sharing == 2) {
            if (hpool_n + ni > hpool_cap) {
                hpool_cap = (hpool_n + ni) * 2 + 1024;
                hpool = (int32_t *)realloc(hpool, sizeof(int32_t) * (size_t)hpool_cap);
            }
            hoff[qi] = hpool_n;
            hlen[qi] = ni;
            for (int64_t t = 0; t < ni; ++t) hpool[hpool_n++] = I[t];
        }

        /* emit */
        for (int64_t t = 0; t < ni; ++t) {
            if (npairs < cap) {
                oq[npairs] = (int32_t)qi;
                ox[npairs] = I[t];
                od[npairs] = dq[I[t]];
            }
            ++npairs;
        }
        st[ST_PAIRS] = (int32_t)ni;
        st[ST_FRAGILE] = fragile;
        if (stats) memcpy(stats + i * ST_N, st, sizeof(st));
#undef IN_RANGE
#undef VISIT
#undef EXPAND
    }
    free(stamp); free(dq); free(I); free(W); free(H); free(G); free(soft); free(hoff);
    free(hlen); free(hpool); free(inbatch); free(ordr);
    return npairs;
}

/* Self-mode BFS join of many queries on all host cores (timing only; each
 * query runs the same steps as or_join with work_sharing = self, hybrid =
 * off, but writes only its pair count).  Used for the CPU baseline. */
void or_join_self_counts(const float *V, int64_t nx, int64_t nq, int d, int metric,
                         const int32_t *adj, int R, int32_t s, const int32_t *qidx,
                         int64_t n, double eps, int64_t *counts)
{
    int64_t N = nx + nq;
#pragma omp parallel
    {
        int64_t *stamp = (int64_t *)malloc(sizeof(int64_t) * (size_t)N);
        int32_t *W = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
        for (int64_t k = 0; k < N; ++k) stamp[k] = -1;
#pragma omp for schedule(dynamic, 8)
        for (int64_t i = 0; i < n; ++i) {
            int32_t q = (int32_t)(nx + qidx[i]);
            const float *qv = V + (int64_t)q * d;
            int64_t nw = 0, wh = 0;
            stamp[q] = i;
            if (stamp[s] != i) {
                stamp[s] = i;
                if (s < nx && dist64(qv, V + (int64_t)s * d, d, metric) < eps) W[nw++] = s;
            }
            for (int j = 0; j < R; ++j) {
                int32_t v = adj[(int64_t)q * R + j];
                if (v < 0 || stamp[v] == i) continue;
                stamp[v] = i;
                double t = dist64(qv, V + (int64_t)v * d, d, metric);
                if (v < nx && t < eps) W[nw++] = v;
            }
            while (wh < nw) {
                int32_t u = W[wh++];
                for (int j = 0; j < R; ++j) {
                    int32_t v = adj[(int64_t)u * R + j];
                    if (v < 0 || v >= nx || stamp[v] == i) continue;
                    stamp[v] = i;
                    if (dist64(qv, V + (int64_t)v * d, d, metric) < eps) W[nw++] = v;
                }
            }
            counts[i] = nw;
        }
        free(stamp); free(W);
    }
}

/* ------------------------------------------------------------------------
 * O5 input: per-query features known once the probe of Algorithm 4 is done
 * (q, its neighbour list N(q), the entry s, eps), extending the d1/d2 signal
 * of CheckHybrid (Section 4.4).  With A = N(q) restricted to data nodes:
 *   f0 = eps
 *   f1 = dist(q, s)
 *   f2 = min over A of dist(q, y)                       (0 if A is empty)
 *   f3 = d1 = mean over A of the L2 length |q - y|      (0 if A is empty)
 *   f4 = d2 = mean L2 edge length |y - z| over y in A, z in N(y), z a data
 *        node other than q                              (0 if none)
 *   f5 = d1 / d2                                        (0 if d2 is 0)
 *   f6 = |A| / R
 *   f7 = |{y in A : dist(q, y) < eps}| / R
 * dist is the join metric (L2, or 1 - <q, y> for IP); d1 and d2 are in L2
 * units as in the OOD test (reading: for IP, |q - y| = sqrt(2 (1 - <q, y>))
 * on unit vectors, computed here from the vectors directly).  Output row i:
 * the query vector (d values) followed by f0..f7.
 * ---------------------------------------------------------------------- */
void or_features(const float *V, int64_t nx, int64_t nq, int d, int metric,
                 const int32_t *adj, int R, int32_t entry, const int32_t *qidx,
                 int64_t n, double eps, double *out)
{
    (void)nq;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t q = nx + qidx[i];
        const float *qv = V + q * d;
        double *o = out + i * (int64_t)(d + 8);
        for (int k = 0; k < d; ++k) o[k] = (double)qv[k];
        double f1 = dist64(qv, V + (int64_t)entry * d, d, metric);
        double mn = 0.0, s1 = 0.0, s2 = 0.0;
        int64_t na = 0, nin = 0, c2 = 0;
        for (int j = 0; j < R; ++j) {
            int32_t y = adj[q * R + j];
            if (y < 0 || y >= nx) continue;
            double dy = dist64(qv, V + (int64_t)y * d, d, metric);
            if (na == 0 || dy < mn) mn = dy;
            if (dy < eps) ++nin;
            s1 += l2_64(qv, V + (int64_t)y * d, d);
            ++na;
            for (int k = 0; k < R; ++k) {
                int32_t z = adj[(int64_t)y * R + k];
                if (z < 0 || z >= nx || z == q) continue;
                s2 += l2_64(V + (int64_t)y * d, V + (int64_t)z * d, d);
                ++c2;
            }
        }
        double d1 = na ? s1 / (double)na : 0.0;
        double d2 = c2 ? s2 / (double)c2 : 0.0;
        o[d + 0] = eps;
        o[d + 1] = f1;
        o[d + 2] = na ? mn : 0.0;
        o[d + 3] = d1;
        o[d + 4] = d2;
        o[d + 5] = d2 > 0.0 ? d1 / d2 : 0.0;
        o[d + 6] = (double)na / (double)R;
        o[d + 7] = (double)nin / (double)R;
    }
}

/* ------------------------------------------------------------------------
 * O5: the difficulty predictor, a plain MLP  din -> h1 -> h2 -> k  with ReLU
 * on the hidden layers and k sigmoid heads (not in the paper; a project
 * addition).  Weights are row-major W[out][in].
 * ---------------------------------------------------------------------- */
static void dense(int n, int din, int dout, const double *X, const double *W,
                  const double *b, int relu, double *Y)
{
    for (int r = 0; r < n; ++r)
        for (int o = 0; o < dout; ++o) {
            double acc = b[o];
            for (int i = 0; i < din; ++i) acc += W[(int64_t)o * din + i] * X[(int64_t)r * din + i];
            Y[(int64_t)r * dout + o] = (relu && acc < 0.0) ? 0.0 : acc;
        }
}

void or_mlp_forward(int n, int din, int h1, int h2, int k, const double *X,
                    const double *W1, const double *b1, const double *W2,
                    const double *b2, const double *W3, const double *b3,
                    double *logits)
{
    double *a1 = (double *)malloc(sizeof(double) * (size_t)n * h1);
    double *a2 = (double *)malloc(sizeof(double) * (size_t)n * h2);
    dense(n, din, h1, X, W1, b1, 1, a1);
    dense(n, h1, h2, a1, W2, b2, 1, a2);
    dense(n, h2, k, a2, W3, b3, 0, logits);
    free(a1); free(a2);
}

/* Mean binary cross-entropy with logits over the entries where mask != 0
 * (mask NULL: all), and its gradients with respect to every parameter. */
double or_mlp_bce_backward(int n, int din, int h1, int h2, int k, const double *X,
                           const double *W1, const double *b1, const double *W2,
                           const double *b2, const double *W3, const double *b3,
                           const double *Y, const double *mask, double *gW1,
                           double *gb1, double *gW2, double *gb2, double *gW3,
                           double *gb3)
{
    double *a1 = (double *)malloc(sizeof(double) * (size_t)n * h1);
    double *a2 = (double *)malloc(sizeof(double) * (size_t)n * h2);
    double *z = (double *)malloc(sizeof(double) * (size_t)n * k);
    double *g3 = (double *)malloc(sizeof(double) * (size_t)n * k);
    double *g2 = (double *)malloc(sizeof(double) * (size_t)n * h2);
    double *g1 = (double *)malloc(sizeof(double) * (size_t)n * h1);
    dense(n, din, h1, X, W1, b1, 1, a1);
    dense(n, h1, h2, a1, W2, b2, 1, a2);
    dense(n, h2, k, a2, W3, b3, 0, z);
    double cnt = 0.0, loss = 0.0;
    for (int64_t t = 0; t < (int64_t)n * k; ++t) cnt += mask ? (mask[t] != 0.0) : 1.0;
    if (cnt == 0.0) cnt = 1.0;
    for (int64_t t = 0; t < (int64_t)n * k; ++t) {
        double m = mask ? (mask[t] != 0.0) : 1.0;
        double zz = z[t], y = Y[t];
        /* BCE(sigmoid(z), y) = max(z, 0) - z y + log(1 + exp(-|z|)) */
        loss += m * (fmax(zz, 0.0) - zz * y + log1p(exp(-fabs(zz))));
        double sg = 1.0 / (1.0 + exp(-zz));
        g3[t] = m * (sg - y) / cnt;
    }
    loss /= cnt;
    /* layer 3 */
    memset(gW3, 0, sizeof(double) * (size_t)k * h2);
    memset(gb3, 0, sizeof(double) * (size_t)k);
    for (int r = 0; r < n; ++r)
        for (int o = 0; o < k; ++o) {
            double g = g3[(int64_t)r * k + o];
            gb3[o] += g;
            for (int i = 0; i < h2; ++i) gW3[(int64_t)o * h2 + i] += g * a2[(int64_t)r * h2 + i];
        }
    for (int r = 0; r < n; ++r)
        for (int i = 0; i < h2; ++i) {
            double acc = 0.0;
            for (int o = 0; o < k; ++o) acc += W3[(int64_t)o * h2 + i] * g3[(int64_t)r * k + o];
            g2[(int64_t)r * h2 + i] = a2[(int64_t)r * h2 + i] > 0.0 ? acc : 0.0;
        }
    /* layer 2 */
    memset(gW2, 0, sizeof(double) * (size_t)h2 * h1);
    memset(gb2, 0, sizeof(double) * (size_t)h2);
    for (int r = 0; r < n; ++r)
        for (int o = 0; o < h2; ++o) {
            double g = g2[(int64_t)r * h2 + o];
            gb2[o] += g;
            for (int i = 0; i < h1; ++i) gW2[(int64_t)o * h1 + i] += g * a1[(int64_t)r * h1 + i];
        }
    for (int r = 0; r < n; ++r)
        for (int i = 0; i < h1; ++i) {
            double acc = 0.0;
            for (int o = 0; o < h2; ++o) acc += W2[(int64_t)o * h1 + i] * g2[(int64_t)r * h2 + o];
            g1[(int64_t)r * h1 + i] = a1[(int64_t)r * h1 + i] > 0.0 ? acc : 0.0;
        }
    /* layer 1 */
    memset(gW1, 0, sizeof(double) * (size_t)h1 * din);
    memset(gb1, 0, sizeof(double) * (size_t)h1);
    for (int r = 0; r < n; ++r)
        for (int o = 0; o < h1; ++o) {
            double g = g1[(int64_t)r * h1 + o];
            gb1[o] += g;
            for (int i = 0; i < din; ++i) gW1[(int64_t)o * din + i] += g * X[(int64_t)r * din + i];
        }
    free(a1); free(a2); free(z); free(g3); free(g2); free(g1);
    return loss;
}

/* ------------------------------------------------------------------------
 * O5: one step of Adam (Kingma and Ba, "Adam: a method for stochastic
 * optimization", ICLR 2015, Algorithm 1) on n parameters, step number t >= 1:
 *   m <- b1 m + (1 - b1) g
 *   v <- b2 v + (1 - b2) g^2
 *   p <- p - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
 * (bias-corrected moments; eps added outside the square root).  The
 * optimizer that trains the difficulty MLP; not in the paper.
 * ---------------------------------------------------------------------- */
void or_adam_step(int64_t n, double *p, const double *g, double *m, double *v, int64_t t,
                  double lr, double b1, double b2, double eps)
{
    double c1 = 1.0 - pow(b1, (double)t);
    double c2 = 1.0 - pow(b2, (double)t);
    for (int64_t i = 0; i < n; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        double mhat = m[i] / c1;
        double vhat = v[i] / c2;
        p[i] -= lr * mhat / (sqrt(vhat) + eps);
    }
}

/* ------------------------------------------------------------------------
 * NN-Map build (Section 6, planned in the paper): for every query q its
 * nearest data node w[q] by the join metric (exact, fp64, ties to the
 * smaller id), dist[q] = dist(q, w[q]), and an OOD bit.  Reading of the OOD
 * bit (the paper says only that it is the score the merged index would
 * derive): the d1/d2 rule of Section 4.4 with A = {w[q]}, i.e. d1 = the L2
 * distance |q - w[q]| and d2 = the mean L2 length of w[q]'s edges to data
 * nodes in the data graph (adj rows 0..nx-1); OOD iff d1/d2 > ratio (no edge:
 * not OOD).
 * ---------------------------------------------------------------------- */
void or_nnmap(const float *V, int64_t nx, int64_t nq, int d, int metric, const int32_t *adj,
              int R, double ratio, int32_t *w, double *dist, uint8_t *ood)
{
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t i = 0; i < nq; ++i) {
        const float *qv = V + (nx + i) * (int64_t)d;
        int32_t bi = -1;
        double bd = INFINITY;
        for (int64_t j = 0; j < nx; ++j) {
            double t = dist64(qv, V + j * (int64_t)d, d, metric);
            if (t < bd) { bd = t; bi = (int32_t)j; }   /* strict: ties keep the smaller id */
        }
        w[i] = bi;
        dist[i] = bd;
        double s2 = 0.0;
        int64_t c2 = 0;
        for (int k = 0; k < R; ++k) {
            int32_t z = adj[(int64_t)bi * R + k];
            if (z < 0 || z >= nx) continue;
            s2 += l2_64(V + (int64_t)bi * d, V + (int64_t)z * d, d);
            ++c2;
        }
        double d1 = l2_64(qv, V + (int64_t)bi * d, d);
        ood[i] = c2 > 0 && d1 / (s2 / (double)c2) > ratio;
    }
}

/* ------------------------------------------------------------------------
 * Incremental insertion of a batch of query nodes into a merged graph
 * (Section 4.3, index maintenance: a node update needs only its set label;
 * existing update mechanisms apply).  Reading: the new nodes get the
 * build's recipe -- exact kNN (K = Kc) among ALL nodes, old and new, RNG
 * prune to R -- and their kept edges are offered as reverse edges; a node v
 * that receives offers gets cand(v) = its current row (old nodes) or its
 * pruned list (new nodes) plus the offers, kept whole if |cand| <= R, else
 * RNG-pruned; rows without offers stay as they are.  Then the build's
 * connectivity repair from the (unchanged) entry, and the edge lengths.
 * V holds all n_old + n_new rows; adj [n_old + n_new][R] holds the old rows
 * on entry (the new rows are written).  Returns the repair edges added.
 * ---------------------------------------------------------------------- */
int64_t or_insert_batch(const float *V, int64_t n_old, int64_t n_new, int d, int R, int Kc,
                        int32_t *adj, double *elen, int32_t s)
{
    int64_t n = n_old + n_new;
    int32_t *knn = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_new * Kc + 1));
    double *kd = (double *)malloc(sizeof(double) * (size_t)(n_new * Kc + 1));
    int32_t *fwd = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_new * R + 1));
    int *fdeg = (int *)calloc((size_t)n_new + 1, sizeof(int));
    /* exact kNN of each new node among all nodes (self excluded) */
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < n_new; ++i) {
        int64_t u = n_old + i;
        int32_t *ri = knn + i * Kc;
        double *rd = kd + i * Kc;
        int cnt = 0;
        for (int64_t v = 0; v < n; ++v) {
            if (v == u) continue;
            double t = l2_64(V + u * d, V + v * d, d);
            if (cnt == Kc && !lt_pair(t, (int32_t)v, rd[Kc - 1], ri[Kc - 1])) continue;
            int p = cnt < Kc ? cnt++ : Kc - 1;
            while (p > 0 && lt_pair(t, (int32_t)v, rd[p - 1], ri[p - 1])) {
                rd[p] = rd[p - 1]; ri[p] = ri[p - 1]; --p;
            }
            rd[p] = t; ri[p] = (int32_t)v;
        }
        for (int p = cnt; p < Kc; ++p) { ri[p] = -1; rd[p] = INFINITY; }
        fdeg[i] = or_rng_prune(V, d, u, ri, rd, Kc, R, fwd + i * R);
    }
    /* offers: v gets u for every kept (u, v) of a new node u */
    int64_t *ocnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t i = 0; i < n_new; ++i)
        for (int j = 0; j < fdeg[i]; ++j) ocnt[fwd[i * R + j] + 1]++;
    for (int64_t v = 0; v < n; ++v) ocnt[v + 1] += ocnt[v];
    int32_t *off = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ocnt[n] + 1));
    int64_t *opos = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t v = 0; v < n; ++v) opos[v] = ocnt[v];
    for (int64_t i = 0; i < n_new; ++i)
        for (int j = 0; j < fdeg[i]; ++j) off[opos[fwd[i * R + j]]++] = (int32_t)(n_old + i);
    /* new rows start as their pruned lists */
    for (int64_t i = 0; i < n_new; ++i) {
        int32_t *row = adj + (n_old + i) * R;
        for (int j = 0; j < R; ++j) row[j] = j < fdeg[i] ? fwd[i * R + j] : -1;
    }
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t v = 0; v < n; ++v) {
        int64_t no = ocnt[v + 1] - ocnt[v];
        if (no == 0) continue;
        int32_t *row = adj + v * R;
        int deg = row_degree(row, R);
        or_cand *c = (or_cand *)malloc(sizeof(or_cand) * (size_t)(deg + no + 1));
        int m = 0;
        for (int j = 0; j < deg; ++j) c[m++].id = row[j];
        for (int64_t t = ocnt[v]; t < ocnt[v + 1]; ++t) {
            int32_t u = off[t];
            int dup = 0;
            for (int j = 0; j < m; ++j) if (c[j].id == u) { dup = 1; break; }
            if (!dup) c[m++].id = u;
        }
        for (int j = 0; j < m; ++j) c[j].d = l2_64(V + v * d, V + (int64_t)c[j].id * d, d);
        qsort(c, (size_t)m, sizeof(or_cand), cmp_cand);
        for (int j = 0; j < R; ++j) row[j] = -1;
        if (m <= R) {
            for (int j = 0; j < m; ++j) row[j] = c[j].id;
        } else {
            int32_t *ci = (int32_t *)malloc(sizeof(int32_t) * (size_t)m);
            double *cdd = (double *)malloc(sizeof(double) * (size_t)m);
            for (int j = 0; j < m; ++j) { ci[j] = c[j].id; cdd[j] = c[j].d; }
            or_rng_prune(V, d, v, ci, cdd, m, R, row);
            free(ci); free(cdd);
        }
        free(c);
    }
    /* connectivity repair from s, as in the build */
    uint8_t *reach = (uint8_t *)malloc((size_t)n);
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int64_t added = 0;
    for (;;) {
        bfs_reach(adj, n, R, s, reach, queue);
        int64_t w = -1;
        for (int64_t u = 0; u < n; ++u) if (!reach[u]) { w = u; break; }
        if (w < 0) break;
        int64_t pf = -1, pa = -1;
        double df = INFINITY, da = INFINITY;
        for (int64_t p = 0; p < n; ++p) {
            if (!reach[p]) continue;
            double t = l2_64(V + p * d, V + w * d, d);
            if (lt_pair(t, (int32_t)p, da, (int32_t)pa)) { da = t; pa = p; }
            if (row_degree(adj + p * R, R) < R && lt_pair(t, (int32_t)p, df, (int32_t)pf)) {
                df = t; pf = p;
            }
        }
        if (pf >= 0) {
            int32_t *row = adj + pf * R;
            row[row_degree(row, R)] = (int32_t)w;
            sort_row(V, d, pf, row, R);
        } else {
            int32_t *row = adj + pa * R;
            row[R - 1] = (int32_t)w;
            sort_row(V, d, pa, row, R);
        }
        ++added;
    }
    for (int64_t u = 0; u < n; ++u)
        for (int j = 0; j < R; ++j) {
            int32_t v = adj[u * R + j];
            elen[u * R + j] = v >= 0 ? l2_64(V + u * d, V + (int64_t)v * d, d) : INFINITY;
        }
    free(knn); free(kd); free(fwd); free(fdeg); free(ocnt); free(off); free(opos);
    free(reach); free(queue);
    return added;
}

/* ---------------------------------------------------------------------------
 * HNSW-style upper layers over the data graph (the paper's index-type
 * experiment, Section 5: the method treats the graph index as a black box,
 * and HNSW reaches its base layer through a greedy descent over sparser
 * upper layers).
 *
 * Levels: data node v gets L(v) = the number of trailing zero 4-bit digits
 * of output v + 1 of SplitMix64 (Steele, Lea and Flood 2014) seeded with
 * `seed`, capped at max_levels.  So P(L >= l) = 16^-l and the layers are
 * nested.  Layer l (l >= 1) holds the nodes with L >= l; its graph is the
 * merged-graph recipe over those nodes alone (built by the Python wrapper
 * with or_build_merged, ids mapped to data ids).
 *
 * Descent (reading: HNSW's upper-layer search with a queue of one): from
 * the top layer's entry, repeatedly move to the neighbour in that layer that
 * is smallest by (dist(q, .), id) while it is smaller than the current node
 * by (dist, id); then continue in the next layer down from the node reached.
 * The node reached in layer 1 seeds the query's greedy phase on the data
 * graph (or_join's qseed) in place of the data graph's entry.
 * ---------------------------------------------------------------------------
 */

/* output k (k >= 1) of SplitMix64 seeded with `seed` */
uint64_t or_splitmix64(uint64_t seed, uint64_t k)
{
    uint64_t z = seed + k * 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

void or_levels(int64_t n, uint64_t seed, int max_levels, int8_t *lvl)
{
    for (int64_t v = 0; v < n; ++v) {
        uint64_t z = or_splitmix64(seed, (uint64_t)v + 1);
        int l = 0;
        while (l < max_levels && (z & 15u) == 0) { ++l; z >>= 4; }
        lvl[v] = (int8_t)l;
    }
}

/* V = [X; Q].  Layer j (0 = layer 1) has rows layer_off[j] .. of adj
 * ([rows][R], data ids, -1 padded); pos[j * nx + v] is node v's row within
 * layer j (-1 if absent); entries[j] is layer j's entry.  For each listed
 * query qidx[i] (query index) writes the seed and the number of moves. */
void or_descend(const float *V, int64_t nx, int64_t nq, int d, int metric, int nl,
                const int64_t *layer_off, const int32_t *pos, const int32_t *adj, int R,
                const int32_t *entries, const int32_t *qidx, int64_t n, int32_t *seed,
                int32_t *moves)
{
    (void)nq;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        const float *qv = V + (nx + (int64_t)qidx[i]) * d;
        int32_t c = entries[nl - 1];
        double dc = dist64(qv, V + (int64_t)c * d, d, metric);
        int32_t mv = 0;
        for (int j = nl - 1; j >= 0; --j) {
            for (;;) {
                const int32_t *row = adj + (layer_off[j] + pos[(int64_t)j * nx + c]) * R;
                int32_t b = c;
                double db = dc;
                for (int k = 0; k < R; ++k) {
                    int32_t v = row[k];
                    if (v < 0) continue;
                    double dv = dist64(qv, V + (int64_t)v * d, d, metric);
                    if (dv < db || (dv == db && v < b)) { b = v; db = dv; }
                }
                if (b == c) break;
                c = b;
                dc = db;
                ++mv;
            }
        }
        seed[i] = c;
        moves[i] = mv;
    }
}
