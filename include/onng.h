/*
 * onng.h — C-ABI of the MI355X (gfx950) implementation of the adjusted
 * k-nearest-neighbour-graph index and search of Iwasaki & Miyazaki,
 * "Optimization of Indexing Based on k-Nearest Neighbor Graph for Proximity
 * Search in High-dimensional Data" (arXiv 1810.07355).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every buffer pointer is DEVICE memory owned by the caller, unless the
 *    comment says "host".  The library keeps no pointer after a call returns.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Calls enqueue their kernels on it and return after argument validation;
 *    results are valid once the stream is synchronised.  Calls that return a
 *    count or result to a host pointer (onng_adjust_degree,
 *    onng_adjust_degree_constrained, onng_adjust_path, onng_graph_stats)
 *    synchronise the stream themselves.
 *  - Scratch memory comes from the caller: `ws`/`ws_bytes`, sized by the
 *    matching *_workspace_size function.  The library allocates no device
 *    memory of its own (the tuning cache is host memory).
 *  - Errors are return codes; nothing throws or aborts across the ABI.
 *    Argument errors are detected before any kernel is enqueued, and then no
 *    output is touched.  onng_last_error() gives a message for the calling
 *    thread.  A HIP runtime failure is ONNG_ERR_DEVICE.
 *  - Distances: squared Euclidean (ONNG_L2SQ) or cosine distance 1 - <x, y>
 *    (ONNG_COSINE, meant for unit vectors).  On u8 data with ONNG_L2SQ every
 *    distance is an exact integer and is stored as int32; everything else is
 *    stored as float.  This is the "distance type" of the data set.
 *  - Ties are broken by node id: every ordering uses the pair (distance, id).
 *  - Calls on distinct streams with distinct workspaces may run concurrently.
 */
#ifndef ONNG_H
#define ONNG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ONNG_OK = 0,
    ONNG_ERR_INVALID_ARG = -1,   /* null pointer, bad size, k > n-1, ... */
    ONNG_ERR_UNSUPPORTED = -2,   /* dtype/metric combination not provided */
    ONNG_ERR_CAPACITY = -3,      /* an output capacity is too small */
    ONNG_ERR_WORKSPACE = -4,     /* ws_bytes below the *_workspace_size value */
    ONNG_ERR_DEVICE = -5         /* HIP runtime error */
} onng_status;

typedef enum {
    ONNG_U8 = 0,        /* uint8 components */
    ONNG_F32 = 1,       /* IEEE binary32 */
    ONNG_F16 = 2,       /* IEEE binary16, round-to-nearest-even from f32 */
    ONNG_BF16 = 3,      /* bfloat16, round-to-nearest-even from f32 */
    ONNG_FP8_E4M3 = 4   /* OCP e4m3fn with a per-row f32 scale: x = code * scale */
} onng_dtype;

typedef enum { ONNG_L2SQ = 0, ONNG_COSINE = 1 } onng_metric;

/* A set of vectors: n rows of `dim` components, `pitch_bytes` apart (a
 * multiple of 16 and at least dim * element size; bytes past the last
 * component must be zero).  `scale` is the per-row f32 scale of FP8 rows, or
 * NULL for FP8 rows that carry their scale as an f32 in their last 4 bytes
 * (then pitch_bytes >= 16 * ceil(dim / 16) + 16, so a 100-component row fits
 * one 128-byte line); NULL for the other types.  The objects of the paper's
 * Section 2 problem statement. */
typedef struct {
    const void *data;
    const float *scale;
    int64_t n;
    int32_t dim;
    int32_t dtype;        /* onng_dtype */
    int64_t pitch_bytes;
    int32_t metric;       /* onng_metric */
    int32_t reserved;
} onng_vectors;

/* A neighbourhood graph in CSR form: the edges of node v are
 * nbrs[offsets[v] .. offsets[v+1]), sorted ascending by (length, id), and
 * lens holds each edge's length d(v, nbrs[e]) in the distance type.  This is
 * the graph of Section 2 whose edges are kept sorted by length. */
typedef struct {
    const int64_t *offsets;   /* [n + 1] */
    const int32_t *nbrs;      /* [nnz] */
    const void *lens;         /* [nnz] int32 or float; may be NULL for onng_search */
    int64_t n;
    int64_t nnz;
} onng_graph;

/* ------------------------------------------------------------------------ */
/* Exact k-nearest neighbours (brute force, matrix cores)                   */
/* ------------------------------------------------------------------------ */

/* The exact k-NN graph of `base`: for every row i the k rows j != i with the
 * smallest (d(i, j), j), ascending.  It stands in for the approximate KNNG that
 * ConstructGraph (Algorithm 8) derives from an ANNG; Section 2.6 notes that
 * the exact graph is the costly ideal.
 * ids: [n][k] int32; dists: [n][k] in the distance type.  Requires
 * 1 <= k <= n - 1 and k <= 256.  On float data the distances are f32: from
 * f32 matrix-core products (|x|^2 + |y|^2 - 2<x, y>), or, for many rows, from
 * a bf16 matrix-core screen with a bound on its rounding whose survivors are
 * recomputed in f32 from the rows; rows can differ from an exact computation
 * by rounding near ties.  u8 data is exact. */
onng_status onng_build_knn(const onng_vectors *base, int32_t k, int32_t *ids, void *dists,
                           void *ws, size_t ws_bytes, void *stream);

/* General form: for each query row the k smallest (d(q, j), j) over the base
 * rows, or over the candidate ids `cand` (device [n_cand]) when it is not
 * NULL.  exclude_self skips j == query row index (queries == base).  Used for
 * seeds (the nearest pivots), ground truth and the k-NN graph.  Rows with
 * fewer than k candidates are padded with id -1 and distance INT32_MAX or
 * +inf. */
onng_status onng_topk(const onng_vectors *queries, const onng_vectors *base,
                      const int32_t *cand, int64_t n_cand, int32_t k, int32_t exclude_self,
                      int32_t *ids, void *dists, void *ws, size_t ws_bytes, void *stream);
size_t onng_topk_workspace_size(const onng_vectors *queries, const onng_vectors *base,
                                int64_t n_cand, int32_t k);

/* ------------------------------------------------------------------------ */
/* Static degree adjustment — Algorithm 2 (ConstructAdjustedGraph)          */
/* ------------------------------------------------------------------------ */

/* From a k-NN table (rows sorted by (dist, id), padded with -1), build G_e:
 * node o keeps its first min(e_o, k) edges and receives the reverse of every
 * edge m -> o among the first min(e_i, k) edges of m (Algorithm 2, with the
 * loop running while p <= e_o or p <= e_i).  An edge produced both ways is
 * kept once, with the length of the copy Algorithm 2 inserts first (its loop
 * runs over nodes in ascending id): the reverse copy when the far end has the
 * smaller id, else the forward copy.  Each list is sorted by (length, id), so
 * the result equals a sequential run of Algorithm 2 on the same table.
 * knn_dists and lens are in the distance type of `data_dtype`/`metric`.
 * offsets: [n+1] int64; nbrs/lens: capacity nnz_capacity.
 * nnz_out (host): edge count.  ONNG_ERR_CAPACITY when it exceeds
 * nnz_capacity (then *nnz_out is the size needed and the outputs are
 * unspecified).  n * (min(e_o,k) + min(e_i,k)) always suffices. */
onng_status onng_adjust_degree(const int32_t *knn_ids, const void *knn_dists, int64_t n, int32_t k,
                               int32_t data_dtype, int32_t metric, int32_t e_o, int32_t e_i,
                               int64_t *offsets, int32_t *nbrs, void *lens, int64_t nnz_capacity,
                               int64_t *nnz_out, void *ws, size_t ws_bytes, void *stream);
size_t onng_adjust_degree_workspace_size(int64_t n, int32_t k, int32_t e_o, int32_t e_i);

/* ------------------------------------------------------------------------ */
/* Static degree adjustment with constraints — Algorithm 3                  */
/* (ConstructAdjustedGraphWithConstraint)                                   */
/* ------------------------------------------------------------------------ */

/* Same inputs, outputs, errors and capacity rule as onng_adjust_degree.
 * G_t is Algorithm 2 with (0, e_i): N(G_t, o) = the nodes m that have o among
 * the first min(e_i, k) of their row, each edge with row m's length.  Nodes
 * are taken in ascending (|N(G_t, x)|, x); each takes the members of
 * N(G_t, o) in ascending (length, id) and keeps o -> n while its out-degree
 * is below e_o, or whenever n has no incoming edge yet.  Then every node
 * below e_o edges appends the members of its own row it lacks, nearest
 * first, up to e_o.  Each list is sorted by (length, id); the result equals a
 * sequential run of Algorithm 3 on the same table.  e_o may exceed k (no
 * clamp); e_i is clamped to k.  n * (min(e_o,k) + min(e_i,k)) always
 * suffices for nnz_capacity. */
onng_status onng_adjust_degree_constrained(const int32_t *knn_ids, const void *knn_dists,
                                           int64_t n, int32_t k, int32_t data_dtype,
                                           int32_t metric, int32_t e_o, int32_t e_i,
                                           int64_t *offsets, int32_t *nbrs, void *lens,
                                           int64_t nnz_capacity, int64_t *nnz_out, void *ws,
                                           size_t ws_bytes, void *stream);
size_t onng_adjust_degree_constrained_workspace_size(int64_t n, int32_t k, int32_t e_o,
                                                      int32_t e_i);

/* ------------------------------------------------------------------------ */
/* Path adjustment — Algorithms 4 (AdjustPath) and 5 (HasPath)              */
/* ------------------------------------------------------------------------ */

/* G_p from G: rounds j = 0, 1, ... visit every node n with more than j edges
 * in ascending id; n's j-th edge n -> n_d is kept unless G_p (including
 * edges kept earlier in the same round) has an edge n -> c and an edge
 * c -> n_d with len(c, n_d) < len(n, n_d).  Result: an order-preserving
 * subset of each list.  `in` must have lens.  Output capacity is in->nnz.
 * nnz_out (host): edges kept. */
onng_status onng_adjust_path(const onng_graph *in, int32_t data_dtype, int32_t metric,
                             int64_t *offsets, int32_t *nbrs, void *lens, int64_t *nnz_out,
                             void *ws, size_t ws_bytes, void *stream);
size_t onng_adjust_path_workspace_size(int64_t n, int64_t nnz);

/* ------------------------------------------------------------------------ */
/* Graph statistics — Table 4                                                */
/* ------------------------------------------------------------------------ */

/* Degree shape and incoming-edge lengths of a graph (Section 3.2, Table 4),
 * with t = max(1, floor(frac * n)) (0 when n = 0).  out (host, [3]):
 *   out[0]  mean out-degree of the t nodes of largest out-degree;
 *   out[1]  mean in-degree of the t nodes of smallest in-degree;
 *   out[2]  mean edge length after transposing the graph and keeping each
 *           node's `keep` shortest incoming edges (all of them when it has
 *           fewer), over all kept edges; a squared-L2 length enters as its
 *           square root (the Euclidean distance), a cosine length as is.
 *           0 when no edge is kept.
 * Table 4 uses frac = 0.05 and keep = 10.  Edges to ids outside [0, n) are
 * left out of the in-degrees and the transposed graph.  lens must be present, in the
 * distance type of data_dtype/metric.  Sums are in double in a fixed order.
 * Synchronises the stream. */
onng_status onng_graph_stats(const onng_graph *g, int32_t data_dtype, int32_t metric, double frac,
                             int32_t keep, double *out, void *ws, size_t ws_bytes, void *stream);
size_t onng_graph_stats_workspace_size(int64_t n, int64_t nnz);

/* ------------------------------------------------------------------------ */
/* Edge insertion — the graph updates of ConstructANNG (Appendix, Alg 9)    */
/* ------------------------------------------------------------------------ */

/* out = in plus the edges src[e] -> dst[e] of length lens[e], e < n_edges
 * (device arrays; an edge with an id outside [0, n) is skipped).  Each output
 * list holds the node's old and new edges sorted by (length, id); duplicates
 * are kept (ConstructANNG never produces one).  Same capacity rule and
 * errors as onng_adjust_degree; in->nnz + n_edges always suffices.
 * Synchronises the stream. */
onng_status onng_graph_add_edges(const onng_graph *in, const int32_t *src, const int32_t *dst,
                                 const void *lens, int64_t n_edges, int32_t data_dtype,
                                 int32_t metric, int64_t *offsets, int32_t *nbrs, void *out_lens,
                                 int64_t nnz_capacity, int64_t *nnz_out, void *ws,
                                 size_t ws_bytes, void *stream);
size_t onng_graph_add_edges_workspace_size(int64_t n, int64_t nnz, int64_t n_edges);

/* The first step of ConstructGraph (Algorithm 8, Section 2.6):
 * G_k = ConstructAdjustedGraph(G_a, k_c, 0), Algorithm 2 with e_i = 0, which
 * keeps the k = k_c shortest edges of every node of the graph (an ANNG) and
 * adds no reverse edge: the approximate k-NN graph (AKNNG) the degree
 * adjustments start from.  Output as the table they take: ids [n][k] and
 * dists [n][k] (device), row v = the first min(k, deg(v)) entries of v's
 * (length, id)-sorted list, padded with -1 and INT32_MAX (u8, squared L2) or
 * +inf.  Needs g->lens.  Asynchronous. */
onng_status onng_graph_head(const onng_graph *g, int32_t data_dtype, int32_t metric, int32_t k,
                            int32_t *ids, void *dists, void *stream);

/* ------------------------------------------------------------------------ */
/* Entry seeds from a tree — Section 3.2 (tree-based index), Table 5        */
/* ------------------------------------------------------------------------ */

/* A 4-way vantage-point tree over the base rows.  A node of m > leaf_size
 * rows takes its row of lowest (priority[row], row) as vantage point v; its
 * other m-1 rows, sorted by (d(v, x), x), are cut at floor(c (m-1) / 4),
 * c = 0..4, into four children, and node_mu[3 node + c - 1] is the distance
 * of child c's first row.  A node of at most leaf_size rows is a leaf; its
 * seeds are its n_seeds rows nearest its own vantage point, in (d, id)
 * order, padded with -1.  Nodes are numbered breadth first (root 0);
 * node_child[v] is the first of four consecutive children, or -1 - leaf.
 * Tree distances: exact on u8 (squared L2); on f32 rows (squared L2 or
 * cosine) fp32 in coordinate order, no fused multiply-add.  The paper's tree
 * has leaves of at most 100 rows and uses the 10 rows nearest a leaf's
 * vantage point as seeds; its fan-out is not stated, 4 gives the 6-8
 * distance computations per query of Table 5.
 * Device arrays are caller-owned with the stated capacities; node_capacity
 * = leaf_capacity = n always suffices. */
typedef struct {
    int32_t *node_vp;         /* [node_capacity] */
    int32_t *node_child;      /* [node_capacity] */
    void *node_mu;            /* [3 * node_capacity], distance type of the rows */
    int32_t *leaf_seeds;      /* [leaf_capacity * n_seeds] */
    int64_t node_capacity;
    int64_t leaf_capacity;
    int32_t leaf_size;        /* 4 .. 256 */
    int32_t n_seeds;          /* 1 .. 256 */
    int64_t n_nodes;          /* written by onng_vptree_build */
    int64_t n_leaves;         /* written by onng_vptree_build */
} onng_vptree;

/* Builds `tree` (a host struct; its arrays and counts are written) from
 * `base` (u8 with ONNG_L2SQ, or f32 with either metric) and one priority per
 * row (device [n]; a random permutation makes every vantage point a uniform
 * draw).  ONNG_ERR_CAPACITY when a capacity is too small.  Synchronises the
 * stream. */
onng_status onng_vptree_build(const onng_vectors *base, const uint32_t *priority,
                              onng_vptree *tree, void *ws, size_t ws_bytes, void *stream);
size_t onng_vptree_build_workspace_size(int64_t n);

/* Descends the tree for every query (same dtype, dim and metric as the
 * base): seeds [nq][n_seeds] (device) get the leaf's seeds, dc [nq] (device)
 * the distance computations spent (one per inner node).  A query whose
 * descent leaves the tree's counts (a tree not made by onng_vptree_build)
 * gets seeds -1 and dc -1. */
onng_status onng_vptree_seeds(const onng_vectors *base, const onng_vptree *tree,
                              const onng_vectors *queries, int32_t *seeds, int32_t *dc,
                              void *stream);

/* ------------------------------------------------------------------------ */
/* Search — Algorithm 1 (KnnSearch)                                         */
/* ------------------------------------------------------------------------ */

/* Optional learned search range: a 2-layer MLP (F -> H ReLU -> T heads)
 * evaluated on the state after the probe expansions.  Not part of the paper.
 *  mode 0 (ONNG_PRED_LOG_EPS): head `head` (or head_per_query[q]) predicts
 *    log10(eps + 0.01); eps = 10^(y + shift[head]) - 0.01.
 *  mode 1 (ONNG_PRED_CURVE): n_cand candidate ranges eps_cand[g]; head g
 *    predicts the query's recall at eps_cand[g] and head n_cand + g the
 *    log(1 + cost) there, the cost in distance-computation units (the count
 *    itself, or a search time scaled to it: the library only evaluates it);
 *    the query takes the candidate maximising
 *    recall_g - lambda * (exp(y_{n_cand+g}) - 1), with lambda from
 *    lambda_per_query[q] when given.  With max_dc_factor > 0 the budget
 *    after the switch is min(max_dc, max(64, int32(max_dc_factor * cost))).
 * Weights are bf16 (w1: [H][F], w2: [T][H]); biases, feature statistics,
 * shifts and candidates are f32.  The chosen eps is clamped to
 * [eps_min, eps_max]; e_p follows Equation 1 with (e0, we) unless we < 0. */
typedef struct {
    const uint16_t *w1_bf16;
    const float *b1;
    const uint16_t *w2_bf16;
    const float *b2;
    const float *feat_mean;        /* [F] z-scoring of the transformed features */
    const float *feat_std;         /* [F] */
    const float *shift;            /* [T] calibration shift added to each head (mode 0), or NULL */
    const int32_t *head_per_query; /* [nq] head index per query (mode 0), or NULL: use `head` */
    int32_t head;
    int32_t n_features;            /* must be ONNG_NFEAT */
    int32_t hidden;                /* <= 64 */
    int32_t n_heads;               /* <= 16 */
    float eps_min, eps_max;        /* predicted eps is clamped to this range */
    float e0, we;                  /* e_p = floor(10^(we*eps) + e0) (Equation 1); we < 0: use e_p */
    int32_t mode;                  /* ONNG_PRED_LOG_EPS or ONNG_PRED_CURVE */
    int32_t n_cand;                /* mode 1: candidates, n_heads = 2 * n_cand, <= 8 */
    const float *eps_cand;         /* mode 1: [n_cand] candidate search ranges */
    float lambda;                  /* mode 1: price of one unit of cost in recall */
    const float *lambda_per_query; /* mode 1: [nq] or NULL */
} onng_predictor;

#define ONNG_PRED_LOG_EPS 0
#define ONNG_PRED_CURVE 1
#define ONNG_NFEAT 14

struct onng_query_stats_s;

/* Launch shape of the search kernel (0 = library default for a field). */
typedef struct {
    int32_t waves_per_block;   /* 1..8 */
    int32_t lanes_per_row;     /* 4, 8, 16 or 32: lanes that share one vector */
    int32_t s_capacity;        /* candidate-set entries held on chip per query */
    int32_t visited_log2;      /* on-chip visited bits: 2^visited_log2 words covering a
                                  window of 32 * 2^visited_log2 ids around the first
                                  seed (other ids: a global bitset); negative = none */
    int32_t pool_capacity;     /* rerank pool entries held on chip per query */
    int32_t blocks;            /* persistent grid size; 0 = one wave per query */
} onng_launch_config;

typedef struct {
    int32_t k;                     /* results per query when k_per_query is NULL */
    int32_t k_stride;              /* row length of ids/dists, >= every k, <= 256 */
    const int32_t *k_per_query;    /* [nq] or NULL */
    float epsilon;                 /* search range eps when eps_per_query is NULL */
    const float *eps_per_query;    /* [nq] or NULL */
    uint32_t e_p;                  /* explored-edge limit when ep_per_query is NULL;
                                      0xFFFFFFFF = unlimited (Equation 1's e_p) */
    const uint32_t *ep_per_query;  /* [nq] or NULL */
    /* Two-phase mode: when two_phase != 0 the first probe_hops expansions
     * use an unlimited range and e_p = ep_first; the search range of every
     * later step comes from the predictor (if set) or from eps/e_p above.
     * Features at the switch: 0-7 the seed distances ascending (the last
     * repeated when fewer), 8 |S|, 9-11 the smallest, the ceil(m/2)-th and
     * the m-th smallest distance in S with m = min(|S|, 64) (all equal to
     * feature 12 when S is empty), 12 the largest distance in R, 13 the
     * distance computations so far. */
    int32_t two_phase;
    uint32_t ep_first;
    const onng_predictor *predictor;   /* requires two_phase */
    float *features_out;           /* [nq][ONNG_NFEAT] raw state after the probe
                                      expansions (two_phase only), or NULL */
    /* Rerank: search on the stored (possibly low-precision) rows, keep the
     * pool_factor*k best visited ids, recompute their distances from
     * rerank_base (f32 rows of the same objects) and return the best k. */
    const onng_vectors *rerank_base;   /* NULL = no rerank */
    int32_t pool_factor;
    const onng_launch_config *launch;  /* NULL = tuned or default shape */
    uint32_t probe_hops;           /* two_phase: expansions run with the unlimited range
                                      and e_p = ep_first before the switch (0 means 1) */
    /* Scheduling of a learned search in two passes:
     * predict_only != 0 (needs two_phase and a predictor): each query stops
     *   at the switch and only reports its eps, e_p and cost estimate in stats;
     * range_from: per-query eps and e_p taken from the stats of such a pass
     *   (overrides epsilon/e_p; two_phase must be 0);
     * order: [nq] permutation, the order in which the persistent waves take
     *   the queries (e.g. from onng_order_by_cost), or NULL for 0..nq-1. */
    int32_t predict_only;
    const struct onng_query_stats_s *range_from;
    const int32_t *order;
    /* Distance-computation budget (not in the paper): no expansion starts
     * once a query has made max_dc distance computations (seeds included);
     * the query then returns its current R and sets ONNG_QF_BUDGET.  0 = no
     * budget.  max_dc_per_query [nq] (or NULL) overrides it per query, values
     * <= 0 meaning none.  Bounds the latency of the rare queries whose range
     * holds very many objects. */
    int32_t max_dc;
    const int32_t *max_dc_per_query;
    /* With a learned range (range_from, or the predictor in curve mode):
     * when > 0, each query's budget is further limited to
     * max(64, (int32)(max_dc_factor * its predicted cost)), the cost in
     * distance-computation units and the product taken in fp32, so that a
     * query far costlier than predicted is cut short. */
    float max_dc_factor;
    /* Output ids are id_map[id] when non-NULL (e.g. the permutation of
     * onng_locality_order, to report original row ids). */
    const int32_t *id_map;
    /* Pipelines with a predictor (onng_pipeline_create): 0 = a predict-only
     * pass, longest-first ordering and the search (three steps); 1 = one
     * search with the predictor fused after the probe expansions. */
    int32_t single_pass;
    /* Workspace reuse.  Every onng_search leaves the visited bitsets of its
     * workspace all zero and records the layout they belong to in the
     * workspace.  ws_reuse = 1 vouches that nothing but onng_search calls has
     * written `ws` since the last onng_search on it: when the recorded layout
     * is this call's, the bitsets are trusted and not zeroed again.  0 (or a
     * fresh workspace): they are zeroed first (N/8 bytes per wave slot). */
    int32_t ws_reuse;
} onng_search_params;

/* Per-query statistics written by onng_search. */
typedef struct onng_query_stats_s {
    int32_t dc;        /* distance computations (seeds included) */
    int32_t hops;      /* expansions (pops that passed the range test) */
    int32_t flags;     /* ONNG_QF_* bits */
    uint32_t e_p;      /* explored-edge limit used after the probe expansions */
    float eps;         /* search range used after the probe expansions */
    int32_t scanned;   /* adjacency entries read: sum over expansions of min(deg, e_p) */
    float cost;        /* predicted distance computations of the chosen range
                          (curve predictor), else the range itself */
    float us;          /* wall time on the device from taking the query to its
                          last write, microseconds (for tail-latency analysis) */
} onng_query_stats;

#define ONNG_QF_PADDED 1      /* fewer than k results were reachable */
#define ONNG_QF_SPILLED 2     /* exceeded on-chip capacity, finished by the exact off-chip pass */
#define ONNG_QF_CAPACITY 4    /* exceeded even the off-chip capacity: result not exact */
#define ONNG_QF_BUDGET 8      /* stopped by the distance-computation budget */

/* Batched KnnSearch (Algorithm 1) for every query row: best-first expansion
 * from the seeds with search range r(1 + eps), at most e_p edges per node,
 * visited set C, result set R of size k (radius r).  Seeds: [nq][n_seeds]
 * node ids (duplicates and ids < 0 ignored); each seed is a distance
 * computation, is marked visited and is offered to R.  Outputs: ids
 * [nq][k_stride], dists [nq][k_stride] in the distance type (or f32 after a
 * rerank), ascending, padded with -1 / INT32_MAX or +inf; stats [nq].
 * With range factor f = (1+eps)^2 for ONNG_L2SQ and 1+eps for ONNG_COSINE
 * (rounded to f32), a node is pushed to the candidate set when
 * d <= f32(r * f) and the search stops when the nearest candidate is beyond it.
 * An adjacency list may repeat an id: only its first copy is visited (the
 * later ones still count towards e_p), as with Algorithm 1's visited set. */
onng_status onng_search(const onng_vectors *base, const onng_graph *graph,
                        const onng_vectors *queries, const int32_t *seeds, int32_t n_seeds,
                        const onng_search_params *params, int32_t *ids, void *dists,
                        onng_query_stats *stats, void *ws, size_t ws_bytes, void *stream);
size_t onng_search_workspace_size(const onng_vectors *base, int64_t n_queries,
                                  const onng_search_params *params);

/* onng_search for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, results and errors as onng_search, without the workspace; it
 * calls no hipMalloc, hipFree or allocating library routine.  Its scratch
 * (work counter, visited bitsets, visit logs, spill buffers) is one static
 * device array of ONNG_SEARCH_STATIC_SCRATCH_BYTES, a copy of which each
 * device the library runs on holds until the process ends.  The persistent
 * grid is cut to the wave slots that fit in it (results do not depend on
 * the slot count, throughput may drop); a base so large that one block of
 * slots does not fit returns ONNG_ERR_CAPACITY with nothing enqueued.  Every
 * call on a device shares that device's array and leaves its contents for
 * the next call: calls that overlap in time on one device (other streams or
 * threads) race on it and must not be issued. */
#define ONNG_SEARCH_STATIC_SCRATCH_BYTES ((size_t)128 << 20)
onng_status onng_search_static(const onng_vectors *base, const onng_graph *graph,
                               const onng_vectors *queries, const int32_t *seeds, int32_t n_seeds,
                               const onng_search_params *params, int32_t *ids, void *dists,
                               onng_query_stats *stats, void *stream);

/* order[0..n) = query indices by descending stats[q].cost (ties: ascending
 * index), so that a persistent search starts the most expensive queries
 * first and the batch ends when the cheap ones do (longest first).
 * ws: onng_order_by_cost_workspace_size(n) bytes. */
onng_status onng_order_by_cost(const onng_query_stats *stats, int64_t n, int32_t *order, void *ws,
                               size_t ws_bytes, void *stream);
size_t onng_order_by_cost_workspace_size(int64_t n);

/* Locality order of a base (not part of the paper; a memory layout for the
 * search): perm[0..n) lists the rows grouped by their nearest pivot (rows
 * ascending within a group), and the groups follow a hierarchical order of
 * the pivots, so that objects close in space get close positions.  Level 0
 * is `pivots` as given; level i + 1 is every 10th pivot of level i, up to the
 * first level with at most 16.  The top level keeps its given order; each
 * level below is ordered by (position of each pivot's nearest pivot of the
 * ordered level above, its own position); the rows likewise against the
 * ordered level 0.  Nearest means smallest (distance, id), as everywhere.
 * Searching rows gathered in this order touches fewer cache lines and fewer
 * words of the visited set per query.  pivots: [n_pivots] row ids of `base`
 * (device), n_pivots <= n.  ws: onng_locality_order_workspace_size.
 * A graph built on the reordered rows has reordered ids; search outputs are
 * mapped back with onng_search_params.id_map = perm. */
onng_status onng_locality_order(const onng_vectors *base, const int32_t *pivots,
                                int64_t n_pivots, int32_t *perm, void *ws, size_t ws_bytes,
                                void *stream);
size_t onng_locality_order_workspace_size(const onng_vectors *base, int64_t n_pivots);

/* dst row i = src row ids[i], for n rows of pitch_bytes (a multiple of 16;
 * any type; device).  Every ids[i] must be a row of src. */
onng_status onng_gather_rows(const void *src, int64_t pitch_bytes, const int32_t *ids, int64_t n,
                             void *dst, void *stream);

/* ------------------------------------------------------------------------ */
/* Low-precision storage and exact rerank (not part of the paper)           */
/* ------------------------------------------------------------------------ */

/* f32 rows [n][dim] (row stride dim) -> rows of `dtype`, dst_pitch bytes
 * apart, padding zero.  Round-to-nearest-even; FP8 saturates at +-448 after
 * dividing by the per-row scale maxabs/448 (scale 1 for an all-zero row),
 * written to `scale` [n], or, when scale is NULL, into the last 4 bytes of
 * each row (dst_pitch >= 16 * ceil(dim / 16) + 16). */
onng_status onng_encode(const float *src, int64_t n, int32_t dim, int32_t dtype, void *dst,
                        int64_t dst_pitch, float *scale, void *stream);

/* For each query the k best (d, id) among pool ids [nq][pool_size] (ids < 0
 * skipped), with distances recomputed from `base` in f32 (use_f64 = 0) or
 * f64 (use_f64 = 1).  dists: f32 or f64 [nq][k]. */
onng_status onng_rerank(const onng_vectors *queries, const onng_vectors *base,
                        const int32_t *pool, int32_t pool_size, int32_t k, int32_t use_f64,
                        int32_t *ids, void *dists, void *stream);

/* ------------------------------------------------------------------------ */
/* Learned search range: training kernels (not part of the paper)           */
/* ------------------------------------------------------------------------ */

/* Y = W2 relu(W1 X + b1) + b2, all f32 row-major; hidden [batch][H] optional.
 * H <= 64, T <= 16. */
onng_status onng_mlp_forward(const float *X, int32_t batch, int32_t F, const float *W1,
                             const float *b1, int32_t H, const float *W2, const float *b2,
                             int32_t T, float *hidden, float *Y, void *stream);
/* Gradients of mean(w * (Y - target)^2) over batch*T (w NULL = all ones) and
 * the loss itself (device scalar).  Sums over the batch run in a fixed order
 * (deterministic).  ws: onng_mlp_backward_workspace_size(batch, H, T) bytes. */
onng_status onng_mlp_backward(const float *X, const float *target, const float *w, int32_t batch,
                              int32_t F, const float *W1, const float *b1, int32_t H,
                              const float *W2, const float *b2, int32_t T, float *gW1,
                              float *gb1, float *gW2, float *gb2, float *loss, void *ws,
                              size_t ws_bytes, void *stream);
size_t onng_mlp_backward_workspace_size(int32_t batch, int32_t H, int32_t T);
/* One Adam step with bias correction (t >= 1). */
onng_status onng_adam_step(float *p, const float *g, float *m, float *v, int64_t n, float lr,
                           float beta1, float beta2, float eps, int32_t t, void *stream);
/* raw features [n][ONNG_NFEAT] -> predictor inputs, the transform the search
 * kernel applies before z-scoring. */
onng_status onng_feature_transform(const float *raw, int64_t n, int32_t metric, float *out,
                                   void *stream);
/* Training support of the learned range (not part of the paper).
 * onng_column_stats: mean[c] and std[c] of the columns of x [n][cols]
 * (device), weighted by w [n][cols] when w is not NULL: mean = sum(w x) /
 * sum(w), std = sqrt(sum(w (x - mean)^2) / sum(w)), sums in double; a std
 * below 1e-6 is stored as 1 (the z-score the predictor applies, and the
 * target scaling of training).  onng_standardize: out = (x - mean) / std per
 * column (out may alias x).  onng_mlp_fold_output: turns the output layer of
 * a network trained on targets (y - shift) / scale into the same network on
 * y: w2[t][h] *= scale[t], b2[t] = b2[t] * scale[t] + shift[t] (in place).
 * All asynchronous on the stream; ONNG_ERR_INVALID_ARG on negative sizes. */
onng_status onng_column_stats(const float *x, const float *w, int64_t n, int32_t cols,
                              float *mean, float *std_out, void *stream);
onng_status onng_standardize(const float *x, int64_t n, int32_t cols, const float *mean,
                             const float *std_in, float *out, void *stream);
onng_status onng_mlp_fold_output(float *w2, float *b2, int32_t T, int32_t H, const float *scale,
                                 const float *shift, void *stream);

/* ------------------------------------------------------------------------ */
/* Degree-parameter loss (Section 2.6, Equation 2)                          */
/* ------------------------------------------------------------------------ */

/* L of Equation 2 from n >= 1 measured samples (precision p[i], mean
 * distance computations c[i] > 0), host arrays: the samples sorted by
 * precision, the trapezoidal rule over log10 c, divided by the samples'
 * precision span (the printed normalisation by p_u - p_l, with the span the
 * bracketed searches actually reach); with a zero span, the mean of log10 c.
 * Host computation, no device work.  ONNG_ERR_INVALID_ARG when n < 1 or some
 * c[i] <= 0. */
onng_status onng_degree_loss(const double *p, const double *c, int32_t n, double *loss);

/* ------------------------------------------------------------------------ */
/* Launch tuning and graph capture (not part of the paper)                  */
/* ------------------------------------------------------------------------ */

/* Times candidate launch shapes of onng_search on the given calibration
 * batch and writes the fastest to *best (host).  Results are cached in host
 * memory per (dtype, dim, n, k_stride, rerank); *best is then returned at once. */
onng_status onng_autotune_search(const onng_vectors *base, const onng_graph *graph,
                                 const onng_vectors *queries, const int32_t *seeds,
                                 int32_t n_seeds, const onng_search_params *params,
                                 int32_t *ids, void *dists, onng_query_stats *stats, void *ws,
                                 size_t ws_bytes, void *stream, onng_launch_config *best);

/* Captures the query pipeline for a fixed batch into a HIP graph, returned
 * in *handle (host): seed selection against `pivots`, then the search and
 * rerank.  With a predictor the search runs as three steps (a predict-only
 * pass, onng_order_by_cost, and the search with the predicted ranges in that
 * order), or as one fused search when params->single_pass is set.  The
 * launch shape is params->launch, else the one onng_autotune_search cached
 * for this index and parameters, else the default.  All pointers must stay
 * valid while the handle lives, and `ws` belongs to the pipeline meanwhile:
 * its replays keep search state in it (params->ws_reuse is ignored). */
typedef struct onng_pipeline onng_pipeline;
onng_status onng_pipeline_create(const onng_vectors *base, const onng_graph *graph,
                                 const onng_vectors *queries, const int32_t *pivots,
                                 int64_t n_pivots, int32_t n_seeds, int32_t *seeds,
                                 const onng_search_params *params, int32_t *ids, void *dists,
                                 onng_query_stats *stats, void *ws, size_t ws_bytes,
                                 void *stream, onng_pipeline **handle);
size_t onng_pipeline_workspace_size(const onng_vectors *base, const onng_vectors *queries,
                                    int64_t n_pivots, int32_t n_seeds,
                                    const onng_search_params *params);
onng_status onng_pipeline_launch(onng_pipeline *handle, void *stream);
onng_status onng_pipeline_destroy(onng_pipeline *handle);

/* ------------------------------------------------------------------------ */
/* Diagnostics                                                              */
/* ------------------------------------------------------------------------ */

const char *onng_status_string(onng_status st);
const char *onng_last_error(void);          /* calling thread's last message */
int32_t onng_version(void);                 /* major*10000 + minor*100 + patch */

#ifdef __cplusplus
}
#endif
#endif /* ONNG_H */
