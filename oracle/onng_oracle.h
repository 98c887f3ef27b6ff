/*
 * Plain CPU oracle for the degree/path-adjusted kNN-graph search of
 * Iwasaki & Miyazaki, "Optimization of Indexing Based on k-Nearest Neighbor
 * Graph for Proximity Search in High-dimensional Data" (arXiv 1810.07355).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the HIP library under paper_1810_07355_amd/.
 *
 * Arithmetic: u8 distances are exact integers (accumulated in int64, held in
 * double, exact below 2^53).  Float data is decoded exactly to double and all
 * distances are computed in fp64.  The search-range threshold on u8 data is
 * an IEEE fp32 product, the precision in which the HIP kernels take the same
 * decision.
 *
 * Every function returns 0 on success, a negative value on bad arguments.
 */
#ifndef ONNG_ORACLE_H
#define ONNG_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_U8 = 0, OR_F32 = 1, OR_F16 = 2, OR_BF16 = 3, OR_FP8 = 4 };
enum { OR_L2SQ = 0, OR_COS = 1 };

typedef struct {
    const void *data;     /* n rows, each `pitch` bytes apart */
    const float *scale;   /* per-row scale (FP8 only), else NULL */
    int64_t n;
    int32_t dim;
    int64_t pitch;        /* bytes between rows */
    int32_t dtype;        /* OR_U8 ... OR_FP8 */
    int32_t metric;       /* OR_L2SQ or OR_COS */
} or_vecs;

/* ---- scalar codecs (exact decode; round-to-nearest-even encode) ---- */
double or_decode(int32_t dtype, uint32_t code);
uint32_t or_encode_f16(float x);
uint32_t or_encode_bf16(float x);
uint32_t or_encode_fp8(float x);           /* OCP e4m3fn, saturating */
/* Encode rows of fp32 into dtype, rows `dst_pitch` bytes apart, padding zero.
 * FP8 also writes a per-row scale maxabs/448 (1 if the row is all zero). */
int or_encode_rows(const float *src, int64_t n, int32_t dim, int32_t dtype,
                   void *dst, int64_t dst_pitch, float *scale);

/* ---- distances ---- */
double or_dist(const or_vecs *a, int64_t i, const or_vecs *b, int64_t j);

/* ---- exact top-k by the total order (distance, id) ---- */
/* For each query row r (q_rows[r], or r when q_rows is NULL), the k smallest
 * (d, j) over candidates j (cand[c], or every base row when cand is NULL),
 * skipping j == query row when exclude_self != 0.  Missing entries are
 * (-1, +inf). */
int or_topk(const or_vecs *Q, const int64_t *q_rows, int64_t nq,
            const or_vecs *B, const int32_t *cand, int64_t ncand,
            int32_t k, int32_t exclude_self,
            int32_t *out_ids, double *out_d, int32_t nthreads);

/* ---- Algorithm 2 (ConstructAdjustedGraph) ---- */
/* knn: n rows of k (id, dist) sorted by (dist, id).  Two calls: with
 * nbrs == NULL it only returns the edge count in *nnz_out. */
int or_adjust_degree(const int32_t *knn_ids, const double *knn_d, int64_t n,
                     int32_t k, int32_t e_o, int32_t e_i,
                     int64_t *offsets, int32_t *nbrs, double *lens,
                     int64_t nnz_cap, int64_t *nnz_out);

/* ---- Algorithm 3 (ConstructAdjustedGraphWithConstraint) ---- */
/* Same table and two-call protocol as or_adjust_degree.  G_t is Algorithm 2
 * with (0, e_i); nodes are taken in ascending (|N(G_t, x)|, x) (R10); the
 * inner loops take members in ascending (d, id).  Lists come out sorted by
 * (len, id).  Phase-1 lengths are G_t's (the row the reverse edge came from);
 * phase-2 lengths are the node's own row's. */
int or_adjust_degree_constrained(const int32_t *knn_ids, const double *knn_d, int64_t n,
                                 int32_t k, int32_t e_o, int32_t e_i,
                                 int64_t *offsets, int32_t *nbrs, double *lens,
                                 int64_t nnz_cap, int64_t *nnz_out);

/* ---- Tree-based seeds: 4-way vantage-point tree (Section 3.2, Table 5) ----
 * A node holding m > leaf_size rows takes its lowest-priority row (ties by
 * id) as vantage point; the other m-1 rows sorted by (d(vp, x), x) are cut
 * at floor(c (m-1) / 4), c = 0..4, into four children, and mu[c-1] is the
 * distance of child c's first row.  A node of at most leaf_size rows is a
 * leaf; its seeds are its n_seeds rows nearest its own vantage point (padded
 * with -1).  Nodes are numbered breadth first; node_child holds the first of
 * four consecutive children or -1 - leaf.  A query takes child
 * #{c : d(q, vp) >= mu[c]} at every inner node (one distance computation
 * each).  f32 distances are fp32 in coordinate order; u8 exact. */
int or_vptree_build(const or_vecs *B, const uint32_t *prio, int32_t leaf_size, int32_t n_seeds,
                    int32_t *node_vp, int32_t *node_child, double *node_mu,
                    int32_t *leaf_seeds, int64_t *n_nodes, int64_t *n_leaves);
int or_vptree_seeds(const or_vecs *B, const or_vecs *Q, int64_t nq, const int32_t *node_vp,
                    const int32_t *node_child, const double *node_mu,
                    const int32_t *leaf_seeds, int32_t n_seeds, int32_t *seeds, int32_t *dc);

/* ---- Algorithms 4 and 5 (AdjustPath, HasPath) ---- */
int or_adjust_path(const int64_t *in_off, const int32_t *in_nbrs,
                   const double *in_lens, int64_t n,
                   int64_t *out_off, int32_t *out_nbrs, double *out_lens,
                   int64_t *nnz_out);

/* ---- Algorithm 1 (KnnSearch) with the visited set of Algorithms 6/7 ---- */
/* Per query q: k[q], search range eps[q] and explored-edge limit ep[q] (UINT32_MAX
 * = unlimited).  When eps1/ep1 are non-NULL the first probe_hops expansions use
 * (eps1[q], ep1[q]) and every later step uses (eps[q], ep[q]).
 * Outputs: ids/dists rows of k_stride (padded -1/+inf), distance computations,
 * expansions, and the smallest relative decision margin seen (float data).
 * feat (optional, nq x OR_NFEAT) receives the state at the switch: 8 seed
 * distances ascending, |S|, the smallest / ceil(m/2)-th / m-th distance of the
 * m = min(|S|, 64) smallest in S, the largest distance in R, the distance
 * computations so far.
 * max_dc (optional, per query; <= 0 = none): a distance-computation budget,
 * an addition to the paper: before each pop, a query that has made max_dc[q]
 * or more distance computations stops and returns its current R.
 * pool_k > 0 (an addition for the rerank of low-precision rows): pool_ids /
 * pool_d [nq][pool_k] receive the pool_k smallest (d, id) over every distance
 * the search computed (seeds and visited nodes), ascending, padded -1/+inf;
 * like R this set does not depend on the order of the visits.  pool_margin
 * (optional, [nq]) the relative gap between the pool_k-th and the next
 * computed distance (+inf when fewer were computed).
 * probe_only != 0 (needs eps1/ep1): stop at the switch after the probe
 * expansions, as a pass that only predicts the range does; the outputs and
 * the margin then describe that state. */
#define OR_NFEAT 14
int or_search(const or_vecs *base, const int64_t *offsets, const int32_t *nbrs,
              int64_t n_nodes, const or_vecs *queries, int64_t nq,
              const int32_t *seeds, int32_t n_seeds,
              const int32_t *k, const float *eps, const uint32_t *ep,
              const float *eps1, const uint32_t *ep1, int32_t probe_hops,
              const int32_t *max_dc, int32_t k_stride, int32_t *out_ids, double *out_d,
              int64_t *out_dc, int64_t *out_hops, double *out_margin,
              double *feat, int32_t pool_k, int32_t *pool_ids, double *pool_d,
              double *pool_margin, int32_t probe_only, int32_t nthreads);

/* Visited-node table of Algorithms 6/7, exposed for tests. */
int64_t or_hash_size(int64_t n, int32_t b);
/* Replays ops (id >= 0: Set(id); id < 0: IsSet(-id-1)) and writes the IsSet
 * answers (1/0) for the IsSet ops, in order. */
int or_visited_replay(int64_t n, const int64_t *ops, int64_t nops, int32_t *answers);

/* ---- exact rerank of a candidate pool ---- */
int or_rerank(const or_vecs *Q, const or_vecs *B, const int32_t *pool, int32_t pool_sz,
              int64_t nq, int32_t k, int32_t *out_ids, double *out_d);

/* ---- 2-layer MLP (F -> H ReLU -> T), fp64 ---- */
int or_mlp_forward(const double *X, int32_t batch, int32_t F,
                   const double *W1, const double *b1, int32_t H,
                   const double *W2, const double *b2, int32_t T,
                   double *hidden, double *Y);
/* Mean of w*(y-t)^2 over batch*T; gradients of that loss. */
double or_mlp_loss_grad(const double *X, const double *target, const double *w,
                        int32_t batch, int32_t F,
                        const double *W1, const double *b1, int32_t H,
                        const double *W2, const double *b2, int32_t T,
                        double *gW1, double *gb1, double *gW2, double *gb2);
void or_adam_step(double *p, const double *g, double *m, double *v, int64_t n,
                  double lr, double beta1, double beta2, double eps, int32_t t);

#ifdef __cplusplus
}
#endif
#endif
