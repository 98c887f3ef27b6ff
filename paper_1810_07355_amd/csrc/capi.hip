// C-ABI entry points: argument validation, launch shapes, workspace layout,
// launch tuning and graph capture.  Kernels live in the other sources.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include <hipcub/hipcub.hpp>

#include "onng_internal.h"
#include "search_args.h"

namespace onng {

// kernels implemented elsewhere
onng_status adjust_degree_launch(const int32_t *knn, const void *kd, int64_t n, int32_t k,
                                 bool int_len, int32_t e_o, int32_t e_i, int64_t *offsets,
                                 int32_t *nbrs, void *lens, int64_t nnz_cap, int64_t *nnz_out,
                                 void *ws, hipStream_t st);
size_t adjust_degree_ws(int64_t n, int32_t k, int32_t e_o, int32_t e_i);
onng_status adjust_degree_constrained_launch(const int32_t *knn, const void *kd, int64_t n,
                                             int32_t k, bool int_len, int32_t e_o, int32_t e_i,
                                             int64_t *offsets, int32_t *nbrs, void *lens,
                                             int64_t nnz_cap, int64_t *nnz_out, void *ws,
                                             hipStream_t st);
size_t adjust_degree_constrained_ws(int64_t n, int32_t k, int32_t e_o, int32_t e_i);
onng_status graph_stats_launch(const onng_graph *g, bool int_len, bool sqrt_len, double frac,
                               int keep, double *out, void *ws, hipStream_t st);
size_t graph_stats_ws(int64_t n, int64_t nnz);
onng_status vptree_build_launch(const onng_vectors *base, const uint32_t *prio, onng_vptree *t,
                                void *ws, hipStream_t st);
onng_status vptree_seeds_launch(const onng_vectors *base, const onng_vptree *t,
                                const onng_vectors *q, int32_t *seeds, int32_t *dc,
                                hipStream_t st);
size_t vptree_ws(int64_t n);
onng_status add_edges_launch(const onng_graph *g, const int32_t *src, const int32_t *dst,
                             const void *len, int64_t m, bool int_len, int64_t *out_off,
                             int32_t *out_nb, void *out_len, int64_t nnz_cap, int64_t *nnz_out,
                             void *ws, hipStream_t st);
size_t add_edges_ws(int64_t n, int64_t nnz, int64_t m);
onng_status graph_head_launch(const onng_graph *g, bool int_len, int32_t k, int32_t *ids,
                              void *dists, hipStream_t st);
onng_status adjust_path_launch(const onng_graph *g, bool int_len, int64_t *offsets,
                               int32_t *nbrs, void *lens, int64_t *nnz_out, void *ws,
                               hipStream_t st);
size_t adjust_path_ws(int64_t n, int64_t nnz);
onng_status encode_launch(const float *src, int64_t n, int32_t dim, int32_t dtype, void *dst,
                          int64_t pitch, float *scale, hipStream_t st);
onng_status rerank_launch(const onng_vectors *Q, const onng_vectors *B, const int32_t *pool,
                          int32_t psz, int32_t k, int32_t use_f64, int32_t *ids, void *dists,
                          hipStream_t st);
size_t mlp_backward_ws(int32_t batch, int32_t H, int32_t T);
onng_status mlp_forward_launch(const float *X, int32_t batch, int32_t F, const float *W1,
                               const float *b1, int32_t H, const float *W2, const float *b2,
                               int32_t T, float *hidden, float *Y, hipStream_t st);
onng_status mlp_backward_launch(const float *X, const float *target, const float *w,
                                int32_t batch, int32_t F, const float *W1, const float *b1,
                                int32_t H, const float *W2, const float *b2, int32_t T,
                                float *gW1, float *gb1, float *gW2, float *gb2, float *loss,
                                void *ws, hipStream_t st);
onng_status adam_launch(float *p, const float *g, float *m, float *v, int64_t n, float lr,
                        float b1, float b2, float eps, int32_t t, hipStream_t st);
onng_status column_stats_launch(const float *x, const float *w, int64_t n, int32_t cols,
                                float *mean, float *stdv, hipStream_t st);
onng_status standardize_launch(const float *x, int64_t n, int32_t cols, const float *mean,
                               const float *stdv, float *out, hipStream_t st);
onng_status fold_output_launch(float *w2, float *b2, int32_t T, int32_t H, const float *scale,
                               const float *shift, hipStream_t st);
onng_status feature_transform_launch(const float *raw, int64_t n, int32_t metric, float *out,
                                     hipStream_t st);

static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }
const char *get_error() { return g_err.c_str(); }

int device_cu_count() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 256;
    return cus > 0 ? cus : 256;
}

// period of the device's constant-rate wall clock (wall_clock64) in microseconds
float device_us_per_tick() {
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0.0f;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
        return 0.0f;
    return 1000.0f / (float)khz;
}

onng_status check_vectors(const onng_vectors *v, const char *what) {
    std::string w(what);
    if (!v) { set_error(w + " is null"); return ONNG_ERR_INVALID_ARG; }
    if (v->n < 0 || v->dim <= 0) { set_error(w + ": bad n or dim"); return ONNG_ERR_INVALID_ARG; }
    if (v->n > 0 && !v->data) { set_error(w + ": data is null"); return ONNG_ERR_INVALID_ARG; }
    if (v->dtype < ONNG_U8 || v->dtype > ONNG_FP8_E4M3) {
        set_error(w + ": unknown dtype");
        return ONNG_ERR_INVALID_ARG;
    }
    if (v->metric != ONNG_L2SQ && v->metric != ONNG_COSINE) {
        set_error(w + ": unknown metric");
        return ONNG_ERR_INVALID_ARG;
    }
    if (v->pitch_bytes < (int64_t)v->dim * elem_bytes(v->dtype) || v->pitch_bytes % 16 != 0) {
        set_error(w + ": pitch_bytes must be a multiple of 16 and hold dim elements");
        return ONNG_ERR_INVALID_ARG;
    }
    if (reinterpret_cast<uintptr_t>(v->data) % 16 != 0) {
        set_error(w + ": data must be 16-byte aligned");
        return ONNG_ERR_INVALID_ARG;
    }
    if (v->dtype == ONNG_FP8_E4M3 && !v->scale && v->pitch_bytes < fp8_inrow_pitch(v->dim)) {
        set_error(w + ": FP8 rows need a scale array or room for the scale in the row");
        return ONNG_ERR_INVALID_ARG;
    }
    if (v->dtype == ONNG_U8 && v->metric != ONNG_L2SQ) {
        set_error(w + ": u8 data supports squared L2 only");
        return ONNG_ERR_UNSUPPORTED;
    }
    if (v->n > 0x7fffffffLL) { set_error(w + ": more than 2^31-1 rows"); return ONNG_ERR_UNSUPPORTED; }
    return ONNG_OK;
}

#define ONNG_TRY(x)                        \
    do {                                   \
        onng_status s_ = (x);              \
        if (s_ != ONNG_OK) return s_;      \
    } while (0)

// ------------------------------------------------------------- search -----

struct SearchPlan {
    const void *fn = nullptr;
    int L = 8, s_cap = 256, vis_log2 = 11, pool_cap = 64, wpb = 4, blocks = 0;
    int lds_per_wave = 0;
    int off_pool, off_s, off_stage, off_stage2, off_ids, off_vis, off_misc;
    int64_t gbits_words = 0;
    int vlog_cap = 16384, spill_cap = 8192;
    int slots = 0;
    size_t ws = 0;
};

// 16-byte pieces of a row per lane (matches the search kernel's query registers)
static int ppl_for(int) { return 2; }

static int align16(int x) { return (x + 15) / 16 * 16; }

// 16-byte pieces that hold a row's components (rows may be padded further,
// e.g. to whole cache lines; the padding is zero and never read)
static int row_pieces(const onng_vectors *v) {
    return (int)(((int64_t)v->dim * elem_bytes(v->dtype) + 15) / 16);
}

static onng_status make_plan(const onng_vectors *base, int64_t nq, const onng_search_params *p,
                             const onng_launch_config *cfg, SearchPlan *plan) {
    SearchPlan P;
    P.fn = search_kernel_ptr(base->dtype, base->metric);
    if (!P.fn) {
        set_error("onng_search: unsupported dtype/metric");
        return ONNG_ERR_UNSUPPORTED;
    }
    const int n16 = row_pieces(base);
    const int ppl = ppl_for(base->dtype);
    int L = cfg && cfg->lanes_per_row ? cfg->lanes_per_row : 0;
    if (!L) {
        L = 4;
        while (L < 32 && (n16 + L - 1) / L > std::min(ppl, 2)) L <<= 1;
    }
    if (L != 4 && L != 8 && L != 16 && L != 32) {
        set_error("onng_search: lanes_per_row must be 4, 8, 16 or 32");
        return ONNG_ERR_INVALID_ARG;
    }
    if ((n16 + L - 1) / L > ppl) {
        set_error("onng_search: row too wide for lanes_per_row (use more lanes per row)");
        return ONNG_ERR_UNSUPPORTED;
    }
    P.L = L;
    P.s_cap = cfg && cfg->s_capacity ? cfg->s_capacity : 256;
    // the fused rerank collects its k best in the candidate array
    if (p->rerank_base) P.s_cap = std::max(P.s_cap, (p->k_stride + 63) / 64 * 64);
    P.vis_log2 = cfg && cfg->visited_log2 >= 0 && cfg->visited_log2 != 0 ? cfg->visited_log2 : 11;
    if (cfg && cfg->visited_log2 < 0) P.vis_log2 = 0;   // negative: global bitset only
    if (P.s_cap < 64 || P.s_cap % 64 || P.s_cap > 8192) {
        set_error("onng_search: s_capacity must be a multiple of 64 in [64, 8192]");
        return ONNG_ERR_INVALID_ARG;
    }
    if (P.vis_log2 != 0 && (P.vis_log2 < 8 || P.vis_log2 > 15)) {
        set_error("onng_search: visited_log2 must be in [8, 15] (or negative for off-chip)");
        return ONNG_ERR_INVALID_ARG;
    }
    int want_pool = p->k_stride;
    if (p->rerank_base) want_pool = std::max(p->k_stride, p->pool_factor * p->k_stride);
    if (cfg && cfg->pool_capacity) want_pool = std::max(want_pool, cfg->pool_capacity);
    P.pool_cap = (want_pool + 63) / 64 * 64;
    if (P.pool_cap > 1024) {
        set_error("onng_search: pool (k_stride * pool_factor) above 1024");
        return ONNG_ERR_UNSUPPORTED;
    }
    P.wpb = cfg && cfg->waves_per_block ? cfg->waves_per_block : 4;
    if (P.wpb < 1 || P.wpb > 8) {
        set_error("onng_search: waves_per_block must be in [1, 8]");
        return ONNG_ERR_INVALID_ARG;
    }
    int o = 0;
    P.off_pool = o; o = align16(o + P.pool_cap * 8);
    P.off_s = o; o = align16(o + P.s_cap * 8);
    P.off_stage = o; o = align16(o + 64 * 8);
    P.off_stage2 = o; o = align16(o + 64 * 8);
    P.off_ids = o; o = align16(o + 128 * 4);
    P.off_vis = o; o = align16(o + (P.vis_log2 ? (4 << P.vis_log2) : 0));
    P.off_misc = o; o = align16(o + 168 * 4);
    P.lds_per_wave = o;
    // the kernel uses the two stages as one 128-key buffer
    if (P.off_stage2 != P.off_stage + 64 * 8) {
        set_error("onng_search: internal LDS layout");
        return ONNG_ERR_UNSUPPORTED;
    }
    size_t lds = (size_t)o * P.wpb;
    if (lds > 160 * 1024) {
        set_error("onng_search: on-chip state above 160 KiB per block");
        return ONNG_ERR_UNSUPPORTED;
    }
    if (hipFuncSetAttribute(P.fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
        hipSuccess) {
        set_error("onng_search: cannot set shared memory size");
        return ONNG_ERR_DEVICE;
    }
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, P.fn, P.wpb * 64, lds) !=
            hipSuccess ||
        per_cu <= 0)
        per_cu = 1;
    int want = cfg && cfg->blocks ? cfg->blocks : per_cu * device_cu_count();
    int need = (int)std::min<int64_t>((nq + P.wpb - 1) / P.wpb, 1 << 20);
    P.blocks = std::max(1, std::min(want, std::max(need, 1)));
    P.slots = P.blocks * P.wpb;
    // a slot's bitset starts on a 128-byte line
    P.gbits_words = ((base->n + 31) / 32 + 31) / 32 * 32;
    Carver c(nullptr);
    c.take<int32_t>(64);
    c.take<uint32_t>((size_t)P.slots * P.gbits_words);
    c.take<int32_t>((size_t)P.slots * P.vlog_cap);
    c.take<uint64_t>((size_t)P.slots * 2 * P.spill_cap);
    P.ws = c.size() + 256;
    *plan = P;
    return ONNG_OK;
}

static onng_status validate_search(const onng_vectors *base, const onng_graph *g,
                                   const onng_vectors *queries, const int32_t *seeds,
                                   int32_t n_seeds, const onng_search_params *p) {
    ONNG_TRY(check_vectors(base, "base"));
    ONNG_TRY(check_vectors(queries, "queries"));
    ONNG_CHECK_ARG(p, "params is null");
    ONNG_CHECK_ARG(g && g->offsets && (g->nbrs || g->nnz == 0), "graph is null");
    ONNG_CHECK_ARG(g->n == base->n, "graph and base sizes differ");
    ONNG_CHECK_ARG(queries->dim == base->dim, "query and base dims differ");
    ONNG_CHECK_ARG(queries->metric == base->metric, "query and base metrics differ");
    if (base->dtype == ONNG_U8) ONNG_CHECK_ARG(queries->dtype == ONNG_U8, "u8 base needs u8 queries");
    else ONNG_CHECK_ARG(queries->dtype == ONNG_F32, "float base needs f32 queries");
    ONNG_CHECK_ARG(base->n > 0, "empty base");
    ONNG_CHECK_ARG(seeds || queries->n == 0, "seeds is null");
    ONNG_CHECK_ARG(n_seeds >= 1 && n_seeds <= 64, "n_seeds must be in [1, 64]");
    ONNG_CHECK_ARG(p->k_stride >= 1 && p->k_stride <= 256, "k_stride must be in [1, 256]");
    ONNG_CHECK_ARG(p->k_per_query || (p->k >= 1 && p->k <= p->k_stride), "k must be in [1, k_stride]");
    ONNG_CHECK_ARG(p->eps_per_query || p->epsilon >= 0.0f, "epsilon must be >= 0");
    ONNG_CHECK_ARG(p->ep_per_query || p->e_p >= 1, "e_p must be >= 1");
    if (p->rerank_base) {
        ONNG_TRY(check_vectors(p->rerank_base, "rerank_base"));
        ONNG_CHECK_ARG(base->dtype != ONNG_U8, "rerank needs float data");
        ONNG_CHECK_ARG(p->rerank_base->dtype == ONNG_F32 && p->rerank_base->n == base->n &&
                           p->rerank_base->dim == base->dim,
                       "rerank_base must be f32 rows of the same objects");
        ONNG_CHECK_ARG(p->pool_factor >= 1, "pool_factor must be >= 1");
    }
    if (p->predictor) {
        const onng_predictor *pr = p->predictor;
        ONNG_CHECK_ARG(p->two_phase, "a predictor needs two_phase");
        ONNG_CHECK_ARG(pr->n_features == ONNG_NFEAT, "predictor n_features must be ONNG_NFEAT");
        ONNG_CHECK_ARG(pr->hidden >= 1 && pr->hidden <= 64, "predictor hidden must be in [1, 64]");
        ONNG_CHECK_ARG(pr->n_heads >= 1 && pr->n_heads <= 16, "predictor n_heads must be in [1, 16]");
        ONNG_CHECK_ARG(pr->mode == ONNG_PRED_LOG_EPS || pr->mode == ONNG_PRED_CURVE,
                       "unknown predictor mode");
        if (pr->mode == ONNG_PRED_CURVE)
            ONNG_CHECK_ARG(pr->n_cand >= 1 && pr->n_cand <= 8 && pr->n_heads == 2 * pr->n_cand &&
                               pr->eps_cand,
                           "curve predictor needs n_cand in [1, 8], n_heads = 2 n_cand, eps_cand");
        ONNG_CHECK_ARG(pr->w1_bf16 && pr->b1 && pr->w2_bf16 && pr->b2 && pr->feat_mean && pr->feat_std,
                       "predictor weights missing");
        ONNG_CHECK_ARG(pr->mode == ONNG_PRED_CURVE || pr->head_per_query ||
                           (pr->head >= 0 && pr->head < pr->n_heads),
                       "predictor head out of range");
        ONNG_CHECK_ARG(pr->eps_min >= 0.0f && pr->eps_max >= pr->eps_min, "bad eps clamp");
    }
    if (p->two_phase) ONNG_CHECK_ARG(p->ep_first >= 1, "ep_first must be >= 1");
    if (p->predict_only)
        ONNG_CHECK_ARG(p->two_phase && p->predictor, "predict_only needs two_phase and a predictor");
    if (p->range_from)
        ONNG_CHECK_ARG(!p->two_phase, "range_from replaces the two-phase range; set two_phase = 0");
    return ONNG_OK;
}

// Tag of a workspace layout (slot count and per-slot region sizes); never 0.
static uint64_t search_ws_tag(const SearchPlan &P) {
    uint64_t h = 0x6f6e6e6773656172ull;
    for (uint64_t v : {(uint64_t)P.slots, (uint64_t)P.gbits_words, (uint64_t)P.vlog_cap,
                       (uint64_t)P.spill_cap}) {
        h ^= v + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
        h *= 0xbf58476d1ce4e5b9ull;
    }
    return h | 1ull;
}

// reuse_override: -1 takes params->ws_reuse, 0/1 force it (the static
// scratch is only ever written by searches).
static onng_status run_search(const onng_vectors *base, const onng_graph *g,
                              const onng_vectors *queries, const int32_t *seeds, int32_t n_seeds,
                              const onng_search_params *p, int32_t *ids, void *dists,
                              onng_query_stats *stats, void *ws, size_t ws_bytes, hipStream_t st,
                              const onng_launch_config *cfg, int reuse_override = -1) {
    ONNG_TRY(validate_search(base, g, queries, seeds, n_seeds, p));
    ONNG_CHECK_ARG(ids && dists && stats, "outputs are null");
    if (queries->n == 0) return ONNG_OK;
    SearchPlan P;
    ONNG_TRY(make_plan(base, queries->n, p, cfg, &P));

    if (!ws || ws_bytes < P.ws) {
        set_error("onng_search: workspace too small (" + std::to_string(P.ws) + " bytes needed)");
        return ONNG_ERR_WORKSPACE;
    }
    Carver c(ws);
    SearchKArgs a{};
    a.counter = c.take<int32_t>(64);
    a.ws_tag_at = reinterpret_cast<uint64_t *>(a.counter + 2);
    a.ws_tag = search_ws_tag(P);
    a.ws_reuse = reuse_override >= 0 ? reuse_override : p->ws_reuse;
    a.gbits = c.take<uint32_t>((size_t)P.slots * P.gbits_words);
    a.vlog = c.take<int32_t>((size_t)P.slots * P.vlog_cap);
    a.spill = c.take<uint64_t>((size_t)P.slots * 2 * P.spill_cap);
    a.base = static_cast<const uint8_t *>(base->data);
    a.base_scale = base->scale;
    a.scale_in_row = base->dtype == ONNG_FP8_E4M3 && !base->scale;
    a.base_pitch = base->pitch_bytes;
    a.n_base = base->n;
    a.dim = base->dim;
    a.n16 = row_pieces(base);
    a.offsets = g->offsets;
    a.nbrs = g->nbrs;
    a.qry = static_cast<const uint8_t *>(queries->data);
    a.q_pitch = queries->pitch_bytes;
    a.nq = (int32_t)queries->n;
    a.seeds = seeds;
    a.n_seeds = n_seeds;
    a.k = p->k;
    a.k_pq = p->k_per_query;
    a.k_stride = p->k_stride;
    a.eps = p->epsilon;
    a.eps_pq = p->eps_per_query;
    a.ep = p->e_p;
    a.ep_pq = p->ep_per_query;
    a.two_phase = p->two_phase;
    a.ep_first = p->ep_first;
    a.probe_hops = p->probe_hops ? p->probe_hops : 1;
    a.predict_only = p->predict_only;
    a.us_per_tick = device_us_per_tick();
    a.range_from = p->range_from;
    a.order = p->order;
    a.max_dc = p->max_dc;
    a.max_dc_pq = p->max_dc_per_query;
    a.max_dc_factor = p->max_dc_factor;
    a.id_map = p->id_map;
    a.has_pred = p->predictor != nullptr;
    if (p->predictor) {
        const onng_predictor *pr = p->predictor;
        a.pred.w1 = pr->w1_bf16;
        a.pred.b1 = pr->b1;
        a.pred.w2 = pr->w2_bf16;
        a.pred.b2 = pr->b2;
        a.pred.mean = pr->feat_mean;
        a.pred.stdv = pr->feat_std;
        a.pred.shift = pr->shift;
        a.pred.head_pq = pr->head_per_query;
        a.pred.head = pr->head;
        a.pred.F = pr->n_features;
        a.pred.H = pr->hidden;
        a.pred.T = pr->n_heads;
        a.pred.eps_min = pr->eps_min;
        a.pred.eps_max = pr->eps_max;
        a.pred.e0 = pr->e0;
        a.pred.we = pr->we;
        a.pred.mode = pr->mode;
        a.pred.n_cand = pr->n_cand;
        a.pred.eps_cand = pr->eps_cand;
        a.pred.lambda = pr->lambda;
        a.pred.lambda_pq = pr->lambda_per_query;
    }
    a.feat_out = p->two_phase ? p->features_out : nullptr;
    a.has_rr = p->rerank_base != nullptr;
    if (a.has_rr) {
        a.rr_base = static_cast<const uint8_t *>(p->rerank_base->data);
        a.rr_pitch = p->rerank_base->pitch_bytes;
        a.pool_factor = p->pool_factor;
    }
    a.out_ids = ids;
    a.out_d = dists;
    a.stats = stats;
    a.gbits_words = P.gbits_words;
    a.vlog_cap = P.vlog_cap;
    a.spill_cap = P.spill_cap;
    a.lanes_per_row = P.L;
    a.s_cap = P.s_cap;
    a.vis_log2 = P.vis_log2;
    a.pool_cap = P.pool_cap;
    a.waves_per_block = P.wpb;
    a.lds_per_wave = P.lds_per_wave;
    a.off_pool = P.off_pool;
    a.off_s = P.off_s;
    a.off_stage = P.off_stage;
    a.off_stage2 = P.off_stage2;
    a.off_ids = P.off_ids;
    a.off_vis = P.off_vis;
    a.off_misc = P.off_misc;
    void *cargs[] = {&a.counter};
    ONNG_HIP(hipLaunchKernel(reset_counter_kernel_ptr(), dim3(1), dim3(1), cargs, 0, st));
    void *args[] = {&a};
    ONNG_HIP(hipLaunchKernel(P.fn, dim3(P.blocks), dim3(P.wpb * 64), args,
                             (size_t)P.lds_per_wave * P.wpb, st));
    return ONNG_OK;
}

// ----------------------------------------------------------- autotune -----

typedef std::tuple<int, int, int, int64_t, int, int, int> TuneKey;
static std::mutex g_tune_mu;
static std::map<TuneKey, onng_launch_config> g_tune;

static bool lookup_tuned(const onng_vectors *base, const onng_search_params *p,
                         onng_launch_config *out) {
    TuneKey key{base->dtype, base->metric, base->dim, base->n, p->k_stride,
                p->rerank_base ? p->pool_factor : 0, p->two_phase};
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    if (it == g_tune.end()) return false;
    *out = it->second;
    return true;
}

// ----------------------------------------------------- order by cost -----

__global__ void cost_keys_kernel(const onng_query_stats *st, int64_t n, float *cost, int32_t *idx) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    cost[i] = st[i].cost;
    idx[i] = (int32_t)i;
}

static size_t sort_temp_bytes(int64_t n) {
    size_t bytes = 0;
    (void)hipcub::DeviceRadixSort::SortPairsDescending(nullptr, bytes, (const float *)nullptr,
                                                       (float *)nullptr, (const int32_t *)nullptr,
                                                       (int32_t *)nullptr, (int)n);
    return bytes;
}

static size_t order_ws(int64_t n) {
    Carver c(nullptr);
    c.take<float>(n);
    c.take<float>(n);
    c.take<int32_t>(n);
    c.take<char>(sort_temp_bytes(n));
    return c.size() + 256;
}

static onng_status order_launch(const onng_query_stats *st, int64_t n, int32_t *order, void *ws,
                                size_t ws_bytes, hipStream_t s) {
    if (n == 0) return ONNG_OK;
    if (!ws || ws_bytes < order_ws(n)) {
        set_error("onng_order_by_cost: workspace too small");
        return ONNG_ERR_WORKSPACE;
    }
    Carver c(ws);
    float *cost = c.take<float>(n);
    float *cost_sorted = c.take<float>(n);
    int32_t *idx = c.take<int32_t>(n);
    size_t tb = sort_temp_bytes(n);
    void *tmp = c.take<char>(tb);
    hipLaunchKernelGGL(cost_keys_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, st, n,
                       cost, idx);
    ONNG_HIP(hipcub::DeviceRadixSort::SortPairsDescending(tmp, tb, cost, cost_sorted, idx, order,
                                                          (int)n, 0, 32, s));
    ONNG_HIP(hipGetLastError());
    return ONNG_OK;
}

// ------------------------------------------------------ locality order ---

// key[i] = position of row i's nearest pivot in the ordered pivot list
__global__ void nearest_key_kernel(const int32_t *nn, int64_t n, const int32_t *pos_of,
                                   uint32_t *key, int32_t *idx) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    key[i] = (uint32_t)pos_of[nn[i]];
    idx[i] = (int32_t)i;
}

// pos_of[ids[j]] = j
__global__ void position_kernel(const int32_t *ids, int64_t m, int32_t *pos_of) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < m) pos_of[ids[j]] = (int32_t)j;
}

// dst[j] = src[j * stride]
__global__ void strided_kernel(const int32_t *src, int64_t m, int stride, int32_t *dst) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < m) dst[j] = src[j * stride];
}

// dst[j] = src[idx[j]]
__global__ void permute_kernel(const int32_t *src, const int32_t *idx, int64_t m, int32_t *dst) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < m) dst[j] = src[idx[j]];
}

__global__ void gather_bytes_kernel(const uint8_t *src, int64_t pitch, const int32_t *ids,
                                    int64_t n, uint8_t *dst) {
    int64_t i = blockIdx.x;
    if (i >= n) return;
    const uint8_t *s = src + (int64_t)ids[i] * pitch;
    uint8_t *d = dst + i * pitch;
    for (int64_t c = threadIdx.x * 16; c < pitch; c += blockDim.x * 16)
        *reinterpret_cast<uint4 *>(d + c) = *reinterpret_cast<const uint4 *>(s + c);
}

static size_t locality_sort_bytes(int64_t n) {
    size_t bytes = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, (const uint32_t *)nullptr,
                                             (uint32_t *)nullptr, (const int32_t *)nullptr,
                                             (int32_t *)nullptr, (int)n);
    return bytes;
}

// Pivot levels of the locality order: level 0 is the given pivots, level
// i + 1 every LOC_STRIDE-th pivot of level i, up to the first level with at
// most LOC_TOP pivots.
constexpr int LOC_STRIDE = 10, LOC_TOP = 16;

static std::vector<int64_t> locality_levels(int64_t n_pivots) {
    std::vector<int64_t> sz{n_pivots};
    while (sz.back() > LOC_TOP) sz.push_back((sz.back() + LOC_STRIDE - 1) / LOC_STRIDE);
    return sz;
}

// top-k workspace of the largest pass: the rows against level 0, level i
// against level i + 1
static size_t locality_topk_ws(const onng_vectors *base, const std::vector<int64_t> &sz) {
    size_t w = topk_ws_size(base, base, sz[0], 1);
    for (size_t i = 1; i < sz.size(); i++) {
        onng_vectors q = *base;
        q.n = sz[i - 1];
        w = std::max(w, topk_ws_size(&q, base, sz[i], 1));
    }
    return w;
}

static size_t locality_ws(const onng_vectors *base, int64_t n_pivots) {
    const std::vector<int64_t> sz = locality_levels(n_pivots);
    int64_t lv = 0;
    for (int64_t m : sz) lv += m;
    Carver c(nullptr);
    c.take<int32_t>(base->n);                 // nearest pivot
    c.take<float>(base->n);                   // its distance (unused)
    c.take<uint32_t>(base->n);
    c.take<uint32_t>(base->n);
    c.take<int32_t>(base->n);
    c.take<int32_t>(base->n);                 // position of an id in an ordered level
    c.take<int32_t>(base->n);                 // sorted index
    c.take<int32_t>(lv);                      // the levels, as given
    c.take<int32_t>(lv);                      // the levels, ordered
    c.take<uint8_t>((size_t)n_pivots * base->pitch_bytes);   // rows of one level
    c.take<char>(locality_sort_bytes(std::max(base->n, n_pivots)));
    c.take<char>(locality_topk_ws(base, sz));
    return c.size() + 256;
}

}  // namespace onng

using namespace onng;

extern "C" {

const char *onng_status_string(onng_status st) {
    switch (st) {
    case ONNG_OK: return "ok";
    case ONNG_ERR_INVALID_ARG: return "invalid argument";
    case ONNG_ERR_UNSUPPORTED: return "unsupported";
    case ONNG_ERR_CAPACITY: return "capacity too small";
    case ONNG_ERR_WORKSPACE: return "workspace too small";
    case ONNG_ERR_DEVICE: return "device error";
    }
    return "unknown status";
}

const char *onng_last_error(void) { return get_error(); }

int32_t onng_version(void) { return 10000; }

// ------------------------------------------------------------- top-k ------

size_t onng_topk_workspace_size(const onng_vectors *queries, const onng_vectors *base,
                                int64_t n_cand, int32_t k) {
    if (!queries || !base) return 0;
    return topk_ws_size(queries, base, n_cand, k);
}

onng_status onng_topk(const onng_vectors *queries, const onng_vectors *base,
                      const int32_t *cand, int64_t n_cand, int32_t k, int32_t exclude_self,
                      int32_t *ids, void *dists, void *ws, size_t ws_bytes, void *stream) {
    set_error("");
    ONNG_TRY(check_vectors(queries, "queries"));
    ONNG_TRY(check_vectors(base, "base"));
    ONNG_CHECK_ARG(queries->dim == base->dim && queries->metric == base->metric,
                   "queries and base differ in dim or metric");
    ONNG_CHECK_ARG(k >= 1 && k <= 256, "k must be in [1, 256]");
    ONNG_CHECK_ARG(!cand || n_cand >= 0, "bad n_cand");
    ONNG_CHECK_ARG(ids && dists, "outputs are null");
    ONNG_CHECK_ARG(ws, "workspace is null");
    if (queries->dtype == ONNG_U8) ONNG_CHECK_ARG(queries->dim <= 512, "u8 dim above 512");
    else ONNG_CHECK_ARG(queries->dim <= 256, "f32 dim above 256");
    return launch_topk(queries, base, cand, cand ? n_cand : 0, k, exclude_self, ids, dists, ws,
                       ws_bytes, as_stream(stream));
}

onng_status onng_build_knn(const onng_vectors *base, int32_t k, int32_t *ids, void *dists,
                           void *ws, size_t ws_bytes, void *stream) {
    set_error("");
    ONNG_TRY(check_vectors(base, "base"));
    ONNG_CHECK_ARG(k >= 1 && k <= base->n - 1, "k must be in [1, n-1]");
    return onng_topk(base, base, nullptr, 0, k, 1, ids, dists, ws, ws_bytes, stream);
}

// ------------------------------------------------------- adjustments ------

size_t onng_adjust_degree_workspace_size(int64_t n, int32_t k, int32_t e_o, int32_t e_i) {
    if (n < 0 || k < 0 || e_o < 0 || e_i < 0) return 0;
    return adjust_degree_ws(n, k, e_o, e_i);
}

onng_status onng_adjust_degree(const int32_t *knn_ids, const void *knn_dists, int64_t n, int32_t k,
                               int32_t data_dtype, int32_t metric, int32_t e_o, int32_t e_i,
                               int64_t *offsets, int32_t *nbrs, void *lens, int64_t nnz_capacity,
                               int64_t *nnz_out, void *ws, size_t ws_bytes, void *stream) {
    set_error("");
    ONNG_CHECK_ARG(n >= 0 && k >= 1 && e_o >= 0 && e_i >= 0, "bad sizes");
    ONNG_CHECK_ARG(n == 0 || (knn_ids && knn_dists), "kNN table is null");
    ONNG_CHECK_ARG(offsets && nnz_out, "outputs are null");
    ONNG_CHECK_ARG(nnz_capacity == 0 || (nbrs && lens), "nbrs/lens are null");
    ONNG_CHECK_ARG(data_dtype >= ONNG_U8 && data_dtype <= ONNG_FP8_E4M3, "unknown dtype");
    ONNG_CHECK_ARG(n <= 0x7fffffffLL, "more than 2^31-1 nodes");
    if (ws_bytes < adjust_degree_ws(n, k, e_o, e_i) || !ws) {
        set_error("onng_adjust_degree: workspace too small");
        return ONNG_ERR_WORKSPACE;
    }
    return adjust_degree_launch(knn_ids, knn_dists, n, k, int_dist(data_dtype, metric), e_o, e_i,
                                offsets, nbrs, lens, nnz_capacity, nnz_out, ws, as_stream(stream));
}

size_t onng_adjust_degree_constrained_workspace_size(int64_t n, int32_t k, int32_t e_o,
                                                      int32_t e_i) {
    if (n < 0 || k < 0 || e_o < 0 || e_i < 0) return 0;
    return adjust_degree_constrained_ws(n, k, e_o, e_i);
}

onng_status onng_adjust_degree_constrained(const int32_t *knn_ids, const void *knn_dists,
                                           int64_t n, int32_t k, int32_t data_dtype,
                                           int32_t metric, int32_t e_o, int32_t e_i,
                                           int64_t *offsets, int32_t *nbrs, void *lens,
                                           int64_t nnz_capacity, int64_t *nnz_out, void *ws,
                                           size_t ws_bytes, void *stream) {
    set_error("");
    ONNG_CHECK_ARG(n >= 0 && k >= 1 && e_o >= 0 && e_i >= 0, "bad sizes");
    ONNG_CHECK_ARG(n == 0 || (knn_ids && knn_dists), "kNN table is null");
    ONNG_CHECK_ARG(offsets && nnz_out, "outputs are null");
    ONNG_CHECK_ARG(nnz_capacity == 0 || (nbrs && lens), "nbrs/lens are null");
    ONNG_CHECK_ARG(data_dtype >= ONNG_U8 && data_dtype <= ONNG_FP8_E4M3, "unknown dtype");
    ONNG_CHECK_ARG(n <= 0x7fffffffLL, "more than 2^31-1 nodes");
    if (ws_bytes < adjust_degree_constrained_ws(n, k, e_o, e_i) || !ws) {
        set_error("onng_adjust_degree_constrained: workspace too small");
        return ONNG_ERR_WORKSPACE;
    }
    return adjust_degree_constrained_launch(knn_ids, knn_dists, n, k, int_dist(data_dtype, metric),
                                            e_o, e_i, offsets, nbrs, lens, nnz_capacity, nnz_out,
                                            ws, as_stream(stream));
}

size_t onng_graph_stats_workspace_size(int64_t n, int64_t nnz) {
    if (n < 0 || nnz < 0) return 0;
    return graph_stats_ws(n, nnz);
}

onng_status onng_graph_stats(const onng_graph *g, int32_t data_dtype, int32_t metric, double frac,
                             int32_t keep, double *out, void *ws, size_t ws_bytes, void *stream) {
    set_error("");
    ONNG_CHECK_ARG(g && out, "null argument");
    ONNG_CHECK_ARG(g->n >= 0 && g->nnz >= 0 && g->n <= 0x7fffffffLL && g->nnz <= 0x7fffffffLL,
                   "bad graph sizes");
    ONNG_CHECK_ARG(g->offsets && (g->nnz == 0 || (g->nbrs && g->lens)), "graph arrays are null");
    ONNG_CHECK_ARG(frac > 0.0 && frac <= 1.0 && keep >= 0, "frac must be in (0, 1], keep >= 0");
    ONNG_CHECK_ARG(data_dtype >= ONNG_U8 && data_dtype <= ONNG_FP8_E4M3, "unknown dtype");
    ONNG_CHECK_ARG(metric == ONNG_L2SQ || metric == ONNG_COSINE, "unknown metric");
    if (ws_bytes < graph_stats_ws(g->n, g->nnz) || !ws) {
        set_error("onng_graph_stats: workspace too small");
        return ONNG_ERR_WORKSPACE;
    }
    return graph_stats_launch(g, int_dist(data_dtype, metric), metric == ONNG_L2SQ, frac, keep,
                              out, ws, as_stream(stream));
}

// ---------------------------------------------------------- edge insertion --

size_t onng_graph_add_edges_workspace_size(int64_t n, int64_t nnz, int64_t n_edges) {
    if (n < 0 || nnz < 0 || n_edges < 0) return 0;
    return add_edges_ws(n, nnz, n_edges);
}

onng_status onng_graph_add_edges(const onng_graph *in, const int32_t *src, const int32_t *dst,
                                 const void *lens, int64_t n_edges, int32_t data_dtype,
                                 int32_t metric, int64_t *offsets, int32_t *nbrs, void *out_lens,
                                 int64_t nnz_capacity, int64_t *nnz_out, void *ws,
                                 size_t ws_bytes, void *stream) {
    set_error("");
    ONNG_CHECK_ARG(in && offsets && nnz_out, "null argument");
    ONNG_CHECK_ARG(in->n >= 0 && in->nnz >= 0 && in->n <= 0x7fffffffLL && n_edges >= 0 &&
                   in->nnz + n_edges <= 0x7fffffffLL, "bad sizes");
    ONNG_CHECK_ARG(in->offsets && (in->nnz == 0 || (in->nbrs && in->lens)), "graph arrays are null");
    ONNG_CHECK_ARG(n_edges == 0 || (src && dst && lens), "edge arrays are null");
    ONNG_CHECK_ARG(nnz_capacity == 0 || (nbrs && out_lens), "outputs are null");
    ONNG_CHECK_ARG(data_dtype >= ONNG_U8 && data_dtype <= ONNG_FP8_E4M3, "unknown dtype");
    if (ws_bytes < add_edges_ws(in->n, in->nnz, n_edges) || !ws) {
        set_error("onng_graph_add_edges: workspace too small");
        return ONNG_ERR_WORKSPACE;
    }
    return add_edges_launch(in, src, dst, lens, n_edges, int_dist(data_dtype, metric), offsets,
                            nbrs, out_lens, nnz_capacity, nnz_out, ws, as_stream(stream));
}

onng_status onng_graph_head(const onng_graph *g, int32_t data_dtype, int32_t metric, int32_t k,
                            int32_t *ids, void *dists, void *stream) {
    set_error("");
    ONNG_CHECK_ARG(g && g->offsets && (g->nnz == 0 || (g->nbrs && g->lens)), "graph is null");
    ONNG_CHECK_ARG(g->n >= 0 && g->nnz >= 0 && g->n <= 0x7fffffffLL, "bad sizes");
    ONNG_CHECK_ARG(k >= 1 && k <= 4096, "k must be in [1, 4096]");
    ONNG_CHECK_ARG(g->n == 0 || (ids && dists), "outputs are null");
    ONNG_CHECK_ARG(data_dtype >= ONNG_U8 && data_dtype <= ONNG_FP8_E4M3, "unknown dtype");
    ONNG_CHECK_ARG(metric == ONNG_L2SQ || metric == ONNG_COSINE, "unknown metric");
    return graph_head_launch(g, int_dist(data_dtype, metric), k, ids, dists, as_stream(stream));
}

// ------------------------------------------------------- tree-based seeds --

static onng_status check_vptree_rows(const onng_vectors *v, const char *what) {
    ONNG_TRY(check_vectors(v, what));
    ONNG_CHECK_ARG((v->dtype == ONNG_U8 && v->metric == ONNG_L2SQ) || v->dtype == ONNG_F32,
                   "tree rows must be u8 (squared L2) or f32");
    return ONNG_OK;
}

size_t onng_vptree_build_workspace_size(int64_t n) {
    if (n < 0) return 0;
    return vptree_ws(n);
}

onng_status onng_vptree_build(const onng_vectors *base, const uint32_t *priority,
                              onng_vptree *tree, void *ws, size_t ws_bytes, void *stream) {
    set_error("");
    ONNG_TRY(check_vptree_rows(base, "base"));
    ONNG_CHECK_ARG(base->n >= 1 && base->n <= 0x7fffffffLL, "base must hold 1 .. 2^31-1 rows");
    ONNG_CHECK_ARG(priority && tree, "null argument");
    ONNG_CHECK_ARG(tree->node_vp && tree->node_child && tree->node_mu && tree->leaf_seeds,
                   "tree arrays are null");
    ONNG_CHECK_ARG(tree->leaf_size >= 4 && tree->leaf_size <= 256, "leaf_size must be in [4, 256]");
    ONNG_CHECK_ARG(tree->n_seeds >= 1 && tree->n_seeds <= 256, "n_seeds must be in [1, 256]");
    ONNG_CHECK_ARG(tree->node_capacity >= 1 && tree->leaf_capacity >= 1, "capacities must be >= 1");
    if (ws_bytes < vptree_ws(base->n) || !ws) {
        set_error("onng_vptree_build: workspace too small");
        return ONNG_ERR_WORKSPACE;
    }
    return vptree_build_launch(base, priority, tree, ws, as_stream(stream));
}

onng_status onng_vptree_seeds(const onng_vectors *base, const onng_vptree *tree,
                              const onng_vectors *queries, int32_t *seeds, int32_t *dc,
                              void *stream) {
    set_error("");
    ONNG_TRY(check_vptree_rows(base, "base"));
    ONNG_TRY(check_vptree_rows(queries, "queries"));
    ONNG_CHECK_ARG(queries->dtype == base->dtype && queries->dim == base->dim &&
                   queries->metric == base->metric, "queries must match the base rows");
    ONNG_CHECK_ARG(tree && tree->n_nodes >= 1 && tree->n_leaves >= 1 && tree->node_vp &&
                   tree->node_child && tree->node_mu && tree->leaf_seeds,
                   "tree is not built");
    ONNG_CHECK_ARG(tree->n_seeds >= 1 && tree->n_seeds <= 256, "n_seeds must be in [1, 256]");
    ONNG_CHECK_ARG(queries->n == 0 || (seeds && dc), "outputs are null");
    return vptree_seeds_launch(base, tree, queries, seeds, dc, as_stream(stream));
}

size_t onng_adjust_path_workspace_size(int64_t n, int64_t nnz) {
    if (n < 0 || nnz < 0) return 0;
    return adjust_path_ws(n, nnz);
}

onng_status onng_adjust_path(const onng_graph *in, int32_t data_dtype, int32_t metric,
                             int64_t *offsets, int32_t *nbrs, void *lens, int64_t *nnz_out,
                             void *ws, size_t ws_bytes, void *stream) {
    set_error("");
    ONNG_CHECK_ARG(in && in->offsets && in->n >= 0 && in->nnz >= 0, "graph is null");
    ONNG_CHECK_ARG(in->nnz == 0 || (in->nbrs && in->lens), "graph needs nbrs and lens");
    ONNG_CHECK_ARG(offsets && nnz_out && (in->nnz == 0 || (nbrs && lens)), "outputs are null");
    ONNG_CHECK_ARG(in->n <= 0x7fffffffLL, "more than 2^31-1 nodes");
    if (ws_bytes < adjust_path_ws(in->n, in->nnz) || !ws) {
        set_error("onng_adjust_path: workspace too small");
        return ONNG_ERR_WORKSPACE;
    }
    return adjust_path_launch(in, int_dist(data_dtype, metric), offsets, nbrs, lens, nnz_out, ws,
                              as_stream(stream));
}

// ------------------------------------------------------------- search -----

size_t onng_search_workspace_size(const onng_vectors *base, int64_t n_queries,
                                  const onng_search_params *params) {
    if (!base || !params || check_vectors(base, "base") != ONNG_OK) return 0;
    onng_launch_config tuned;
    const onng_launch_config *cfg = params->launch;
    if (!cfg && lookup_tuned(base, params, &tuned)) cfg = &tuned;
    SearchPlan P;
    if (make_plan(base, n_queries, params, cfg, &P) != ONNG_OK) return 0;
    return P.ws;
}

onng_status onng_search(const onng_vectors *base, const onng_graph *graph,
                        const onng_vectors *queries, const int32_t *seeds, int32_t n_seeds,
                        const onng_search_params *params, int32_t *ids, void *dists,
                        onng_query_stats *stats, void *ws, size_t ws_bytes, void *stream) {
    set_error("");
    onng_launch_config tuned;
    const onng_launch_config *cfg = params ? params->launch : nullptr;
    if (params && !cfg && base && lookup_tuned(base, params, &tuned)) cfg = &tuned;
    return run_search(base, graph, queries, seeds, n_seeds, params, ids, dists, stats, ws,
                      ws_bytes, as_stream(stream), cfg);
}

// -------------------------------------------- search without allocation ----

// Scratch of onng_search_static: work counter, visited bitsets, visit logs and
// spill buffers of the persistent waves.  Each device the library runs on
// holds its own copy until the process ends.  Host code never uses this name
// as a device address: the address on a device comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[ONNG_SEARCH_STATIC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static std::map<int, void *> g_scratch_ptr;   // device ordinal -> its `scratch`

// Address of `scratch` on the current device, looked up once per device.
static onng_status scratch_on_current_device(void **out) {
    int dev = 0;
    ONNG_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it != g_scratch_ptr.end()) {
        *out = it->second;
        return ONNG_OK;
    }
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        set_error(std::string("onng_search_static: hipGetSymbolAddress failed: ") +
                  hipGetErrorString(e));
        return ONNG_ERR_DEVICE;
    }
    g_scratch_ptr[dev] = p;
    *out = p;
    return ONNG_OK;
}

onng_status onng_search_static(const onng_vectors *base, const onng_graph *graph,
                               const onng_vectors *queries, const int32_t *seeds, int32_t n_seeds,
                               const onng_search_params *params, int32_t *ids, void *dists,
                               onng_query_stats *stats, void *stream) {
    set_error("");
    ONNG_TRY(validate_search(base, graph, queries, seeds, n_seeds, params));
    ONNG_CHECK_ARG(ids && dists && stats, "outputs are null");
    if (queries->n == 0) return ONNG_OK;
    void *ws = nullptr;
    ONNG_TRY(scratch_on_current_device(&ws));
    onng_launch_config tuned;
    const onng_launch_config *cfg0 = params->launch;
    if (!cfg0 && lookup_tuned(base, params, &tuned)) cfg0 = &tuned;
    SearchPlan P;
    ONNG_TRY(make_plan(base, queries->n, params, cfg0, &P));
    // the same shape with as many persistent blocks as the scratch holds; the
    // carve adds at most 256 bytes of alignment per region (five regions)
    const size_t per_slot = (size_t)P.gbits_words * 4 + (size_t)P.vlog_cap * 4 +
                            (size_t)P.spill_cap * 16;
    const size_t fixed = 6 * 256 + 64 * 4;
    const size_t cap = ONNG_SEARCH_STATIC_SCRATCH_BYTES;
    const int64_t max_blocks =
        cap > fixed ? (int64_t)((cap - fixed) / (per_slot * (size_t)P.wpb)) : 0;
    if (max_blocks < 1) {
        set_error("onng_search_static: a block of " + std::to_string(P.wpb) + " waves needs " +
                  std::to_string(per_slot * P.wpb + fixed) + " bytes of scratch for " +
                  std::to_string(base->n) + " rows; the static scratch holds " +
                  std::to_string(cap) + " (use onng_search with a workspace)");
        return ONNG_ERR_CAPACITY;
    }
    onng_launch_config c = cfg0 ? *cfg0 : onng_launch_config{};
    c.blocks = (int32_t)std::min<int64_t>(P.blocks, max_blocks);
    SearchPlan P2;
    ONNG_TRY(make_plan(base, queries->n, params, &c, &P2));
    if (P2.ws > cap) {
        set_error("onng_search_static: internal scratch layout");
        return ONNG_ERR_CAPACITY;
    }
    return run_search(base, graph, queries, seeds, n_seeds, params, ids, dists, stats, ws, cap,
                      as_stream(stream), &c, 1);
}

size_t onng_order_by_cost_workspace_size(int64_t n) { return n < 0 ? 0 : order_ws(n); }

onng_status onng_order_by_cost(const onng_query_stats *stats, int64_t n, int32_t *order, void *ws,
                               size_t ws_bytes, void *stream) {
    set_error("");
    ONNG_CHECK_ARG(n >= 0 && n <= 0x7fffffffLL, "bad n");
    ONNG_CHECK_ARG(n == 0 || (stats && order), "null pointer");
    return order_launch(stats, n, order, ws, ws_bytes, as_stream(stream));
}

onng_status onng_autotune_search(const onng_vectors *base, const onng_graph *graph,
                                 const onng_vectors *queries, const int32_t *seeds,
                                 int32_t n_seeds, const onng_search_params *params,
                                 int32_t *ids, void *dists, onng_query_stats *stats, void *ws,
                                 size_t ws_bytes, void *stream, onng_launch_config *best) {
    set_error("");
    ONNG_CHECK_ARG(best, "best is null");
    ONNG_TRY(validate_search(base, graph, queries, seeds, n_seeds, params));
    if (lookup_tuned(base, params, best)) return ONNG_OK;
    hipStream_t st = as_stream(stream);
    std::vector<onng_launch_config> cands;
    const int n16 = row_pieces(base);
    for (int L : {4, 8, 16, 32})
        for (int s_cap : {128, 256, 512})
            for (int vl : {10, 11, 12, 13, -1})
                for (int wpb : {2, 4}) {
                    if ((n16 + L - 1) / L > ppl_for(base->dtype)) continue;
                    onng_launch_config c{};
                    c.waves_per_block = wpb;
                    c.lanes_per_row = L;
                    c.s_capacity = s_cap;
                    c.visited_log2 = vl;
                    cands.push_back(c);
                }
    hipEvent_t e0, e1;
    ONNG_HIP(hipEventCreate(&e0));
    ONNG_HIP(hipEventCreate(&e1));
    float best_ms = 1e30f;
    bool found = false;
    for (const auto &c : cands) {
        SearchPlan P;
        if (make_plan(base, queries->n, params, &c, &P) != ONNG_OK) continue;
        if (P.ws > ws_bytes) continue;
        // warm-up, then two timed runs
        // the warm-up zeroes the bitsets of this shape; the timed runs reuse them
        if (run_search(base, graph, queries, seeds, n_seeds, params, ids, dists, stats, ws,
                       ws_bytes, st, &c, 0) != ONNG_OK)
            continue;
        ONNG_HIP(hipEventRecord(e0, st));
        for (int r = 0; r < 2; r++)
            run_search(base, graph, queries, seeds, n_seeds, params, ids, dists, stats, ws,
                       ws_bytes, st, &c, 1);
        ONNG_HIP(hipEventRecord(e1, st));
        ONNG_HIP(hipEventSynchronize(e1));
        float ms = 0.0f;
        ONNG_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best_ms) {
            best_ms = ms;
            *best = c;
            found = true;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!found) {
        set_error("onng_autotune_search: no launch shape fits the workspace");
        return ONNG_ERR_WORKSPACE;
    }
    TuneKey key{base->dtype, base->metric, base->dim, base->n, params->k_stride,
                params->rerank_base ? params->pool_factor : 0, params->two_phase};
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = *best;
    return ONNG_OK;
}

// ------------------------------------------------------ codecs, rerank ----

size_t onng_locality_order_workspace_size(const onng_vectors *base, int64_t n_pivots) {
    if (!base || n_pivots < 1) return 0;
    return locality_ws(base, n_pivots);
}

onng_status onng_locality_order(const onng_vectors *base, const int32_t *pivots,
                                int64_t n_pivots, int32_t *perm, void *ws, size_t ws_bytes,
                                void *stream) {
    set_error("");
    ONNG_TRY(check_vectors(base, "base"));
    ONNG_CHECK_ARG(pivots && perm && n_pivots >= 1 && n_pivots <= base->n, "bad arguments");
    ONNG_CHECK_ARG(base->dtype == ONNG_U8 || base->dtype == ONNG_F32, "base must be u8 or f32");
    ONNG_CHECK_ARG(base->n < (int64_t)INT32_MAX, "too many rows");
    if (!ws || ws_bytes < locality_ws(base, n_pivots)) {
        set_error("onng_locality_order: workspace too small");
        return ONNG_ERR_WORKSPACE;
    }
    const int64_t n = base->n;
    if (n == 0) return ONNG_OK;
    hipStream_t st = as_stream(stream);
    const std::vector<int64_t> sz = locality_levels(n_pivots);
    const int top = (int)sz.size() - 1;
    int64_t lv = 0;
    for (int64_t m : sz) lv += m;
    Carver c(ws);
    int32_t *nn = c.take<int32_t>(n);
    float *nd = c.take<float>(n);
    uint32_t *key = c.take<uint32_t>(n);
    uint32_t *key_sorted = c.take<uint32_t>(n);
    int32_t *idx = c.take<int32_t>(n);
    int32_t *pos_of = c.take<int32_t>(n);
    int32_t *sidx = c.take<int32_t>(n);
    int32_t *given = c.take<int32_t>(lv);
    int32_t *ordered = c.take<int32_t>(lv);
    uint8_t *rows = c.take<uint8_t>((size_t)n_pivots * base->pitch_bytes);
    size_t tb = locality_sort_bytes(std::max(n, n_pivots));
    void *tmp = c.take<char>(tb);
    size_t tkb = locality_topk_ws(base, sz);
    void *tk = c.take<char>(tkb);
    auto blocks = [](int64_t m) { return dim3((unsigned)((m + 255) / 256)); };
    std::vector<int64_t> at(sz.size(), 0);    // offset of each level in given/ordered
    for (size_t i = 1; i < sz.size(); i++) at[i] = at[i - 1] + sz[i - 1];
    ONNG_HIP(hipMemcpyAsync(given, pivots, sizeof(int32_t) * n_pivots, hipMemcpyDeviceToDevice,
                            st));
    for (int i = 1; i <= top; i++)
        hipLaunchKernelGGL(strided_kernel, blocks(sz[i]), dim3(256), 0, st, given + at[i - 1],
                           sz[i], LOC_STRIDE, given + at[i]);
    ONNG_HIP(hipMemcpyAsync(ordered + at[top], given + at[top], sizeof(int32_t) * sz[top],
                            hipMemcpyDeviceToDevice, st));
    // Order level i: its pivots by (position of their nearest pivot of the
    // ordered level i + 1, position in level i); then the rows the same way
    // against the ordered level 0.  Stable radix sorts keep the second key.
    for (int i = top; i >= 0; i--) {
        const int32_t *cand = ordered + at[i];
        const int64_t m = sz[i];
        hipLaunchKernelGGL(position_kernel, blocks(m), dim3(256), 0, st, cand, m, pos_of);
        const bool rows_pass = i == 0;
        const int64_t nq = rows_pass ? n : sz[i - 1];
        onng_vectors Q = *base;
        if (!rows_pass) {
            hipLaunchKernelGGL(gather_bytes_kernel, dim3((unsigned)nq), dim3(64), 0, st,
                               static_cast<const uint8_t *>(base->data), base->pitch_bytes,
                               given + at[i - 1], nq, rows);
            Q.data = rows;
            Q.n = nq;
            Q.scale = nullptr;
        }
        ONNG_TRY(launch_topk(&Q, base, cand, m, 1, 0, nn, nd, tk, tkb, st));
        hipLaunchKernelGGL(nearest_key_kernel, blocks(nq), dim3(256), 0, st, nn, nq, pos_of, key,
                           idx);
        int32_t *out = rows_pass ? perm : sidx;
        ONNG_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, tb, key, key_sorted, idx, out, (int)nq, 0,
                                                    32, st));
        if (!rows_pass)
            hipLaunchKernelGGL(permute_kernel, blocks(nq), dim3(256), 0, st, given + at[i - 1],
                               sidx, nq, ordered + at[i - 1]);
    }
    ONNG_HIP(hipGetLastError());
    return ONNG_OK;
}

onng_status onng_gather_rows(const void *src, int64_t pitch_bytes, const int32_t *ids, int64_t n,
                             void *dst, void *stream) {
    set_error("");
    ONNG_CHECK_ARG(n >= 0 && pitch_bytes > 0 && pitch_bytes % 16 == 0, "bad sizes");
    ONNG_CHECK_ARG(n == 0 || (src && ids && dst), "null pointer");
    if (n == 0) return ONNG_OK;
    hipLaunchKernelGGL(gather_bytes_kernel, dim3((unsigned)n), dim3(64), 0, as_stream(stream),
                       static_cast<const uint8_t *>(src), pitch_bytes, ids, n,
                       static_cast<uint8_t *>(dst));
    ONNG_HIP(hipGetLastError());
    return ONNG_OK;
}

onng_status onng_encode(const float *src, int64_t n, int32_t dim, int32_t dtype, void *dst,
                        int64_t dst_pitch, float *scale, void *stream) {
    set_error("");
    ONNG_CHECK_ARG(n >= 0 && dim > 0, "bad sizes");
    ONNG_CHECK_ARG(n == 0 || (src && dst), "null pointer");
    ONNG_CHECK_ARG(dtype >= ONNG_F32 && dtype <= ONNG_FP8_E4M3, "dtype must be a float format");
    ONNG_CHECK_ARG(dst_pitch >= (int64_t)dim * elem_bytes(dtype), "dst_pitch too small");
    ONNG_CHECK_ARG(dtype != ONNG_FP8_E4M3 || scale || dst_pitch >= fp8_inrow_pitch(dim),
                   "FP8 needs a scale array or room for the scale in the row");
    return encode_launch(src, n, dim, dtype, dst, dst_pitch, scale, as_stream(stream));
}

onng_status onng_rerank(const onng_vectors *queries, const onng_vectors *base,
                        const int32_t *pool, int32_t pool_size, int32_t k, int32_t use_f64,
                        int32_t *ids, void *dists, void *stream) {
    set_error("");
    ONNG_TRY(check_vectors(queries, "queries"));
    ONNG_TRY(check_vectors(base, "base"));
    ONNG_CHECK_ARG(queries->dim == base->dim && queries->metric == base->metric,
                   "queries and base differ in dim or metric");
    ONNG_CHECK_ARG(pool_size >= 0 && k >= 1, "bad sizes");
    ONNG_CHECK_ARG(queries->n == 0 || (pool && ids && dists), "null pointer");
    return rerank_launch(queries, base, pool, pool_size, k, use_f64, ids, dists,
                         as_stream(stream));
}

// ---------------------------------------------------------------- MLP -----

onng_status onng_mlp_forward(const float *X, int32_t batch, int32_t F, const float *W1,
                             const float *b1, int32_t H, const float *W2, const float *b2,
                             int32_t T, float *hidden, float *Y, void *stream) {
    set_error("");
    ONNG_CHECK_ARG(batch >= 0 && F >= 1 && H >= 1 && H <= 64 && T >= 1 && T <= 16,
                   "sizes: H in [1, 64], T in [1, 16]");
    ONNG_CHECK_ARG(batch == 0 || (X && W1 && b1 && W2 && b2 && Y), "null pointer");
    return mlp_forward_launch(X, batch, F, W1, b1, H, W2, b2, T, hidden, Y, as_stream(stream));
}

size_t onng_mlp_backward_workspace_size(int32_t batch, int32_t H, int32_t T) {
    if (batch < 0 || H < 1 || T < 1) return 0;
    return mlp_backward_ws(batch, H, T);
}

onng_status onng_mlp_backward(const float *X, const float *target, const float *w, int32_t batch,
                              int32_t F, const float *W1, const float *b1, int32_t H,
                              const float *W2, const float *b2, int32_t T, float *gW1,
                              float *gb1, float *gW2, float *gb2, float *loss, void *ws,
                              size_t ws_bytes, void *stream) {
    set_error("");
    ONNG_CHECK_ARG(batch >= 1 && F >= 1 && H >= 1 && H <= 64 && T >= 1 && T <= 16,
                   "sizes: batch >= 1, H in [1, 64], T in [1, 16]");
    ONNG_CHECK_ARG(X && target && W1 && b1 && W2 && b2 && gW1 && gb1 && gW2 && gb2 && loss,
                   "null pointer");
    if (!ws || ws_bytes < mlp_backward_ws(batch, H, T)) {
        set_error("onng_mlp_backward: workspace too small");
        return ONNG_ERR_WORKSPACE;
    }
    return mlp_backward_launch(X, target, w, batch, F, W1, b1, H, W2, b2, T, gW1, gb1, gW2, gb2,
                               loss, ws, as_stream(stream));
}

onng_status onng_adam_step(float *p, const float *g, float *m, float *v, int64_t n, float lr,
                           float beta1, float beta2, float eps, int32_t t, void *stream) {
    set_error("");
    ONNG_CHECK_ARG(n >= 0 && t >= 1, "bad sizes");
    ONNG_CHECK_ARG(n == 0 || (p && g && m && v), "null pointer");
    return adam_launch(p, g, m, v, n, lr, beta1, beta2, eps, t, as_stream(stream));
}

onng_status onng_feature_transform(const float *raw, int64_t n, int32_t metric, float *out,
                                   void *stream) {
    set_error("");
    ONNG_CHECK_ARG(n >= 0 && (n == 0 || (raw && out)), "bad arguments");
    return feature_transform_launch(raw, n, metric, out, as_stream(stream));
}

onng_status onng_column_stats(const float *x, const float *w, int64_t n, int32_t cols,
                              float *mean, float *std_out, void *stream) {
    set_error("");
    if (n < 0 || cols < 0 || (cols > 0 && (!mean || !std_out)) || (n > 0 && cols > 0 && !x)) {
        set_error("onng_column_stats: negative size or missing array");
        return ONNG_ERR_INVALID_ARG;
    }
    return column_stats_launch(x, w, n, cols, mean, std_out, as_stream(stream));
}

onng_status onng_standardize(const float *x, int64_t n, int32_t cols, const float *mean,
                             const float *std_in, float *out, void *stream) {
    set_error("");
    if (n < 0 || cols < 0 || (n > 0 && cols > 0 && (!x || !mean || !std_in || !out))) {
        set_error("onng_standardize: negative size or missing array");
        return ONNG_ERR_INVALID_ARG;
    }
    return standardize_launch(x, n, cols, mean, std_in, out, as_stream(stream));
}

onng_status onng_mlp_fold_output(float *w2, float *b2, int32_t T, int32_t H, const float *scale,
                                 const float *shift, void *stream) {
    set_error("");
    if (T < 0 || H < 0 || (T > 0 && (!w2 || !b2 || !scale || !shift))) {
        set_error("onng_mlp_fold_output: negative size or missing array");
        return ONNG_ERR_INVALID_ARG;
    }
    return fold_output_launch(w2, b2, T, H, scale, shift, as_stream(stream));
}

onng_status onng_degree_loss(const double *p, const double *c, int32_t n, double *loss) {
    set_error("");
    if (n < 1 || !p || !c || !loss) {
        set_error("onng_degree_loss: needs n >= 1 samples");
        return ONNG_ERR_INVALID_ARG;
    }
    std::vector<int> ord(n);
    for (int i = 0; i < n; i++) {
        if (!(c[i] > 0.0)) {
            set_error("onng_degree_loss: distance counts must be positive");
            return ONNG_ERR_INVALID_ARG;
        }
        ord[i] = i;
    }
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return p[a] < p[b]; });
    const double span = p[ord[n - 1]] - p[ord[0]];
    if (!(span > 0.0)) {
        double s = 0.0;
        for (int i = 0; i < n; i++) s += std::log10(c[i]);
        *loss = s / n;
        return ONNG_OK;
    }
    double area = 0.0;
    for (int i = 0; i + 1 < n; i++) {
        const int a = ord[i], b = ord[i + 1];
        area += (p[b] - p[a]) * (std::log10(c[a]) + std::log10(c[b])) * 0.5;
    }
    *loss = area / span;
    return ONNG_OK;
}

// ----------------------------------------------------------- pipeline -----

struct onng_pipeline {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

size_t onng_pipeline_workspace_size(const onng_vectors *base, const onng_vectors *queries,
                                    int64_t n_pivots, int32_t n_seeds,
                                    const onng_search_params *params) {
    if (!base || !queries || !params) return 0;
    // seeds come from the f32 rows when the searched rows are low precision
    const onng_vectors *seed_base =
        base->dtype == ONNG_U8 || base->dtype == ONNG_F32 ? base : params->rerank_base;
    if (!seed_base) return 0;
    size_t a = onng_topk_workspace_size(queries, seed_base, n_pivots, n_seeds);
    size_t b = onng_search_workspace_size(base, queries->n, params);
    if (!a || !b) return 0;
    size_t extra = 0;
    if (params->predictor) {
        // predict-only stats, the order and its sort scratch
        Carver c(nullptr);
        c.take<onng_query_stats>(queries->n);
        c.take<int32_t>(queries->n);
        c.take<char>(order_ws(queries->n));
        extra = c.size() + 256;
    }
    return (a + 255) / 256 * 256 + extra + b;
}

onng_status onng_pipeline_create(const onng_vectors *base, const onng_graph *graph,
                                 const onng_vectors *queries, const int32_t *pivots,
                                 int64_t n_pivots, int32_t n_seeds, int32_t *seeds,
                                 const onng_search_params *params, int32_t *ids, void *dists,
                                 onng_query_stats *stats, void *ws, size_t ws_bytes,
                                 void *stream, onng_pipeline **handle) {
    set_error("");
    ONNG_CHECK_ARG(handle && pivots && seeds && n_pivots >= 1, "bad pipeline arguments");
    ONNG_TRY(validate_search(base, graph, queries, seeds, n_seeds, params));
    ONNG_CHECK_ARG(base->dtype == ONNG_U8 || base->dtype == ONNG_F32 || params->rerank_base,
                   "low-precision rows need rerank_base (f32 rows) for seeding");
    size_t need = onng_pipeline_workspace_size(base, queries, n_pivots, n_seeds, params);
    if (!need || !ws || ws_bytes < need) {
        set_error("onng_pipeline_create: workspace too small");
        return ONNG_ERR_WORKSPACE;
    }
    // seeds come from the f32 rows when the searched rows are low precision
    const onng_vectors *seed_base = base->dtype == ONNG_U8 || base->dtype == ONNG_F32
                                        ? base : params->rerank_base;
    size_t a = (onng_topk_workspace_size(queries, seed_base, n_pivots, n_seeds) + 255) / 256 * 256;
    char *wsa = static_cast<char *>(ws);
    hipStream_t st = as_stream(stream);
    bool own = false;
    if (!st) {
        ONNG_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
        own = true;
    }
    // seed distances are not needed: write them into the search outputs,
    // which the search overwrites afterwards
    void *seed_d = dists;
    // The captured searches trust the visited bitsets their last replay left
    // zero; the tag of the search workspace is cleared now (outside the
    // graph), so the first replay zeroes them.
    size_t pre_used = 0;
    if (params->predictor && !params->single_pass) {
        Carver c0(nullptr);
        c0.take<onng_query_stats>(queries->n);
        c0.take<int32_t>(queries->n);
        c0.take<char>(order_ws(queries->n));
        pre_used = (c0.size() + 255) / 256 * 256;
    }
    {
        void *targs[] = {nullptr};
        uint64_t *tag_at = reinterpret_cast<uint64_t *>(wsa + a + pre_used) + 1;
        targs[0] = &tag_at;
        if (hipLaunchKernel(clear_tag_kernel_ptr(), dim3(1), dim3(1), targs, 0, st) != hipSuccess) {
            if (own) (void)hipStreamDestroy(st);
            set_error("onng_pipeline_create: launch failed");
            return ONNG_ERR_DEVICE;
        }
    }
    // the launch shape: the caller's, else a tuned one for this index, else the default
    onng_launch_config tuned;
    const onng_launch_config *cfg = params->launch;
    if (!cfg && lookup_tuned(base, params, &tuned)) cfg = &tuned;
    onng_pipeline *pl = new onng_pipeline();
    onng_status rc = ONNG_OK;
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        set_error("onng_pipeline_create: stream capture failed to start");
        delete pl;
        if (own) (void)hipStreamDestroy(st);
        return ONNG_ERR_DEVICE;
    }
    if (params->k_stride < n_seeds) {
        rc = ONNG_ERR_INVALID_ARG;
        set_error("onng_pipeline_create: k_stride must be >= n_seeds");
    }
    if (rc == ONNG_OK)
        rc = launch_topk(queries, seed_base, pivots, n_pivots, n_seeds, 0, seeds, seed_d, wsa, a,
                         st);
    if (rc == ONNG_OK && (!params->predictor || params->single_pass)) {
        rc = run_search(base, graph, queries, seeds, n_seeds, params, ids, dists, stats, wsa + a,
                        ws_bytes - a, st, cfg, 1);
    } else if (rc == ONNG_OK) {
        // predict the range of every query, order the queries by predicted
        // cost (longest first), then search with the predicted ranges
        Carver c(wsa + a);
        onng_query_stats *pst = c.take<onng_query_stats>(queries->n);
        int32_t *order = c.take<int32_t>(queries->n);
        size_t ob = order_ws(queries->n);
        void *ows = c.take<char>(ob);
        size_t used = (c.size() + 255) / 256 * 256;   // == pre_used
        onng_search_params p1 = *params;
        p1.predict_only = 1;
        p1.features_out = nullptr;
        onng_search_params p2 = *params;
        p2.two_phase = 0;
        p2.predictor = nullptr;
        p2.predict_only = 0;
        p2.features_out = nullptr;
        p2.range_from = pst;
        p2.order = order;
        rc = run_search(base, graph, queries, seeds, n_seeds, &p1, ids, dists, pst,
                        wsa + a + used, ws_bytes - a - used, st, cfg, 1);
        if (rc == ONNG_OK) rc = order_launch(pst, queries->n, order, ows, ob, st);
        if (rc == ONNG_OK)
            rc = run_search(base, graph, queries, seeds, n_seeds, &p2, ids, dists, stats,
                            wsa + a + used, ws_bytes - a - used, st, cfg, 1);
    }
    hipGraph_t g = nullptr;
    hipError_t ce = hipStreamEndCapture(st, &g);
    if (rc == ONNG_OK && ce != hipSuccess) {
        rc = ONNG_ERR_DEVICE;
        set_error(std::string("onng_pipeline_create: capture failed: ") + hipGetErrorString(ce));
    }
    if (rc == ONNG_OK && hipGraphInstantiate(&pl->exec, g, nullptr, nullptr, 0) != hipSuccess) {
        rc = ONNG_ERR_DEVICE;
        set_error("onng_pipeline_create: graph instantiation failed");
    }
    pl->graph = g;
    if (own) (void)hipStreamDestroy(st);
    if (rc != ONNG_OK) {
        if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
        if (pl->graph) (void)hipGraphDestroy(pl->graph);
        delete pl;
        return rc;
    }
    *handle = pl;
    return ONNG_OK;
}

onng_status onng_pipeline_launch(onng_pipeline *handle, void *stream) {
    set_error("");
    ONNG_CHECK_ARG(handle && handle->exec, "bad handle");
    ONNG_HIP(hipGraphLaunch(handle->exec, as_stream(stream)));
    return ONNG_OK;
}

onng_status onng_pipeline_destroy(onng_pipeline *handle) {
    if (!handle) return ONNG_OK;
    if (handle->exec) (void)hipGraphExecDestroy(handle->exec);
    if (handle->graph) (void)hipGraphDestroy(handle->graph);
    delete handle;
    return ONNG_OK;
}

}  // extern "C"
