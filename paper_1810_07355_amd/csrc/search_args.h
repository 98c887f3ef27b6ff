// Kernel-argument block of the search kernel and the fused search-range
// predictor evaluated after the first expansion.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/onng.h"
#include "pred_inputs.h"

namespace onng {

struct PredArgs {
    const uint16_t *w1;   // bf16 [H][F]
    const float *b1;      // [H]
    const uint16_t *w2;   // bf16 [T][H]
    const float *b2;      // [T]
    const float *mean;    // [F]
    const float *stdv;    // [F]
    const float *shift;   // [T] or null
    const int32_t *head_pq;
    int32_t head;
    int32_t F, H, T;
    float eps_min, eps_max, e0, we;
    int32_t mode;             // ONNG_PRED_LOG_EPS or ONNG_PRED_CURVE
    int32_t n_cand;
    const float *eps_cand;    // [n_cand]
    float lambda;
    const float *lambda_pq;   // [nq] or null
};

struct SearchKArgs {
    // stored rows
    const uint8_t *base;
    const float *base_scale;
    int32_t scale_in_row;       // FP8 rows keep their scale in the last 4 bytes
    int64_t base_pitch;
    int64_t n_base;
    int32_t dim;
    int32_t n16;            // 16-byte pieces per stored row
    // graph
    const int64_t *offsets;
    const int32_t *nbrs;
    // queries (u8 rows for u8 data, f32 rows otherwise)
    const uint8_t *qry;
    int64_t q_pitch;
    int32_t nq;
    const int32_t *seeds;
    int32_t n_seeds;
    // parameters
    int32_t k;
    const int32_t *k_pq;
    int32_t k_stride;
    float eps;
    const float *eps_pq;
    uint32_t ep;
    const uint32_t *ep_pq;
    int32_t two_phase;
    uint32_t ep_first;
    uint32_t probe_hops;
    int32_t predict_only;
    float us_per_tick;          // wall-clock counter period in microseconds
    const onng_query_stats *range_from;
    const int32_t *order;
    int32_t max_dc;
    const int32_t *max_dc_pq;
    float max_dc_factor;
    const int32_t *id_map;
    int32_t has_pred;
    PredArgs pred;
    float *feat_out;
    // rerank
    int32_t has_rr;
    const uint8_t *rr_base;
    int64_t rr_pitch;
    int32_t pool_factor;
    // outputs
    int32_t *out_ids;
    void *out_d;
    onng_query_stats *stats;
    // scheduling and scratch
    int32_t *counter;       // [0] work ticket, [1] waves finished
    uint64_t *ws_tag_at;    // tag of the workspace layout whose bitsets are all zero
    uint64_t ws_tag;        // this launch's layout
    int32_t ws_reuse;       // caller vouches that only searches wrote the workspace
    uint32_t *gbits;
    int64_t gbits_words;    // per slot, a multiple of 32
    int32_t *vlog;
    int32_t vlog_cap;       // per slot
    uint64_t *spill;
    int32_t spill_cap;      // per slot and buffer (two buffers per slot)
    // on-chip layout, per wave
    int32_t lanes_per_row;
    int32_t s_cap;
    int32_t vis_log2;
    int32_t pool_cap;
    int32_t waves_per_block;
    int32_t lds_per_wave;
    int32_t off_pool, off_s, off_stage, off_stage2, off_ids, off_vis, off_misc;
};

// Search range of one query from the state after the probe expansions.
// Lane t < 14 holds raw feature t (0-7 seed distances ascending, 8 |S|,
// 9-11 smallest / middle / m-th of the m = min(|S|, 64) smallest distances in
// S, 12 the largest distance in R, 13 distance computations).  `scratch` is
// 96 floats of LDS.  Features enter as log distances (relative to the
// nearest seed) and log(1 + count), z-scored; the hidden layer runs one unit
// per lane, the heads one per lane.  All lanes return the same value.
__device__ inline float predict_eps(const PredArgs &P, float fv, int metric, int qi, int lane,
                                    float *scratch, float *cost) {
    const float f0 = __shfl(fv, 0);
    const float x = feature_input(lane, fv, f0, metric);
    float *z = scratch;          // [16]
    float *hid = scratch + 16;   // [64]
    float *yv = scratch + 80;    // [16]
    if (lane < ONNG_NFEAT) z[lane] = (x - P.mean[lane]) / P.stdv[lane];
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    float h = 0.0f;
    if (lane < P.H) {
        float s = P.b1[lane];
        for (int t = 0; t < P.F; t++)
            s = fmaf(__uint_as_float((uint32_t)P.w1[lane * P.F + t] << 16), z[t], s);
        h = fmaxf(s, 0.0f);
        hid[lane] = h;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    float y = 0.0f;
    if (lane < P.T) {
        y = P.b2[lane];
        for (int j = 0; j < P.H; j++)
            y = fmaf(__uint_as_float((uint32_t)P.w2[lane * P.H + j] << 16), hid[j], y);
        yv[lane] = y;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    float eps;
    if (P.mode == ONNG_PRED_CURVE) {
        const float lam = P.lambda_pq ? P.lambda_pq[qi] : P.lambda;
        const int G = P.n_cand;
        // score of candidate g = predicted recall - lambda * predicted cost
        float score = -__builtin_inff();
        if (lane < G) score = yv[lane] - lam * (expf(yv[G + lane]) - 1.0f);
        // argmax over lanes, smallest index on ties
        int best = lane;
        for (int m = 32; m >= 1; m >>= 1) {
            float os = __shfl_xor(score, m);
            int ob = __shfl_xor(best, m);
            if (os > score || (os == score && ob < best)) {
                score = os;
                best = ob;
            }
        }
        best = __shfl(best, 0);
        if (best >= G) best = 0;
        eps = P.eps_cand[best];
        *cost = expf(yv[G + best]) - 1.0f;
    } else {
        const int head = P.head_pq ? P.head_pq[qi] : P.head;
        float yh = yv[head] + (P.shift ? P.shift[head] : 0.0f);
        eps = fminf(fmaxf(exp10f(yh) - 0.01f, P.eps_min), P.eps_max);
        *cost = eps;   // the range itself
    }
    return fminf(fmaxf(eps, P.eps_min), P.eps_max);
}

const void *search_kernel_ptr(int dtype, int metric);
const void *reset_counter_kernel_ptr();
const void *clear_tag_kernel_ptr();

}  // namespace onng
