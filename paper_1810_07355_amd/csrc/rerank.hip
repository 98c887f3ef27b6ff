// Exact rerank of per-query candidate pools: distances recomputed from the
// given rows (f32 or f64 accumulation) and the k best (distance, id) kept.
// Used for the ground truth of float data (f32 screening, then f64) and for
// re-scoring low-precision search results from f32 rows.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "dist.h"
#include "onng_internal.h"
#include "wave.h"

namespace onng {

namespace {

constexpr int MAXPOOL = 1024;

__device__ __forceinline__ double elem_at(const uint8_t *row, int dtype, int c, float sc) {
    switch (dtype) {
    case ONNG_U8: return (double)row[c];
    case ONNG_F32: return (double)reinterpret_cast<const float *>(row)[c];
    case ONNG_F16: return (double)(float)__builtin_bit_cast(_Float16, reinterpret_cast<const uint16_t *>(row)[c]);
    case ONNG_BF16: return (double)__uint_as_float((uint32_t)reinterpret_cast<const uint16_t *>(row)[c] << 16);
    default: return (double)fp8_to_f32(row[c]) * (double)sc;
    }
}

template <bool F64>
__global__ void __launch_bounds__(64) rerank_kernel(const uint8_t *q, int64_t qp, int qdt,
                                                    const float *qsc, const uint8_t *b,
                                                    int64_t bp, int bdt, const float *bsc,
                                                    int dim, int metric, const int32_t *pool,
                                                    int psz, int k, int32_t *out_ids,
                                                    void *out_d) {
    __shared__ double dd[MAXPOOL];
    __shared__ int32_t di[MAXPOOL];
    const int64_t qi = blockIdx.x;
    const int lane = threadIdx.x;
    const uint8_t *qr = q + qi * qp;
    const float qs = qsc ? qsc[qi] : 1.0f;
    for (int i = 0; i < psz; i++) {   // one pool entry per step, lanes split the dimensions
        int32_t id = pool[qi * psz + i];
        double acc = 0.0;
        float accf = 0.0f;
        if (id >= 0) {
            const uint8_t *br = b + (int64_t)id * bp;
            const float bs = bsc ? bsc[id] : 1.0f;
            for (int c = lane; c < dim; c += 64) {
                double xv = elem_at(br, bdt, c, bs), qv = elem_at(qr, qdt, c, qs);
                if (F64) {
                    acc += metric == ONNG_L2SQ ? (xv - qv) * (xv - qv) : xv * qv;
                } else {
                    float xf = (float)xv, qf = (float)qv;
                    accf = metric == ONNG_L2SQ ? fmaf(xf - qf, xf - qf, accf) : fmaf(xf, qf, accf);
                }
            }
        }
        for (int m = 32; m >= 1; m >>= 1) {
            if (F64) acc += __shfl_xor(acc, m);
            else accf += __shfl_xor(accf, m);
        }
        if (lane == 0) {
            double d = F64 ? acc : (double)accf;
            if (metric == ONNG_COSINE) d = F64 ? 1.0 - d : (double)(1.0f - accf);
            dd[i] = id >= 0 ? d : __builtin_inf();
            di[i] = id;
        }
    }
    __syncthreads();
    // rank of each entry under (d, id) with missing ids last
    for (int i = lane; i < psz; i += 64) {
        double d = dd[i];
        int32_t id = di[i];
        if (id < 0) continue;
        int rank = 0;
        for (int j = 0; j < psz; j++) {
            if (di[j] < 0) continue;
            rank += dd[j] < d || (dd[j] == d && di[j] < id);
        }
        if (rank < k) {
            out_ids[qi * k + rank] = id;
            if (F64) reinterpret_cast<double *>(out_d)[qi * k + rank] = d;
            else reinterpret_cast<float *>(out_d)[qi * k + rank] = (float)d;
        }
    }
    // pad
    int valid = 0;
    for (int j = 0; j < psz; j++) valid += di[j] >= 0;
    for (int i = valid + lane; i < k; i += 64) {
        out_ids[qi * k + i] = -1;
        if (F64) reinterpret_cast<double *>(out_d)[qi * k + i] = __builtin_inf();
        else reinterpret_cast<float *>(out_d)[qi * k + i] = __builtin_inff();
    }
}

}  // namespace

onng_status rerank_launch(const onng_vectors *Q, const onng_vectors *B, const int32_t *pool,
                          int32_t psz, int32_t k, int32_t use_f64, int32_t *ids, void *dists,
                          hipStream_t st) {
    if (psz > MAXPOOL) {
        set_error("onng_rerank: pool_size above 1024");
        return ONNG_ERR_UNSUPPORTED;
    }
    if (Q->n == 0) return ONNG_OK;
    auto fn = use_f64 ? rerank_kernel<true> : rerank_kernel<false>;
    hipLaunchKernelGGL(fn, dim3((unsigned)Q->n), dim3(64), 0, st,
                       static_cast<const uint8_t *>(Q->data), Q->pitch_bytes, Q->dtype, Q->scale,
                       static_cast<const uint8_t *>(B->data), B->pitch_bytes, B->dtype, B->scale,
                       Q->dim, Q->metric, pool, psz, k, ids, dists);
    ONNG_HIP(hipGetLastError());
    return ONNG_OK;
}

}  // namespace onng
