// Low-precision storage of f32 rows: f16 and bf16 (round to nearest even),
// and OCP fp8 e4m3fn with a per-row f32 scale (nearest even, saturating).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "onng_internal.h"

namespace onng {

namespace {

__device__ __forceinline__ uint32_t f32_to_bf16(float x) {
    uint32_t b = __float_as_uint(x);
    if ((b & 0x7fffffffu) > 0x7f800000u) return (b >> 16) | 0x40u;   // NaN stays NaN
    b += 0x7fffu + ((b >> 16) & 1u);
    return b >> 16;
}

__device__ __forceinline__ uint32_t f32_to_f16(float x) {
    _Float16 h = (_Float16)x;   // v_cvt_f16_f32, round to nearest even
    return __builtin_bit_cast(uint16_t, h);
}

// e4m3fn: bias 7, largest finite 448 = 1.75 * 2^8, smallest normal 2^-6,
// subnormal spacing 2^-9; S.1111.111 is NaN.
__device__ __forceinline__ uint32_t f32_to_fp8(float x) {
    uint32_t sign = (__float_as_uint(x) >> 31) << 7;
    if (__builtin_isnan(x)) return sign | 0x7fu;
    float a = fabsf(x);
    if (!(a < 448.0f)) return sign | 0x7eu;                 // saturate
    if (a < 0x1p-6f) {
        uint32_t m = (uint32_t)rintf(a * 0x1p9f);          // exact scaling, then RNE
        return sign | m;                                   // m == 8 is the smallest normal
    }
    int e;
    frexpf(a, &e);
    int E = e - 1;                                         // a in [2^E, 2^(E+1))
    float mant = rintf(ldexpf(a, 3 - E));                  // in [8, 16]
    uint32_t M = (uint32_t)mant;
    if (M == 16u) { M = 8u; E += 1; }
    if (E > 8) return sign | 0x7eu;
    return sign | ((uint32_t)(E + 7) << 3) | (M - 8u);
}

__global__ void encode_kernel(const float *src, int64_t n, int dim, int dtype, uint8_t *dst,
                              int64_t pitch, float *scale) {
    int64_t row = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
    int lane = threadIdx.x & 63;
    if (row >= n) return;
    const float *x = src + row * dim;
    uint8_t *out = dst + row * pitch;
    float s = 1.0f;
    if (dtype == ONNG_FP8_E4M3) {
        float mx = 0.0f;
        for (int c = lane; c < dim; c += 64) mx = fmaxf(mx, fabsf(x[c]));
        for (int m = 32; m >= 1; m >>= 1) mx = fmaxf(mx, __shfl_xor(mx, m));
        s = mx > 0.0f ? __fdiv_rn(mx, 448.0f) : 1.0f;
        if (lane == 0) {
            if (scale) scale[row] = s;
            else *reinterpret_cast<float *>(out + pitch - 4) = s;   // in the row's tail
        }
    }
    int esz = dtype == ONNG_F32 ? 4 : (dtype == ONNG_F16 || dtype == ONNG_BF16) ? 2 : 1;
    const int64_t fill = dtype == ONNG_FP8_E4M3 && !scale ? pitch - 4 : pitch;
    for (int64_t c = lane; c * esz < fill; c += 64) {
        if (c >= dim) {
            for (int b = 0; b < esz; b++) out[c * esz + b] = 0;
            continue;
        }
        float v = x[c];
        switch (dtype) {
        case ONNG_F32: reinterpret_cast<float *>(out)[c] = v; break;
        case ONNG_F16: reinterpret_cast<uint16_t *>(out)[c] = (uint16_t)f32_to_f16(v); break;
        case ONNG_BF16: reinterpret_cast<uint16_t *>(out)[c] = (uint16_t)f32_to_bf16(v); break;
        default: out[c] = (uint8_t)f32_to_fp8(__fdiv_rn(v, s)); break;
        }
    }
}

}  // namespace

onng_status encode_launch(const float *src, int64_t n, int32_t dim, int32_t dtype, void *dst,
                          int64_t pitch, float *scale, hipStream_t st) {
    if (n == 0) return ONNG_OK;
    hipLaunchKernelGGL(encode_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, src, n, dim,
                       dtype, static_cast<uint8_t *>(dst), pitch, scale);
    ONNG_HIP(hipGetLastError());
    return ONNG_OK;
}

}  // namespace onng
