// Distance of one stored row to a query held in registers, computed by a
// group of L lanes: a row is a sequence of 16-byte pieces, lane p of the group
// takes pieces p, p+L, p+2L, ... and the partial sums are reduced across the
// group.  Accumulation is exact (integer) for u8, f32 otherwise.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/onng.h"

namespace onng {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <int DT>
struct DistTraits;

// u8 components, squared L2 as an exact integer.
template <>
struct DistTraits<ONNG_U8> {
    typedef uint32_t acc_t;
};
template <int DT>
struct DistTraits {
    typedef float acc_t;
};

__device__ __forceinline__ u32x4 load16(const uint8_t *p) {
    return *reinterpret_cast<const u32x4 *>(p);
}

__device__ __forceinline__ u32x4 load16_nt(const uint8_t *p) {
    return __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p));
}

// Decode 16 bytes of a row into f32 values and fold them against the query
// piece (also 16 bytes of the same encoding, pre-decoded into qf).
// Each specialisation accumulates into acc.

// ---- u8: sum (x - q)^2 = sum x^2 - 2 sum xq + sum q^2 (q^2 part added once) --
__device__ __forceinline__ uint32_t u8_piece(u32x4 x, u32x4 q) {
    uint32_t s = 0;
#pragma unroll
    for (int w = 0; w < 4; w++) {
        uint32_t xx = __builtin_amdgcn_udot4(x[w], x[w], 0u, false);
        uint32_t xq = __builtin_amdgcn_udot4(x[w], q[w], 0u, false);
        s += xx - 2u * xq;
    }
    return s;
}
__device__ __forceinline__ uint32_t u8_norm_piece(u32x4 q) {
    uint32_t s = 0;
#pragma unroll
    for (int w = 0; w < 4; w++) s = __builtin_amdgcn_udot4(q[w], q[w], s, false);
    return s;
}

// ---- float decoders: 16 bytes -> N floats ----
__device__ __forceinline__ void dec_f32(u32x4 x, float *o) {
#pragma unroll
    for (int w = 0; w < 4; w++) o[w] = __uint_as_float(x[w]);
}
__device__ __forceinline__ void dec_f16(u32x4 x, float *o) {
#pragma unroll
    for (int w = 0; w < 4; w++) {
        _Float16 lo = __builtin_bit_cast(_Float16, (uint16_t)(x[w] & 0xffffu));
        _Float16 hi = __builtin_bit_cast(_Float16, (uint16_t)(x[w] >> 16));
        o[2 * w] = (float)lo;
        o[2 * w + 1] = (float)hi;
    }
}
__device__ __forceinline__ void dec_bf16(u32x4 x, float *o) {
#pragma unroll
    for (int w = 0; w < 4; w++) {
        o[2 * w] = __uint_as_float(x[w] << 16);
        o[2 * w + 1] = __uint_as_float(x[w] & 0xffff0000u);
    }
}
// OCP e4m3fn, one code: exact decode by bit placement (normal) or scaling
// (subnormal).
__device__ __forceinline__ float fp8_to_f32(uint32_t c) {
    uint32_t s = (c >> 7) & 1u, e = (c >> 3) & 15u, m = c & 7u;
    float v = e ? __uint_as_float(((e + 120u) << 23) | (m << 20)) : (float)m * 0x1p-9f;
    return s ? -v : v;
}
// OCP e4m3fn by the hardware conversion (v_cvt_pk_f32_fp8: two codes of one
// 16-bit half per instruction; exact, every code checked against the
// bit-level definition).
__device__ __forceinline__ void dec_fp8(u32x4 x, float *o) {
#pragma unroll
    for (int w = 0; w < 4; w++) {
        auto lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)x[w], false);
        auto hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)x[w], true);
        o[4 * w] = lo[0];
        o[4 * w + 1] = lo[1];
        o[4 * w + 2] = hi[0];
        o[4 * w + 3] = hi[1];
    }
}

template <int DT>
struct Piece {
    static constexpr int N = DT == ONNG_F32 ? 4 : (DT == ONNG_F16 || DT == ONNG_BF16) ? 8 : 16;
    __device__ static __forceinline__ void decode(u32x4 x, float *o) {
        if constexpr (DT == ONNG_F32) dec_f32(x, o);
        else if constexpr (DT == ONNG_F16) dec_f16(x, o);
        else if constexpr (DT == ONNG_BF16) dec_bf16(x, o);
        else dec_fp8(x, o);
    }
};

}  // namespace onng
