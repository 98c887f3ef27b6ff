// Shared by the two top-k kernels (topk.hip, topk_wide.hip): the kernel
// argument block, tile geometry and the int8 operand staging.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "onng_internal.h"
#include "wave.h"

namespace onng {
namespace topk_detail {

typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int BN = 64;        // base rows per tile
// Per-row list capacity (k rounded up to 8 keys) and candidate slots: a
// tile adds at most BN candidates to a row, whose buffer is merged once it
// holds more than cb - BN.  Small k takes 80 slots (merges after 16
// candidates), which halves the buffer's LDS.
__host__ __device__ inline int topk_kcap(int k) { return (k + 7) / 8 * 8; }
__host__ __device__ inline int topk_cb(int k) { return k <= 16 ? 80 : 128; }

// A staged row is NCH * 64 bytes: u8, NCH k-steps of 64 components (a lane
// feeds 16 of them per step); f32, 4 k-groups of KQ = 4 * NCH components,
// k-group kg covering [kg * KQ, kg * KQ + KQ), so that a lane reads four
// k-steps of its B column with one 16-byte LDS read.  NCH is a compile-time
// constant of the kernel, taken from a short list (rows are zero-extended up
// to it), so the contraction unrolls into one straight run of LDS reads and
// MFMAs.
__host__ __device__ inline int nch_for(int dtype, int dim) {
    if (dtype == ONNG_U8) {
        const int need = (dim + 63) / 64;
        return need <= 1 ? 1 : need <= 2 ? 2 : need <= 4 ? 4 : 8;
    }
    const int need = (dim + 15) / 16;
    return need <= 2 ? 2 : need <= 4 ? 4 : need <= 6 ? 6 : need <= 7 ? 7 : need <= 8 ? 8
           : need <= 12 ? 12 : 16;
}

struct TopkArgs {
    const uint8_t *q;
    int64_t q_pitch;
    int64_t nq;
    const uint8_t *b;         // base rows (or gathered candidate rows)
    int64_t b_pitch;
    int64_t nb;
    const int32_t *b_ids;     // global id of each base row (null: the row index)
    const void *qn;           // query norms (int32 or float), null for cosine
    const void *bn;           // base norms
    int32_t dim;
    int32_t k;
    int32_t kcap;             // list capacity per row (topk_kcap)
    int32_t cb;               // candidate slots per row (topk_cb)
    int32_t bm;               // query rows per block (16 per wave)
    int32_t exclude_self;
    int32_t rotate;           // rows and candidates are the same rows: start at the own tile
    int32_t lds_pitch;        // bytes per staged base row
    int32_t *out_ids;
    void *out_d;
    int32_t side_norms;       // stage the tile's base norms in LDS (L2 metrics)
    int32_t splits;           // blocks sharing one row block's base tiles
    int32_t tiles_per_split;
    uint64_t *part;           // splits > 1: [nq][splits][k] keys of each part
};

// 16 int8 values of (x - 128) at row bytes [c, c+16), zero past dim
__device__ __forceinline__ i32x4 shifted16(const uint8_t *row, int c, int dim) {
    i32x4 out;
#pragma unroll
    for (int w = 0; w < 4; w++) {
        uint32_t v = 0;
#pragma unroll
        for (int b = 0; b < 4; b++) {
            int idx = c + 4 * w + b;
            uint32_t byte = idx < dim ? (uint32_t)(uint8_t)((int)row[idx] - 128) : 0u;
            v |= byte << (8 * b);
        }
        out[w] = (int32_t)v;
    }
    return out;
}

// Bytes of a staged row: what the MFMA operands read (u8: whole 64-byte
// k-steps; f32: 4 k-groups of KQ components), rounded up to an odd number of
// 16-byte chunks, which spreads the 16 rows read together over the LDS banks
// (no more than two rows per bank group).
inline int lds_pitch_for(int dtype, int32_t dim) {
    int p = nch_for(dtype, dim) * 64;
    if ((p / 16) % 2 == 0) p += 16;
    return p;
}

// ---- u8 rows of at most 128 components, many query rows ------------------
// The kernel above keeps every row's list and candidate buffer in LDS: for
// k = 100 that is one block of 64 rows per compute unit, one wave per SIMD,
// whose staging, barriers and epilogue never overlap its MFMAs.  Here a wave
// owns WIDE_RB * 16 = 64 query rows, whose A operands stay in registers for
// the whole sweep, and the lists and candidate buffers live in global memory.
// After the first tiles a row's threshold is tight and few values pass it,
// so those buffers are rarely touched; the LDS holds the staged tile, the
// per-row thresholds and counters and one merge list per wave, so several
// blocks share a compute unit and one wave's epilogue overlaps another's
// MFMAs.  The epilogue's common case is one comparison per distance (the
// column's norm enters as the MFMA chain's initial accumulator, below).
constexpr int WIDE_RB = 4;       // 16-row blocks per wave
constexpr int WIDE_ROWS = 4 * WIDE_RB * 16;   // query rows per block (4 waves)
// Base rows per staged tile: 128 (one barrier pair per 32 MFMAs of each
// 16-row block; 64 was measured 7% slower on the 1M build).
constexpr int WBN = 128;
constexpr int WIDE_CB = 2 * WBN; // global candidate slots per row (a tile adds at most WBN)

__host__ __device__ inline size_t wide_lds_bytes(int lds_pitch, int kcap) {
    return (size_t)WBN * lds_pitch + (size_t)WBN * 12 + (size_t)WIDE_ROWS * 20 +
           (size_t)4 * (kcap + WAVE) * 8;
}

onng_status launch_topk_wide(const TopkArgs &a, int nch, uint64_t *glist, uint64_t *gcand,
                             hipStream_t st);

// f32 rows of at most 128 components: the bf16-screened wide kernel.
constexpr int FW_RB = 2;                  // 16-row blocks per wave
constexpr int FW_ROWS = 4 * FW_RB * 16;   // query rows per block (4 waves)
constexpr int FW_NCH = 4;                 // 64-byte k-steps: 128 bf16 components
constexpr int FW_BN = 64;                 // base rows per staged tile
constexpr int FW_CB = 2 * FW_BN;          // global candidate slots per row
constexpr int FW_LDS_PITCH = FW_NCH * 64 + 16;   // odd count of 16-byte chunks
// |dot(bf16(x), bf16(y)) in f32 - dot(x, y)| <= FW_C |x| |y| for at most 128
// components: 2^-7 + 2^-16 for the rounded factors, 128 * 2^-24 for the sum.
constexpr float FW_C = 0.0078278f + 1.6e-5f;

struct FwRows {
    const uint8_t *q;       // bf16 query rows
    int64_t q_pitch;
    const uint8_t *b;       // bf16 base rows
    int64_t b_pitch;
    const float *ymax;      // max |y| over the base rows
};

__host__ __device__ inline size_t fw_lds_bytes(int kcap) {
    return (size_t)FW_BN * FW_LDS_PITCH + (size_t)FW_BN * 4 + (size_t)FW_ROWS * 20 +
           (size_t)4 * (kcap + WAVE + 64) * 8;
}

onng_status launch_topk_wide_f32(const TopkArgs &a, const onng_vectors *Q, bool same_rows,
                                 uint8_t *qh, uint8_t *bh, uint32_t *ymax, uint64_t *glist,
                                 uint32_t *gcand, hipStream_t st);

}  // namespace topk_detail
}  // namespace onng
