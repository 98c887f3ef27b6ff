// Wave-level (64-lane) building blocks for gfx950: uniform values, ballots,
// bitonic sorting of one key per lane, and the merge of a sorted batch into a
// sorted array that every set-like structure of the search uses.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace onng {

constexpr int WAVE = 64;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint32_t uniu(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)x);
}
__device__ __forceinline__ uint64_t uni64(uint64_t x) {
    uint32_t lo = uniu((uint32_t)x), hi = uniu((uint32_t)(x >> 32));
    return (uint64_t(hi) << 32) | lo;
}
__device__ __forceinline__ float unif(float x) { return __int_as_float(uni(__float_as_int(x))); }
// value of lane l (wave-uniform l)
__device__ __forceinline__ int64_t readlane64(int64_t v, int l) {
    uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), l);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// number of set bits of m below this lane
__device__ __forceinline__ int mbcnt(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
}

// Orders LDS/global accesses of the lanes of one wave across this point.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ uint64_t shfl_xor64(uint64_t v, int m) {
    uint32_t lo = __shfl_xor((int)(uint32_t)v, m);
    uint32_t hi = __shfl_xor((int)(uint32_t)(v >> 32), m);
    return (uint64_t(hi) << 32) | lo;
}
__device__ __forceinline__ uint64_t shfl64(uint64_t v, int src) {
    uint32_t lo = __shfl((int)(uint32_t)v, src);
    uint32_t hi = __shfl((int)(uint32_t)(v >> 32), src);
    return (uint64_t(hi) << 32) | lo;
}

// ---- lane exchanges without LDS traffic ---------------------------------
// DPP controls (GCN/CDNA encoding): quad permutes act within groups of 4
// lanes, row operations within rows of 16 lanes.
constexpr int DPP_QP_1032 = 0xB1;       // quad_perm [1,0,3,2]: partner lane ^ 1
constexpr int DPP_QP_2301 = 0x4E;       // quad_perm [2,3,0,1]: partner lane ^ 2
constexpr int DPP_ROW_ROR4 = 0x124;     // lane (i + 4) mod 16 of the row
constexpr int DPP_ROW_ROR8 = 0x128;     // lane (i + 8) mod 16 = lane ^ 8
constexpr int DPP_HALF_MIRROR = 0x141;  // lane 7 - i within each group of 8

template <int CTRL, typename T>
__device__ __forceinline__ T dpp(T x) {
    static_assert(sizeof(T) == 4, "32-bit lanes");
    return __builtin_bit_cast(
        T, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x), CTRL, 0xF, 0xF, false));
}

// ds_swizzle in bit mode: partner lane ^ X within each half of the wave
// (X < 32); goes through the LDS crossbar but needs no address.
template <int X, typename T>
__device__ __forceinline__ T swz_xor(T x) {
    static_assert(sizeof(T) == 4 && X > 0 && X < 32, "32-bit lanes, xor within 32");
    return __builtin_bit_cast(T, __builtin_amdgcn_ds_swizzle(__builtin_bit_cast(int, x),
                                                             (X << 10) | 0x1F));
}

// value of lane ^ J, for a compile-time J
template <int J, typename T>
__device__ __forceinline__ T xor_lane(T x) {
    if constexpr (J == 1) return dpp<DPP_QP_1032>(x);
    else if constexpr (J == 2) return dpp<DPP_QP_2301>(x);
    else if constexpr (J == 8) return dpp<DPP_ROW_ROR8>(x);
    else if constexpr (J < 32) return swz_xor<J>(x);
    else return __builtin_bit_cast(T, __shfl_xor(__builtin_bit_cast(int, x), J));
}

template <int J>
__device__ __forceinline__ uint64_t xor_lane64(uint64_t v) {
    uint32_t lo = xor_lane<J>((uint32_t)v);
    uint32_t hi = xor_lane<J>((uint32_t)(v >> 32));
    return (uint64_t(hi) << 32) | lo;
}

// Sum over aligned groups of G lanes (G = 1, 2, 4, 8, 16 or 32); every lane
// of a group receives the group's sum.
template <int G, typename T>
__device__ __forceinline__ T group_sum(T x) {
    if constexpr (G >= 16) {
        x += dpp<DPP_ROW_ROR8>(x);
        x += dpp<DPP_ROW_ROR4>(x);
    } else if constexpr (G == 8) {
        x += dpp<DPP_HALF_MIRROR>(x);
    }
    if constexpr (G >= 4) x += dpp<DPP_QP_2301>(x);
    if constexpr (G >= 2) x += dpp<DPP_QP_1032>(x);
    if constexpr (G >= 32) x += swz_xor<16>(x);
    static_assert(G <= 32, "groups of at most 32 lanes");
    return x;
}

// Same for a wave-uniform run-time G in {4, 8, 16, 32}: quad sums first, then
// the other quad of each 8 (half mirror), the other 8 of each 16 (rotate by
// 8), the other 16 of each 32.
template <typename T>
__device__ __forceinline__ T group_sum_rt(T x, int G) {
    x += dpp<DPP_QP_1032>(x);
    x += dpp<DPP_QP_2301>(x);
    if (G >= 8) x += dpp<DPP_HALF_MIRROR>(x);
    if (G >= 16) x += dpp<DPP_ROW_ROR8>(x);
    if (G >= 32) x += swz_xor<16>(x);
    return x;
}

// Minimum over all 64 lanes (every lane receives it).
__device__ __forceinline__ uint64_t wave_min64(uint64_t v) {
    uint64_t o;
    o = xor_lane64<1>(v); v = o < v ? o : v;
    o = xor_lane64<2>(v); v = o < v ? o : v;
    o = xor_lane64<4>(v); v = o < v ? o : v;
    o = xor_lane64<8>(v); v = o < v ? o : v;
    o = xor_lane64<16>(v); v = o < v ? o : v;
    o = xor_lane64<32>(v); v = o < v ? o : v;
    return v;
}

// One compare-exchange step of the bitonic network: block size K, distance J.
template <int K, int J>
__device__ __forceinline__ uint64_t bitonic_step(uint64_t key, int lane) {
    uint64_t other = xor_lane64<J>(key);
    bool up = (lane & K) == 0;
    bool lower = (lane & J) == 0;
    uint64_t mn = key < other ? key : other;
    uint64_t mx = key < other ? other : key;
    return (lower == up) ? mn : mx;
}

template <int K, int J>
__device__ __forceinline__ uint64_t bitonic_merge(uint64_t key, int lane) {
    key = bitonic_step<K, J>(key, lane);
    if constexpr (J > 1) key = bitonic_merge<K, J / 2>(key, lane);
    return key;
}

// Ascending bitonic sort of one key per lane over the first `width` lanes
// (width a power of two, 1..64, wave-uniform); lanes >= width must hold
// keys no smaller than the keys being sorted (KEY_MAX padding).
__device__ __forceinline__ uint64_t wave_sort(uint64_t key, int width) {
    const int lane = lane_id();
    if (width >= 2) key = bitonic_merge<2, 1>(key, lane);
    if (width >= 4) key = bitonic_merge<4, 2>(key, lane);
    if (width >= 8) key = bitonic_merge<8, 4>(key, lane);
    if (width >= 16) key = bitonic_merge<16, 8>(key, lane);
    if (width >= 32) key = bitonic_merge<32, 16>(key, lane);
    if (width >= 64) key = bitonic_merge<64, 32>(key, lane);
    return key;
}

__device__ __forceinline__ int pow2_at_least(int x) {
    int w = 1;
    while (w < x) w <<= 1;
    return w;
}

// First index i in [0, n) with a[i] >= key (n if none).
template <typename P>
__device__ __forceinline__ int lower_bound_u64(P a, int n, uint64_t key) {
    int lo = 0, hi = n;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (a[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Merge a batch into a sorted array, in place.
//   A[base, base+na) sorted ascending (keys unique); batch: lane j < nb holds
//   the j-th smallest batch key (sorted across lanes), other lanes KEY_MAX.
//   `stage` is 64 scratch keys.  Output occupies A[base, base + min(na+nb, cap)).
//   Elements whose merged position is >= cap are handed to `spill(pos - cap,
//   key)` (pos relative to base).  Returns na + nb.
// A's elements move to higher indices only, so they are moved top chunk
// first, each chunk read completely before it is written; batch keys are
// written last.
template <typename PA, typename PS, typename Spill>
__device__ __forceinline__ int merge_sorted(PA A, int base, int na, uint64_t bkey, int nb,
                                            int cap, PS stage, Spill spill) {
    const int lane = lane_id();
    stage[lane] = bkey;
    wave_sync();
    // destination of my batch key
    int bpos = 0;
    if (lane < nb) bpos = lane + lower_bound_u64(A + base, na, bkey);
    // move A's elements, top chunk first; a chunk whose largest element is
    // below the smallest batch key stays in place, and so do all below it
    const uint64_t bmin = nb > 0 ? stage[0] : ~0ull;
    for (int c0 = ((na - 1) >> 6) << 6; c0 >= 0; c0 -= WAVE) {
        if (A[base + min(c0 + WAVE, na) - 1] < bmin) break;
        int i = c0 + lane;
        uint64_t a = 0;
        int apos = 0;
        if (i < na) {
            a = A[base + i];
            apos = i + lower_bound_u64(stage, nb, a);
        }
        wave_sync();
        if (i < na) {
            if (apos < cap) A[base + apos] = a;
            else spill(apos - cap, a);
        }
        wave_sync();
    }
    if (lane < nb) {
        if (bpos < cap) A[base + bpos] = bkey;
        else spill(bpos - cap, bkey);
    }
    wave_sync();
    return na + nb;
}

struct NoSpill {
    __device__ void operator()(int, uint64_t) const {}
};

}  // namespace onng
