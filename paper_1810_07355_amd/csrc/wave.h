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

// Ascending bitonic sort of one key per lane over the first `width` lanes
// (width a power of two, 1..64, wave-uniform); lanes >= width must hold
// keys no smaller than the keys being sorted (KEY_MAX padding).
__device__ __forceinline__ uint64_t wave_sort(uint64_t key, int width) {
    const int lane = lane_id();
    for (int k = 2; k <= width; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            uint64_t other = shfl_xor64(key, j);
            bool up = (lane & k) == 0;
            bool lower = (lane & j) == 0;
            uint64_t mn = key < other ? key : other;
            uint64_t mx = key < other ? other : key;
            key = (lower == up) ? mn : mx;
        }
    }
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
    // move A's elements, top chunk first
    for (int c0 = ((na - 1) >> 6) << 6; c0 >= 0; c0 -= WAVE) {
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
