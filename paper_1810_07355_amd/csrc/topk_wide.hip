// Exact top-k of u8 rows (squared L2, at most 128 components) for many query
// rows: the wide form of the top-k kernel.  Built with MFMA results in
// ordinary VGPRs (see build.py), which the one-comparison epilogue reads
// directly.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "onng_internal.h"
#include "topk_common.h"
#include "wave.h"

namespace onng {
namespace topk_detail {

namespace {

template <int NCH>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) topk_u8_wide_kernel(TopkArgs a, uint64_t *glist,
                                                           uint64_t *gcand) {
    constexpr int RB = WIDE_RB;
    constexpr int CPR = NCH * 4;          // 16-byte chunks of a staged row
    constexpr int STG = WBN * CPR / 256;   // chunks each thread stages per tile
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int lane = lane_id();
    const int wv = threadIdx.x / WAVE;
    const int64_t row0 = (int64_t)blockIdx.x * WIDE_ROWS;
    const int wl0 = wv * RB * 16;         // the wave's first row within the block
    const int64_t wrow0 = row0 + wl0;

    // LDS: [tile WBN*pitch][norms WBN][-norm/2 WBN][ids WBN][tau][|x'|^2][cnt][nlist]
    //      [per wave: list kcap + stage 64]
    char *p = smem;
    uint8_t *btile = reinterpret_cast<uint8_t *>(p);
    p += (size_t)WBN * a.lds_pitch;
    int32_t *t_norm = reinterpret_cast<int32_t *>(p);
    p += WBN * 4;
    int32_t *t_nhalf = reinterpret_cast<int32_t *>(p);
    p += WBN * 4;
    uint32_t *t_gid = reinterpret_cast<uint32_t *>(p);
    p += WBN * 4;
    uint64_t *tau = reinterpret_cast<uint64_t *>(p);
    p += WIDE_ROWS * 8;
    int32_t *q_norm = reinterpret_cast<int32_t *>(p);   // |x'|^2 of the block's rows
    p += WIDE_ROWS * 4;
    int32_t *cnt = reinterpret_cast<int32_t *>(p);
    p += WIDE_ROWS * 4;
    int32_t *nlist = reinterpret_cast<int32_t *>(p);
    p += WIDE_ROWS * 4;
    uint64_t *scr = reinterpret_cast<uint64_t *>(p) + (size_t)wv * (a.kcap + WAVE);
    uint64_t *stage = scr + a.kcap;

    const int32_t *qnorm = reinterpret_cast<const int32_t *>(a.qn);
    for (int i = threadIdx.x; i < WIDE_ROWS; i += blockDim.x) {
        tau[i] = KEY_MAX;
        cnt[i] = 0;
        nlist[i] = 0;
        q_norm[i] = row0 + i < a.nq ? qnorm[row0 + i] : 0;
    }

    const int arow = lane & 15;
    const int kg = lane >> 4;
    i32x4 A8[RB][NCH];
#pragma unroll
    for (int rb = 0; rb < RB; rb++) {
        const int64_t qrow = wrow0 + rb * 16 + arow;
        const bool ok = qrow < a.nq;
        const uint8_t *qp = a.q + (ok ? qrow : 0) * a.q_pitch;
#pragma unroll
        for (int s = 0; s < NCH; s++)
            A8[rb][s] = ok ? shifted16(qp, s * 64 + kg * 16, a.dim) : i32x4{0, 0, 0, 0};
    }
    // Prefilter bound of the rows this lane sees in C (row rb*16 + 4*kg + r):
    // d = |x'|^2 + bn - 2<x', y'> <= hi(tau) iff bn - 2<x', y'> <= hi(tau) -
    // |x'|^2.  Rows past the end take INT32_MIN, which no value reaches
    // (bn - 2<x', y'> >= -2 * 128^3).
    // The MFMA chain of a column starts from C = -floor(bn / 2), so it ends
    // at D = <x', y'> - floor(bn / 2), and with t = hi(tau) - |x'|^2:
    // d <= hi(tau)  iff  bn - 2<x', y'> <= t  iff  2D >= (bn & 1) - t,
    // which implies D >= ceil(-t / 2) = -(t >> 1).  That one comparison per
    // value is the prefilter; the full (distance, id) test follows for the
    // values that pass it.  Rows past the end take 2^30, which no D reaches
    // (|D| <= 128^3 + 2^20).
    int32_t tq[RB][4];
    // The rarely taken paths below recompute their row addresses from an
    // opaque copy of the lane's row offset, so that the compiler does not
    // keep sixteen of them live across the whole sweep.
    auto row_off = [&]() {
        int32_t o = 4 * kg;
        asm volatile("" : "+v"(o));
        return o;
    };
    auto load_tq = [&]() {
        const int32_t ro = row_off();
#pragma unroll
        for (int rb = 0; rb < RB; rb++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int lr = wl0 + rb * 16 + ro + r;
                const int64_t crow = row0 + lr;
                const uint32_t hi = (uint32_t)(tau[lr] >> 32);
                tq[rb][r] = crow < a.nq
                                ? -(((int32_t)min(hi, (uint32_t)INT32_MAX) - q_norm[lr]) >> 1)
                                : (1 << 30);
            }
    };
    __syncthreads();
    load_tq();

    // Merge row lr's candidates into its list (global), through this wave's
    // LDS list.  The candidates and the list were written by this wave's
    // own stores; the fence orders them before the reads.
    auto flush_row = [&](int lr) {
        const int n = uni(cnt[lr]);
        if (n == 0) return;
        int nl = uni(nlist[lr]);
        const int64_t grow = row0 + lr;
        uint64_t *gl = glist + (size_t)grow * a.kcap;
        const uint64_t *gc = gcand + (size_t)grow * WIDE_CB;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        for (int i = lane; i < nl; i += WAVE) scr[i] = gl[i];
        wave_sync();
        for (int c0 = 0; c0 < n; c0 += WAVE) {
            uint64_t key = c0 + lane < n ? gc[c0 + lane] : KEY_MAX;
            const int nb = min(WAVE, n - c0);
            key = wave_sort(key, pow2_at_least(nb));
            const int total = merge_sorted(scr, 0, nl, key, nb, a.k, stage, NoSpill());
            nl = min(total, a.k);
        }
        for (int i = lane; i < nl; i += WAVE) gl[i] = scr[i];
        if (lane == 0) {
            cnt[lr] = 0;
            nlist[lr] = nl;
            tau[lr] = nl == a.k ? scr[a.k - 1] : KEY_MAX;
        }
        wave_sync();
    };

    const int ntiles = (int)((a.nb + WBN - 1) / WBN);
    const uint32_t bp32 = (uint32_t)a.b_pitch;
    const int cmax = (int)min<int64_t>(CPR, a.b_pitch / 16);
    // Staging: x - 128 as int8 is x ^ 0x80.  Components at or past dim need
    // no masking here: the query operands are zero there, so whatever the
    // tile holds in those places adds nothing to <x', y'>.  The next tile's
    // rows are read into registers while the current tile is computed.
    struct Stage {
        uint4 v[STG];
        int32_t norm;
        uint32_t gid;
    };
    auto fetch_into = [&](Stage &S, int t) {
        const int64_t c0 = (int64_t)t * WBN;
        const int rows = (int)min<int64_t>(WBN, a.nb - c0);
        const uint8_t *tb = a.b + c0 * a.b_pitch;
        if (rows == WBN && cmax == CPR) {
#pragma unroll
            for (int j = 0; j < STG; j++) {
                const int i = threadIdx.x + j * 256;
                const int r = i / CPR, c = i - r * CPR;
                S.v[j] = *reinterpret_cast<const uint4 *>(tb + (uint32_t)r * bp32 + (uint32_t)c * 16u);
            }
        } else {
#pragma unroll
            for (int j = 0; j < STG; j++) {
                const int i = threadIdx.x + j * 256;
                const int r = i / CPR, c = i - r * CPR;
                S.v[j] = (r < rows && c < cmax)
                             ? *reinterpret_cast<const uint4 *>(tb + (uint32_t)r * bp32 +
                                                                (uint32_t)c * 16u)
                             : uint4{0, 0, 0, 0};
            }
        }
        S.norm = 0;
        S.gid = 0;
        if (threadIdx.x < WBN && threadIdx.x < rows) {
            S.norm = reinterpret_cast<const int32_t *>(a.bn)[c0 + threadIdx.x];
            if (a.b_ids) S.gid = (uint32_t)a.b_ids[c0 + threadIdx.x];
        }
    };
    auto put_from = [&](const Stage &S) {
#pragma unroll
        for (int j = 0; j < STG; j++) {
            const int i = threadIdx.x + j * 256;
            const int r = i / CPR, c = i - r * CPR;
            *reinterpret_cast<uint4 *>(btile + (uint32_t)r * (uint32_t)a.lds_pitch +
                                       (uint32_t)c * 16u) =
                uint4{S.v[j].x ^ 0x80808080u, S.v[j].y ^ 0x80808080u, S.v[j].z ^ 0x80808080u,
                      S.v[j].w ^ 0x80808080u};
        }
        if (threadIdx.x < WBN) {
            t_norm[threadIdx.x] = S.norm;
            t_nhalf[threadIdx.x] = -(S.norm >> 1);
            t_gid[threadIdx.x] = S.gid;
        }
    };

    // For a kNN graph of rows in locality order the sweep starts at the
    // block's own tile and wraps around: the nearest rows come first, so the
    // thresholds are tight after a few tiles and few later values pass the
    // prefilter.  The result does not depend on the order.  (An outward
    // order, own +1 -1 +2 -2 ..., was measured 7% slower.)
    const int rot0 = a.rotate ? (int)((row0 / WBN) % ntiles) : 0;
    auto tile_at = [&](int i) { const int x = i + rot0; return x >= ntiles ? x - ntiles : x; };
    const bool wave_live = wrow0 < a.nq;

    auto process = [&](int t) {
        if (!wave_live) return;
        const int64_t col0 = (int64_t)tile_at(t) * WBN;
        bool added = false;
#pragma unroll 1
        for (int cb = 0; cb < WBN / 16; cb++) {
            const uint8_t *bp = btile + (uint32_t)(cb * 16 + arow) * (uint32_t)a.lds_pitch + kg * 16;
            i32x4 bv[NCH];
#pragma unroll
            for (int s = 0; s < NCH; s++) bv[s] = *reinterpret_cast<const i32x4 *>(bp + s * 64);
            const int32_t nh = t_nhalf[cb * 16 + arow];
            const i32x4 cinit = {nh, nh, nh, nh};
            i32x4 acc[RB];
#pragma unroll
            for (int rb = 0; rb < RB; rb++) {
                acc[rb] = __builtin_amdgcn_mfma_i32_16x16x64_i8(A8[rb][0], bv[0], cinit, 0, 0, 0);
#pragma unroll
                for (int s = 1; s < NCH; s++)
                    acc[rb] = __builtin_amdgcn_mfma_i32_16x16x64_i8(A8[rb][s], bv[s], acc[rb], 0, 0, 0);
            }
            uint64_t hit = 0;
#pragma unroll
            for (int rb = 0; rb < RB; rb++)
#pragma unroll
                for (int r = 0; r < 4; r++) hit |= ballot(acc[rb][r] >= tq[rb][r]);
            if (!hit) continue;
            // some value passed the prefilter: the full (distance, id) test,
            // d = |x'|^2 + (bn & 1) - 2D
            const int64_t col = col0 + cb * 16 + arow;
            const bool cok = col < a.nb;
            const uint32_t gid = a.b_ids ? t_gid[cb * 16 + arow] : (uint32_t)col;
            const int32_t b0 = t_norm[cb * 16 + arow] & 1;
            const int32_t ro = row_off();
#pragma unroll
            for (int rb = 0; rb < RB; rb++)
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    if (!(cok && acc[rb][r] >= tq[rb][r])) continue;
                    const int lr = wl0 + rb * 16 + ro + r;
                    const int64_t crow = row0 + lr;
                    const uint64_t key =
                        make_key((uint32_t)(q_norm[lr] + b0 - 2 * acc[rb][r]), gid);
                    if (key < tau[lr] && !(a.exclude_self && (int64_t)gid == crow)) {
                        const int slot = atomicAdd(&cnt[lr], 1);
                        gcand[(size_t)crow * WIDE_CB + slot] = key;
                        added = true;
                    }
                }
        }
        if (!ballot(added)) return;
        wave_sync();
        // rows whose buffer could overflow on the next tile (or, while the
        // list is empty, that already hold k keys)
        const int myr = wl0 + lane;   // the wave owns exactly WAVE rows
        const int cr = cnt[myr];
        const int nr = nlist[myr];
        uint64_t over = ballot(row0 + myr < a.nq &&
                               (cr > WIDE_CB - WBN || (nr == 0 && cr >= a.k)));
        if (!over) return;
        while (over) {
            const int r = __builtin_ctzll(over);
            over &= over - 1;
            flush_row(wl0 + r);
        }
        load_tq();
    };

    Stage SA;
    if (ntiles > 0) fetch_into(SA, tile_at(0));
    for (int t = 0; t < ntiles; t++) {
        __syncthreads();
        put_from(SA);
        __syncthreads();
        if (t + 1 < ntiles) fetch_into(SA, tile_at(t + 1));
        process(t);
    }
    if (!wave_live) return;
    for (int r = 0; r < WAVE; r++) {
        const int lr = wl0 + r;
        const int64_t grow = row0 + lr;
        if (grow >= a.nq) break;
        flush_row(lr);
        const int nl = uni(nlist[lr]);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        const uint64_t *gl = glist + (size_t)grow * a.kcap;
        for (int i = lane; i < a.k; i += WAVE) {
            const uint64_t key = i < nl ? gl[i] : KEY_MAX;
            a.out_ids[grow * a.k + i] = i < nl ? (int32_t)(uint32_t)key : -1;
            reinterpret_cast<int32_t *>(a.out_d)[grow * a.k + i] =
                i < nl ? (int32_t)(key >> 32) : INT32_MAX;
        }
    }
}

}  // namespace

onng_status launch_topk_wide(const TopkArgs &a, int nch, uint64_t *glist, uint64_t *gcand,
                             hipStream_t st) {
    const size_t wl = wide_lds_bytes(a.lds_pitch, a.kcap);
    const void *wf = nch == 1 ? (const void *)topk_u8_wide_kernel<1>
                              : (const void *)topk_u8_wide_kernel<2>;
    ONNG_HIP(hipFuncSetAttribute(wf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)wl));
    TopkArgs args = a;
    void *wargs[] = {&args, &glist, &gcand};
    ONNG_HIP(hipLaunchKernel(wf, dim3((unsigned)((a.nq + WIDE_ROWS - 1) / WIDE_ROWS)), dim3(256),
                             wargs, wl, st));
    return ONNG_OK;
}

}  // namespace topk_detail
}  // namespace onng
