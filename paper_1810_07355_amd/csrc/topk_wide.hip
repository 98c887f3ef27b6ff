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

// ---- f32 rows of at most 128 components, many query rows: a bf16 screen --
// The contraction runs on the bf16 matrix cores (16x16x32) over bf16 copies
// of the rows.  Rounding each factor to 8 significant bits and accumulating
// at most 128 products in f32 leaves the dot product within
// FW_C * |x| * |y| of the exact one, so a value whose approximate distance
// is below the row's threshold by more than that bound cannot be a
// candidate; the others are.  A candidate's distance is computed exactly in
// f32 from the f32 rows when its row's buffer is merged, so the lists and
// thresholds hold exact keys and the result equals an f32 brute force.
// The operand layout of 16x16x32 bf16 is that of 16x16x64 int8 (16
// consecutive bytes of a row per lane), so the staging and the reads are
// the u8 kernel's, over 256-byte bf16 rows.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int MT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
topk_f32_wide_kernel(TopkArgs a, FwRows h, uint64_t *glist, uint32_t *gcand) {
    constexpr int RB = FW_RB;
    constexpr int CPR = FW_NCH * 4;          // 16-byte chunks of a bf16 row (256 bytes)
    constexpr int STG = FW_BN * CPR / 256;   // chunks each thread stages per tile
    constexpr int RPW = RB * 16;             // query rows per wave
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int lane = lane_id();
    const int wv = threadIdx.x / WAVE;
    const int64_t row0 = (int64_t)blockIdx.x * FW_ROWS;
    const int wl0 = wv * RPW;
    const int64_t wrow0 = row0 + wl0;
    const int lpitch = FW_LDS_PITCH;

    // LDS: [tile FW_BN*lpitch][-bn/2 FW_BN][tau][|x|^2][cnt][nlist]
    //      [per wave: list kcap + stage 64 keys + the query row, 128 floats]
    char *p = smem;
    uint8_t *btile = reinterpret_cast<uint8_t *>(p);
    p += (size_t)FW_BN * lpitch;
    float *t_nh = reinterpret_cast<float *>(p);
    p += FW_BN * 4;
    uint64_t *tau = reinterpret_cast<uint64_t *>(p);
    p += FW_ROWS * 8;
    float *q_n2 = reinterpret_cast<float *>(p);
    p += FW_ROWS * 4;
    int32_t *cnt = reinterpret_cast<int32_t *>(p);
    p += FW_ROWS * 4;
    int32_t *nlist = reinterpret_cast<int32_t *>(p);
    p += FW_ROWS * 4;
    uint64_t *scr = reinterpret_cast<uint64_t *>(p) + (size_t)wv * (a.kcap + WAVE + 64);
    uint64_t *stage = scr + a.kcap;
    float *qrow_l = reinterpret_cast<float *>(stage + WAVE);   // 128 floats

    const float *qn = reinterpret_cast<const float *>(a.qn);
    const float *bnorm = reinterpret_cast<const float *>(a.bn);
    for (int i = threadIdx.x; i < FW_ROWS; i += blockDim.x) {
        tau[i] = KEY_MAX;
        cnt[i] = 0;
        nlist[i] = 0;
        q_n2[i] = row0 + i < a.nq ? qn[row0 + i] : 0.0f;
    }

    const int arow = lane & 15;
    const int kg = lane >> 4;
    bf16x8 A[RB][FW_NCH];
#pragma unroll
    for (int rb = 0; rb < RB; rb++) {
        const int64_t qr = wrow0 + rb * 16 + arow;
        const bool ok = qr < a.nq;
        const uint8_t *qp = h.q + (ok ? qr : 0) * h.q_pitch + kg * 16;
#pragma unroll
        for (int s = 0; s < FW_NCH; s++) {
            if (ok) A[rb][s] = *reinterpret_cast<const bf16x8 *>(qp + s * 64);
            else A[rb][s] = bf16x8{};
        }
    }
    const float ymax = *h.ymax;
    auto row_off = [&]() {
        int32_t o = 4 * kg;
        asm volatile("" : "+v"(o));
        return o;
    };
    // Prefilter bound of the rows this lane sees in C: the chain starts at
    // C = -bn/2 (L2) or 0 (cosine) and ends at D.  d <= t needs, for L2,
    // dot - bn/2 >= (|x|^2 - t)/2, for cosine dot >= 1 - t; D is within
    // FW_C |x| |y| (plus f32 rounding, covered by a 1e-5 relative slack) of
    // those exact values.  Rows past the end take +inf; an unfilled list,
    // -inf.
    float tq[RB][4];
    auto load_tq = [&]() {
        const int32_t ro = row_off();
#pragma unroll
        for (int rb = 0; rb < RB; rb++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int lr = wl0 + rb * 16 + ro + r;
                const uint64_t tk = tau[lr];
                const float x2 = q_n2[lr];
                float th;
                if (row0 + lr >= a.nq) {
                    th = __builtin_inff();
                } else if (tk == KEY_MAX) {
                    th = -__builtin_inff();
                } else {
                    const float t = unord_f32((uint32_t)(tk >> 32));
                    const float xl = sqrtf(x2);
                    const float m = FW_C * xl * ymax +
                                    1e-5f * (1.0f + x2 + ymax * ymax + fabsf(t));
                    th = MT == ONNG_COSINE ? (1.0f - t) - m : 0.5f * (x2 - t) - m;
                }
                tq[rb][r] = th;
            }
    };
    __syncthreads();
    load_tq();

    // Merge row lr's candidates into its list: each candidate's exact f32
    // distance from the f32 rows, then sort and merge under (d, id).
    auto flush_row = [&](int lr) {
        const int n = uni(cnt[lr]);
        if (n == 0) return;
        int nl = uni(nlist[lr]);
        const int64_t grow = row0 + lr;
        uint64_t *gl = glist + (size_t)grow * a.kcap;
        const uint32_t *gc = gcand + (size_t)grow * FW_CB;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        for (int i = lane; i < nl; i += WAVE) scr[i] = gl[i];
        {
            const float *qf = reinterpret_cast<const float *>(a.q + grow * a.q_pitch);
            for (int c = lane; c < 128; c += WAVE) qrow_l[c] = c < a.dim ? qf[c] : 0.0f;
        }
        wave_sync();
        for (int c0 = 0; c0 < n; c0 += WAVE) {
            uint64_t key = KEY_MAX;
            if (c0 + lane < n) {
                const uint32_t col = gc[c0 + lane];
                const float *yr = reinterpret_cast<const float *>(a.b + (int64_t)col * a.b_pitch);
                float acc = 0.0f;
                int c = 0;
                for (; c + 4 <= a.dim; c += 4) {
                    const float4 y4 = *reinterpret_cast<const float4 *>(yr + c);
                    const float4 x4 = *reinterpret_cast<const float4 *>(qrow_l + c);
                    if constexpr (MT == ONNG_COSINE) {
                        acc = fmaf(x4.x, y4.x, acc);
                        acc = fmaf(x4.y, y4.y, acc);
                        acc = fmaf(x4.z, y4.z, acc);
                        acc = fmaf(x4.w, y4.w, acc);
                    } else {
                        const float d0 = x4.x - y4.x, d1 = x4.y - y4.y, d2 = x4.z - y4.z,
                                    d3 = x4.w - y4.w;
                        acc = fmaf(d0, d0, acc);
                        acc = fmaf(d1, d1, acc);
                        acc = fmaf(d2, d2, acc);
                        acc = fmaf(d3, d3, acc);
                    }
                }
                for (; c < a.dim; c++) {
                    if constexpr (MT == ONNG_COSINE) acc = fmaf(qrow_l[c], yr[c], acc);
                    else {
                        const float d0 = qrow_l[c] - yr[c];
                        acc = fmaf(d0, d0, acc);
                    }
                }
                const float d = MT == ONNG_COSINE ? 1.0f - acc : acc;
                const uint32_t gid = a.b_ids ? (uint32_t)a.b_ids[col] : col;
                key = make_key(ord_f32(d), gid);
            }
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

    const int ntiles = (int)((a.nb + FW_BN - 1) / FW_BN);
    struct Stage {
        uint4 v[STG];
        float nh;
    };
    auto fetch_into = [&](Stage &S, int t) {
        const int64_t c0 = (int64_t)t * FW_BN;
        const int rows = (int)min<int64_t>(FW_BN, a.nb - c0);
        const uint8_t *tb = h.b + c0 * h.b_pitch;
        const uint32_t bp32 = (uint32_t)h.b_pitch;
#pragma unroll
        for (int j = 0; j < STG; j++) {
            const int i = threadIdx.x + j * 256;
            const int r = i / CPR, c = i - r * CPR;
            S.v[j] = r < rows ? *reinterpret_cast<const uint4 *>(tb + (uint32_t)r * bp32 +
                                                                 (uint32_t)c * 16u)
                              : uint4{0, 0, 0, 0};
        }
        S.nh = 0.0f;
        if (MT == ONNG_L2SQ && threadIdx.x < FW_BN && threadIdx.x < rows)
            S.nh = -0.5f * bnorm[c0 + threadIdx.x];
    };
    auto put_from = [&](const Stage &S) {
#pragma unroll
        for (int j = 0; j < STG; j++) {
            const int i = threadIdx.x + j * 256;
            const int r = i / CPR, c = i - r * CPR;
            *reinterpret_cast<uint4 *>(btile + (uint32_t)r * (uint32_t)lpitch + (uint32_t)c * 16u) =
                S.v[j];
        }
        if (threadIdx.x < FW_BN) t_nh[threadIdx.x] = S.nh;
    };

    const int rot0 = a.rotate ? (int)((row0 / FW_BN) % ntiles) : 0;
    auto tile_at = [&](int i) { const int x = i + rot0; return x >= ntiles ? x - ntiles : x; };
    const bool wave_live = wrow0 < a.nq;

    auto process = [&](int t) {
        if (!wave_live) return;
        const int64_t col0 = (int64_t)tile_at(t) * FW_BN;
        bool added = false;
#pragma unroll 1
        for (int cb = 0; cb < FW_BN / 16; cb++) {
            const uint8_t *bp = btile + (uint32_t)(cb * 16 + arow) * (uint32_t)lpitch + kg * 16;
            bf16x8 bv[FW_NCH];
#pragma unroll
            for (int s = 0; s < FW_NCH; s++) bv[s] = *reinterpret_cast<const bf16x8 *>(bp + s * 64);
            const float nh = t_nh[cb * 16 + arow];
            const f32x4 cinit = {nh, nh, nh, nh};
            f32x4 acc[RB];
#pragma unroll
            for (int rb = 0; rb < RB; rb++) {
                acc[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[rb][0], bv[0], cinit, 0, 0, 0);
#pragma unroll
                for (int s = 1; s < FW_NCH; s++)
                    acc[rb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[rb][s], bv[s], acc[rb], 0, 0, 0);
            }
            uint64_t hit = 0;
#pragma unroll
            for (int rb = 0; rb < RB; rb++)
#pragma unroll
                for (int r = 0; r < 4; r++) hit |= ballot(acc[rb][r] >= tq[rb][r]);
            if (!hit) continue;
            const int64_t col = col0 + cb * 16 + arow;
            const bool cok = col < a.nb;
            const int32_t ro = row_off();
#pragma unroll
            for (int rb = 0; rb < RB; rb++)
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    if (!(cok && acc[rb][r] >= tq[rb][r])) continue;
                    const int lr = wl0 + rb * 16 + ro + r;
                    const int64_t crow = row0 + lr;
                    if (a.exclude_self && col == crow) continue;
                    const int slot = atomicAdd(&cnt[lr], 1);
                    gcand[(size_t)crow * FW_CB + slot] = (uint32_t)col;
                    added = true;
                }
        }
        if (!ballot(added)) return;
        wave_sync();
        const int myr = wl0 + (lane & (RPW - 1));
        const int cr = cnt[myr];
        const int nr = nlist[myr];
        uint64_t over = ballot(lane < RPW && row0 + myr < a.nq &&
                               (cr > FW_CB - FW_BN || (nr == 0 && cr >= a.k)));
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
    for (int r = 0; r < RPW; r++) {
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
            reinterpret_cast<float *>(a.out_d)[grow * a.k + i] =
                i < nl ? unord_f32((uint32_t)(key >> 32)) : __builtin_inff();
        }
    }
}

// f32 rows -> bf16 rows (round to nearest even) of FW_NCH * 64 bytes, zero
// past dim; one thread per component.
__global__ void to_bf16_kernel(const uint8_t *src, int64_t pitch, int64_t n, int dim,
                               uint8_t *dst, int64_t dst_pitch) {
    constexpr int W = FW_NCH * 32;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * W) return;
    const int64_t r = i / W;
    const int c = (int)(i - r * W);
    uint16_t o = 0;
    if (c < dim) {
        const uint32_t u = __float_as_uint(reinterpret_cast<const float *>(src + r * pitch)[c]);
        o = (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
    }
    reinterpret_cast<uint16_t *>(dst + r * dst_pitch)[c] = o;
}

// max over i of sqrt(n2[i]) (non-negative floats order as their bits);
// out must hold 0 first.
__global__ void zero_u32_kernel(uint32_t *p) { *p = 0u; }
__global__ void max_len_kernel(const float *n2, int64_t n, uint32_t *out) {
    float m = 0.0f;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        m = fmaxf(m, n2[i]);
    for (int s = 32; s >= 1; s >>= 1) m = fmaxf(m, __shfl_xor(m, s));
    if (lane_id() == 0) atomicMax(out, __float_as_uint(sqrtf(m)));
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

namespace onng {
namespace topk_detail {

onng_status launch_topk_wide_f32(const TopkArgs &a, const onng_vectors *Q, bool same_rows,
                                 uint8_t *qh, uint8_t *bh, uint32_t *ymax, uint64_t *glist,
                                 uint32_t *gcand, hipStream_t st) {
    const int64_t hp = FW_NCH * 64;
    const int W = FW_NCH * 32;
    hipLaunchKernelGGL(to_bf16_kernel, dim3((unsigned)((a.nb * W + 255) / 256)), dim3(256), 0, st,
                       a.b, a.b_pitch, a.nb, a.dim, bh, hp);
    if (!same_rows)
        hipLaunchKernelGGL(to_bf16_kernel, dim3((unsigned)((a.nq * W + 255) / 256)), dim3(256), 0,
                           st, a.q, a.q_pitch, a.nq, a.dim, qh, hp);
    hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(1), 0, st, ymax);
    hipLaunchKernelGGL(max_len_kernel, dim3(1024), dim3(256), 0, st,
                       reinterpret_cast<const float *>(a.bn), a.nb, ymax);
    ONNG_HIP(hipGetLastError());
    FwRows h;
    h.q = same_rows ? bh : qh;
    h.q_pitch = hp;
    h.b = bh;
    h.b_pitch = hp;
    h.ymax = reinterpret_cast<const float *>(ymax);
    const size_t wl = fw_lds_bytes(a.kcap);
    const void *fn = Q->metric == ONNG_COSINE ? (const void *)topk_f32_wide_kernel<ONNG_COSINE>
                                              : (const void *)topk_f32_wide_kernel<ONNG_L2SQ>;
    ONNG_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)wl));
    TopkArgs args = a;
    void *kargs[] = {&args, &h, &glist, &gcand};
    ONNG_HIP(hipLaunchKernel(fn, dim3((unsigned)((a.nq + FW_ROWS - 1) / FW_ROWS)), dim3(256),
                             kargs, wl, st));
    return ONNG_OK;
}

}  // namespace topk_detail
}  // namespace onng
