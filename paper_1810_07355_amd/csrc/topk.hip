// Exact top-k under (distance, id) by brute force on the matrix cores.
//
// The distance matrix is |x|^2 + |y|^2 - 2<x, y>; the dot products are the
// dense contraction and run on MFMA: int8 x int8 -> int32 (16x16x64) for u8
// data, after shifting every component by -128 (the shift cancels in x - y,
// and |<x', y'>| <= dim * 128^2 keeps int32 exact for dim <= 512), f32 x f32
// -> f32 (16x16x4)
// for float data.  Cosine distance on unit vectors is 1 - <x, y>.
//
// A block owns BM query rows (16 per wave) and sweeps the base rows in tiles
// of 64 staged in LDS.  Each row keeps its current k best keys sorted in LDS
// and a buffer of candidates that beat its k-th key; the buffer is sorted and
// merged into the list when it could overflow on the next tile, as soon as it
// holds k keys while the list is empty, and at the end.
// When the query rows alone give too few blocks to fill the chip (e.g. seed
// selection for one query batch), the base tiles are split among several
// blocks per row block, each writes its k best keys, and a second kernel
// merges them (the top k of the union of the parts' top k lists).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "onng_internal.h"
#include "topk_common.h"
#include "wave.h"

namespace onng {

using namespace topk_detail;

namespace {

// ---- per-row norms (int32 |x-128|^2 for u8, f32 |x|^2 otherwise) ----------
__global__ void norms_u8_kernel(const uint8_t *x, int64_t pitch, int64_t n, int dim,
                                int32_t *out) {
    int64_t i = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
    int lane = threadIdx.x & 63;
    if (i >= n) return;
    int32_t s = 0;
    for (int c = lane; c < dim; c += 64) {
        int v = (int)x[i * pitch + c] - 128;
        s += v * v;
    }
    for (int m = 32; m >= 1; m >>= 1) s += __shfl_xor(s, m);
    if (lane == 0) out[i] = s;
}

__global__ void norms_f32_kernel(const uint8_t *x, int64_t pitch, int64_t n, int dim,
                                 float *out) {
    int64_t i = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
    int lane = threadIdx.x & 63;
    if (i >= n) return;
    const float *r = reinterpret_cast<const float *>(x + i * pitch);
    float s = 0.0f;
    for (int c = lane; c < dim; c += 64) s = fmaf(r[c], r[c], s);
    for (int m = 32; m >= 1; m >>= 1) s += __shfl_xor(s, m);
    if (lane == 0) out[i] = s;
}

__global__ void gather_rows_kernel(const uint8_t *src, int64_t pitch, const int32_t *ids,
                                   int64_t n, uint8_t *dst) {
    int64_t i = blockIdx.x;
    if (i >= n) return;
    const uint8_t *s = src + (int64_t)ids[i] * pitch;
    uint8_t *d = dst + i * pitch;
    for (int64_t c = threadIdx.x * 16; c < pitch; c += blockDim.x * 16)
        *reinterpret_cast<uint4 *>(d + c) = *reinterpret_cast<const uint4 *>(s + c);
}

template <int DT, int MT, int NCH>
__global__ void __launch_bounds__(256) topk_kernel(TopkArgs a) {
    constexpr bool U8 = DT == ONNG_U8;
    constexpr int KQ = 4 * NCH;      // f32: components per k-group
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int lane = lane_id();
    const int wv = threadIdx.x / WAVE;
    const int nwaves = a.bm / 16;
    const int64_t row0 = (int64_t)blockIdx.x * a.bm;

    // LDS: [B tile][lists bm*kcap][cands bm*cb][tau bm][cnt bm][nlist bm][stage nwaves*64]
    char *p = smem;
    uint8_t *btile = reinterpret_cast<uint8_t *>(p);
    p += (size_t)BN * a.lds_pitch;
    uint64_t *lists = reinterpret_cast<uint64_t *>(p);
    p += (size_t)a.bm * a.kcap * 8;
    uint64_t *cands = reinterpret_cast<uint64_t *>(p);
    p += (size_t)a.bm * a.cb * 8;
    uint64_t *tau = reinterpret_cast<uint64_t *>(p);
    p += (size_t)a.bm * 8;
    int32_t *cnt = reinterpret_cast<int32_t *>(p);
    p += (size_t)a.bm * 4;
    int32_t *nlist = reinterpret_cast<int32_t *>(p);
    p += (size_t)a.bm * 4;
    uint64_t *stage = reinterpret_cast<uint64_t *>(p) + wv * WAVE;
    p += (size_t)nwaves * WAVE * 8;
    // per tile: base norms and global ids of its 64 rows, when needed
    uint32_t *t_norm = reinterpret_cast<uint32_t *>(p);
    if (a.side_norms) p += BN * 4;
    uint32_t *t_gid = reinterpret_cast<uint32_t *>(p);

    for (int i = threadIdx.x; i < a.bm; i += blockDim.x) {
        tau[i] = KEY_MAX;
        cnt[i] = 0;
        nlist[i] = 0;
    }

    // ---- this wave's 16 query rows as MFMA A operands ----
    const int arow = lane & 15;      // row within the wave's block
    const int kg = lane >> 4;        // k-group of this lane
    const int64_t qrow = row0 + wv * 16 + arow;
    const bool qvalid = qrow < a.nq;
    const uint8_t *qp = a.q + (qvalid ? qrow : 0) * a.q_pitch;
    i32x4 A8[U8 ? NCH : 1];
    float AF[U8 ? 1 : KQ];
    if constexpr (U8) {
#pragma unroll
        for (int s = 0; s < NCH; s++)
            A8[s] = qvalid ? shifted16(qp, s * 64 + kg * 16, a.dim) : i32x4{0, 0, 0, 0};
    } else {
        const float *qf = reinterpret_cast<const float *>(qp);
#pragma unroll
        for (int s = 0; s < KQ; s++) {
            const int c = kg * KQ + s;
            AF[s] = (qvalid && c < a.dim) ? qf[c] : 0.0f;
        }
    }
    // norms of the 4 output rows this lane sees in C (rows 4*kg + r)
    int32_t qn8[4] = {0, 0, 0, 0};
    float qnf[4] = {0, 0, 0, 0};
    int64_t crow[4];
#pragma unroll
    for (int r = 0; r < 4; r++) {
        crow[r] = row0 + wv * 16 + 4 * kg + r;
        if (crow[r] < a.nq) {
            if constexpr (U8) qn8[r] = reinterpret_cast<const int32_t *>(a.qn)[crow[r]];
            else if constexpr (MT == ONNG_L2SQ) qnf[r] = reinterpret_cast<const float *>(a.qn)[crow[r]];
        }
    }
    __syncthreads();

    auto flush_row = [&](int lr) {
        // lr: row within block; whole wave participates
        int n = uni(cnt[lr]);
        if (n == 0) return;
        uint64_t *lst = lists + (size_t)lr * a.kcap;
        int nl = uni(nlist[lr]);
        if (a.kcap <= 16) {
            // short lists (k <= 16): the first kcap lanes hold the list (none
            // while it is empty), the other lanes candidates; one sort of the
            // 64 lanes, the first kcap stay (no merge through LDS)
            const int kl = a.kcap;
            for (int c0 = 0; c0 < n;) {
                const int lo = nl == 0 ? 0 : kl;
                uint64_t key = KEY_MAX;
                if (lane < lo) {
                    if (lane < nl) key = lst[lane];
                } else if (c0 + lane - lo < n) {
                    key = cands[(size_t)lr * a.cb + c0 + lane - lo];
                }
                key = wave_sort(key, WAVE);
                nl = min(nl + min(WAVE - lo, n - c0), a.k);
                if (lane < kl) lst[lane] = key;
                wave_sync();
                c0 += WAVE - lo;
            }
            if (lane == 0) {
                cnt[lr] = 0;
                nlist[lr] = nl;
                tau[lr] = nl == a.k ? lst[a.k - 1] : KEY_MAX;
            }
            wave_sync();
            return;
        }
        for (int c0 = 0; c0 < n; c0 += WAVE) {
            uint64_t key = c0 + lane < n ? cands[(size_t)lr * a.cb + c0 + lane] : KEY_MAX;
            int nb = min(WAVE, n - c0);
            key = wave_sort(key, pow2_at_least(nb));
            int total = merge_sorted(lst, 0, nl, key, nb, a.k, stage, NoSpill());
            nl = min(total, a.k);
        }
        if (lane == 0) {
            cnt[lr] = 0;
            nlist[lr] = nl;
            tau[lr] = nl == a.k ? lst[a.k - 1] : KEY_MAX;
        }
        wave_sync();
    };

    const int ntiles = (int)((a.nb + BN - 1) / BN);
    constexpr int CPR = NCH * 4;     // 16-byte chunks of a staged row
    const int split = blockIdx.y;
    const int t_beg = split * a.tiles_per_split;
    const int t_end = min(ntiles, (split + 1) * a.tiles_per_split);
    // The next tile's rows are read into registers while the current tile is
    // computed (up to STG 16-byte chunks per thread), then stored to LDS.
    constexpr int STG = 9;
    constexpr int total = BN * CPR;
    const bool piped = total <= STG * (int)blockDim.x;
    uint4 stg[STG];
    uint32_t side_n = 0, side_g = 0;
    auto fetch_side = [&](int t) {
        const int64_t col = (int64_t)t * BN + threadIdx.x;
        side_n = 0;
        side_g = 0;
        if (threadIdx.x < BN && col < a.nb) {
            if (a.side_norms) side_n = reinterpret_cast<const uint32_t *>(a.bn)[col];
            if (a.b_ids) side_g = (uint32_t)a.b_ids[col];
        }
    };
    auto put_side = [&]() {
        if (threadIdx.x < BN) {
            if (a.side_norms) t_norm[threadIdx.x] = side_n;
            if (a.b_ids) t_gid[threadIdx.x] = side_g;
        }
    };
    // A thread's chunks sit at the same place in every tile; rows are read
    // with 32-bit offsets from the tile's first row.
    const uint32_t bp32 = (uint32_t)a.b_pitch;
    const int cmax = (int)min<int64_t>(CPR, a.b_pitch / 16);   // chunks a global row holds
    auto load_chunk = [&](const uint8_t *tb, int rows, int i) {
        const int r = i / CPR, c = i - r * CPR;
        if (r < rows && c < cmax)
            return *reinterpret_cast<const uint4 *>(tb + (uint32_t)r * bp32 + (uint32_t)c * 16u);
        return uint4{0, 0, 0, 0};
    };
    auto tile_rows = [&](int t) { return (int)min<int64_t>(BN, a.nb - (int64_t)t * BN); };
    auto tile_ptr = [&](int t) { return a.b + (int64_t)t * BN * a.b_pitch; };
    // Pipelined staging: thread chunk j is i = threadIdx.x + j * blockDim.x,
    // at global offset goff[j] in the tile and LDS offset loff[j] (low 24
    // bits; its chunk index within the row in the high 8).
    uint32_t goff[STG], loff[STG];
#pragma unroll
    for (int j = 0; j < STG; j++) {
        const int i = threadIdx.x + j * blockDim.x;
        const uint32_t r = (uint32_t)(i / CPR), c = (uint32_t)(i % CPR);
        goff[j] = r * bp32 + c * 16u;
        loff[j] = (r * (uint32_t)a.lds_pitch + c * 16u) | (c << 24);
    }
    const bool rows_long = cmax == CPR;
    auto fetch_tile = [&](int t) {
        fetch_side(t);
        const uint8_t *tb = tile_ptr(t);
        const int rows = tile_rows(t);
        if (rows == BN && rows_long) {
#pragma unroll
            for (int j = 0; j < STG; j++) {
                const int i = threadIdx.x + j * blockDim.x;
                if (i < total) stg[j] = *reinterpret_cast<const uint4 *>(tb + goff[j]);
            }
        } else {
#pragma unroll
            for (int j = 0; j < STG; j++) {
                const int i = threadIdx.x + j * blockDim.x;
                stg[j] = i < total ? load_chunk(tb, rows, i) : uint4{0, 0, 0, 0};
            }
        }
    };
    // components at or past dim become 0 (a row's padding may hold anything)
    auto put_chunk_at = [&](uint32_t off, int c, uint4 v) {
        uint32_t w4[4] = {v.x, v.y, v.z, v.w};
        if constexpr (U8) {
            // x - 128 as int8 is x ^ 0x80
#pragma unroll
            for (int w = 0; w < 4; w++) w4[w] ^= 0x80808080u;
            if (c * 16 + 16 > a.dim) {
#pragma unroll
                for (int w = 0; w < 4; w++) {
                    const int valid = a.dim - (c * 16 + 4 * w);
                    if (valid <= 0) w4[w] = 0u;
                    else if (valid < 4) w4[w] &= (1u << (8 * valid)) - 1u;
                }
            }
        } else {
            if (c * 4 + 4 > a.dim) {
#pragma unroll
                for (int w = 0; w < 4; w++)
                    if (c * 4 + w >= a.dim) w4[w] = 0u;
            }
        }
        *reinterpret_cast<uint4 *>(btile + off) = uint4{w4[0], w4[1], w4[2], w4[3]};
    };
    auto put_chunk = [&](int i, uint4 v) {
        const int r = i / CPR, c = i - r * CPR;
        put_chunk_at((uint32_t)r * (uint32_t)a.lds_pitch + (uint32_t)c * 16u, c, v);
    };
    // For a kNN graph of rows in locality order the sweep starts at the row
    // block's own tile and wraps around: the nearest rows come first, so the
    // lists' thresholds are tight from the start and few later candidates
    // pass them.  The result does not depend on the order.
    const int rot0 = a.rotate ? (int)((row0 / BN) % ntiles) : 0;
    auto tile_at = [&](int i) { const int x = i + rot0; return x >= ntiles ? x - ntiles : x; };
    if (piped && t_beg < t_end) fetch_tile(tile_at(t_beg));
    for (int t = t_beg; t < t_end; t++) {
        const int tt = tile_at(t);
        const int64_t col0 = (int64_t)tt * BN;
        __syncthreads();
        // stage 64 base rows
        if (piped) {
#pragma unroll
            for (int j = 0; j < STG; j++) {
                const int i = threadIdx.x + j * blockDim.x;
                if (i < total) put_chunk_at(loff[j] & 0xFFFFFFu, (int)(loff[j] >> 24), stg[j]);
            }
            put_side();
        } else {
            fetch_side(tt);
            put_side();
            const uint8_t *tb = tile_ptr(tt);
            const int rows = tile_rows(tt);
            for (int i = threadIdx.x; i < total; i += blockDim.x) put_chunk(i, load_chunk(tb, rows, i));
        }
        __syncthreads();
        if (piped && t + 1 < t_end) fetch_tile(tile_at(t + 1));
        if (row0 + wv * 16 >= a.nq) continue;

        // ---- 16 query rows x 64 tile columns: four 16x16 blocks, their
        // accumulation chains interleaved ----
        const uint8_t *bbase = btile + arow * a.lds_pitch + (U8 ? kg * 16 : kg * KQ * 4);
        i32x4 acc8[4];
        f32x4 accf[4];
#pragma unroll
        for (int cb = 0; cb < 4; cb++) {
            acc8[cb] = i32x4{0, 0, 0, 0};
            accf[cb] = f32x4{0, 0, 0, 0};
        }
#pragma unroll
        for (int c = 0; c < NCH; c++) {
            if constexpr (U8) {
                i32x4 bv[4];
#pragma unroll
                for (int cb = 0; cb < 4; cb++)
                    bv[cb] = *reinterpret_cast<const i32x4 *>(bbase + cb * 16 * a.lds_pitch + c * 64);
#pragma unroll
                for (int cb = 0; cb < 4; cb++)
                    acc8[cb] = __builtin_amdgcn_mfma_i32_16x16x64_i8(A8[c], bv[cb], acc8[cb], 0, 0, 0);
            } else {
                f32x4 bv[4];
#pragma unroll
                for (int cb = 0; cb < 4; cb++)
                    bv[cb] = *reinterpret_cast<const f32x4 *>(bbase + cb * 16 * a.lds_pitch + c * 16);
#pragma unroll
                for (int j = 0; j < 4; j++)
#pragma unroll
                    for (int cb = 0; cb < 4; cb++)
                        accf[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(AF[4 * c + j], bv[cb][j],
                                                                          accf[cb], 0, 0, 0);
            }
        }

        // ---- epilogue: C layout, lane holds rows 4*kg + r of column arow
        // of each block.  A key can beat a row's list only if its distance
        // part is <= the high half of the row's threshold; that test alone
        // runs on every value, the full one on the few that pass it. ----
        uint64_t thr[4];      // 0 for rows past the end: no key is below it
        uint32_t thi[4];
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const uint64_t tv = tau[wv * 16 + 4 * kg + r];
            thr[r] = crow[r] < a.nq ? tv : 0ull;
            thi[r] = (uint32_t)(thr[r] >> 32);
        }
        uint32_t dd[4][4];
        uint64_t hit[4];      // per block: lanes with a value that passed the prefilter
#pragma unroll
        for (int cb = 0; cb < 4; cb++) {
            int32_t bn8 = 0;
            float bnf = 0.0f;
            if constexpr (U8) bn8 = (int32_t)t_norm[cb * 16 + arow];
            else if constexpr (MT == ONNG_L2SQ) bnf = __uint_as_float(t_norm[cb * 16 + arow]);
            hit[cb] = 0;
#pragma unroll
            for (int r = 0; r < 4; r++) {
                uint32_t dord;
                if constexpr (U8) {
                    dord = (uint32_t)(qn8[r] + bn8 - 2 * acc8[cb][r]);
                } else if constexpr (MT == ONNG_L2SQ) {
                    dord = ord_f32(qnf[r] + bnf - 2.0f * accf[cb][r]);
                } else {
                    dord = ord_f32(1.0f - accf[cb][r]);
                }
                dd[cb][r] = dord;
                hit[cb] |= ballot(dord <= thi[r]);
            }
        }
        const bool partial = col0 + BN > a.nb;
#pragma unroll
        for (int cb = 0; cb < 4; cb++) {
            if (!hit[cb]) continue;
            const int64_t col = col0 + cb * 16 + arow;
            const bool cok = !partial || col < a.nb;
            const uint32_t gid = a.b_ids ? t_gid[cb * 16 + arow] : (uint32_t)col;
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const uint64_t key = make_key(dd[cb][r], gid);
                if (cok && key < thr[r] && !(a.exclude_self && (int64_t)gid == crow[r])) {
                    int lr = wv * 16 + 4 * kg + r;
                    int slot = atomicAdd(&cnt[lr], 1);
                    cands[(size_t)lr * a.cb + slot] = key;
                }
            }
        }
        wave_sync();
        // rows whose buffer could overflow on the next tile
        // (or, while its list is still empty, that already hold k keys: the
        // list then starts from the best k of the first tiles)
        const int cr = cnt[wv * 16 + (lane & 15)];
        const int nr = nlist[wv * 16 + (lane & 15)];
        uint64_t over = ballot(lane < 16 && (cr > a.cb - BN || (nr == 0 && cr >= a.k)));
        while (over) {
            const int r = __builtin_ctzll(over);
            over &= over - 1;
            flush_row(wv * 16 + r);
        }
    }
    __syncthreads();
    if (row0 + wv * 16 >= a.nq) return;
    for (int r = 0; r < 16; r++) {
        int lr = wv * 16 + r;
        int64_t grow = row0 + lr;
        if (grow >= a.nq) break;
        flush_row(lr);
        int nl = uni(nlist[lr]);
        const uint64_t *lst = lists + (size_t)lr * a.kcap;
        if (a.splits > 1) {
            uint64_t *dst = a.part + ((size_t)grow * a.splits + split) * a.k;
            for (int i = lane; i < a.k; i += WAVE) dst[i] = i < nl ? lst[i] : KEY_MAX;
            continue;
        }
        for (int i = lane; i < a.k; i += WAVE) {
            uint64_t key = i < nl ? lst[i] : KEY_MAX;
            a.out_ids[grow * a.k + i] = i < nl ? (int32_t)(uint32_t)key : -1;
            if constexpr (U8) {
                reinterpret_cast<int32_t *>(a.out_d)[grow * a.k + i] =
                    i < nl ? (int32_t)(key >> 32) : INT32_MAX;
            } else {
                reinterpret_cast<float *>(a.out_d)[grow * a.k + i] =
                    i < nl ? unord_f32((uint32_t)(key >> 32)) : __builtin_inff();
            }
        }
    }
}

// One wave per query row: the k best of the splits * k part keys.
template <bool U8>
__global__ void __launch_bounds__(256) merge_parts_kernel(const uint64_t *part, int64_t nq,
                                                          int splits, int k, int kcap,
                                                          int32_t *out_ids, void *out_d) {
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int lane = lane_id();
    const int wv = threadIdx.x / WAVE;
    const int64_t row = (int64_t)blockIdx.x * (blockDim.x / WAVE) + wv;
    if (row >= nq) return;
    uint64_t *lst = reinterpret_cast<uint64_t *>(smem) + (size_t)wv * (kcap + WAVE);
    uint64_t *stage = lst + kcap;
    const uint64_t *src = part + (size_t)row * splits * k;
    const int n = splits * k;
    int nl = 0;
    for (int c0 = 0; c0 < n; c0 += WAVE) {
        uint64_t key = c0 + lane < n ? src[c0 + lane] : KEY_MAX;
        key = wave_sort(key, WAVE);
        // KEY_MAX pads missing entries; they sort last
        int nb = __popcll(ballot(key != KEY_MAX));
        if (nb == 0) continue;
        nl = min(merge_sorted(lst, 0, nl, key, nb, k, stage, NoSpill()), k);
    }
    for (int i = lane; i < k; i += WAVE) {
        uint64_t key = i < nl ? lst[i] : KEY_MAX;
        out_ids[row * k + i] = i < nl ? (int32_t)(uint32_t)key : -1;
        if constexpr (U8)
            reinterpret_cast<int32_t *>(out_d)[row * k + i] = i < nl ? (int32_t)(key >> 32) : INT32_MAX;
        else
            reinterpret_cast<float *>(out_d)[row * k + i] =
                i < nl ? unord_f32((uint32_t)(key >> 32)) : __builtin_inff();
    }
}

// Parts per row block.  With one block per compute unit (the LDS holds one
// block's tile, lists and buffers), the launch takes ceil(blocks / CUs)
// rounds, each as long as one part: about its tiles plus a few tiles' worth
// of list warm-up.  The part count minimises that product (parts keep at
// least 8 tiles).
int topk_splits(int64_t nq, int64_t nb, int bm) {
    const int64_t row_blocks = (nq + bm - 1) / bm;
    const int64_t ntiles = (nb + BN - 1) / BN;
    const int64_t cus = device_cu_count();
    if (row_blocks >= 4 * cus || ntiles < 16) return 1;
    const int64_t top = std::min<int64_t>(64, ntiles / 8);
    int64_t best = 1, best_cost = INT64_MAX;
    for (int64_t sp = 1; sp <= top; sp++) {
        const int64_t rounds = (row_blocks * sp + cus - 1) / cus;
        const int64_t cost = rounds * ((ntiles + sp - 1) / sp + 4);
        if (cost < best_cost) best = sp, best_cost = cost;
    }
    return (int)best;
}


template <int DT, int MT>
const void *topk_fn_for(int nch) {
    if constexpr (DT == ONNG_U8) {
        switch (nch) {
            case 1: return (const void *)topk_kernel<DT, MT, 1>;
            case 2: return (const void *)topk_kernel<DT, MT, 2>;
            case 4: return (const void *)topk_kernel<DT, MT, 4>;
            default: return (const void *)topk_kernel<DT, MT, 8>;
        }
    } else {
        switch (nch) {
            case 2: return (const void *)topk_kernel<DT, MT, 2>;
            case 4: return (const void *)topk_kernel<DT, MT, 4>;
            case 6: return (const void *)topk_kernel<DT, MT, 6>;
            case 7: return (const void *)topk_kernel<DT, MT, 7>;
            case 8: return (const void *)topk_kernel<DT, MT, 8>;
            case 12: return (const void *)topk_kernel<DT, MT, 12>;
            default: return (const void *)topk_kernel<DT, MT, 16>;
        }
    }
}

size_t topk_lds_bytes(int bm, int kcap, int cb, int lds_pitch, int side_words = 0) {
    int nwaves = bm / 16;
    return (size_t)BN * lds_pitch + (size_t)bm * kcap * 8 + (size_t)bm * cb * 8 + (size_t)bm * 16 +
           (size_t)nwaves * WAVE * 8 + (size_t)side_words * BN * 4;
}

// Query rows per block: 64 when the block's tile, lists and buffers fit in
// LDS, else 32.
int topk_side_words(int dtype, int metric, bool cand) {
    return (dtype == ONNG_U8 || metric == ONNG_L2SQ ? 1 : 0) + (cand ? 1 : 0);
}

int topk_bm(int32_t k, int dtype, int32_t dim, int side_words) {
    const int kcap = topk_kcap(k);
    const int lp = lds_pitch_for(dtype, dim);
    return kcap <= 128 && topk_lds_bytes(64, kcap, topk_cb(k), lp, side_words) <= 160 * 1024 ? 64
                                                                                            : 32;
}

// The wide u8 kernel takes over when its 256-row blocks alone fill the chip
// (one per compute unit at least) and the rows fit two 64-byte k-steps.
// The bf16-screened f32 kernel: f32 rows of at most 128 components, its
// 128-row blocks filling the chip.
bool topk_use_wide_f32(const onng_vectors *Q, int64_t nb, int32_t k) {
    return Q->dtype == ONNG_F32 && Q->dim <= FW_NCH * 32 && nb >= 16 * FW_BN &&
           Q->n >= (int64_t)FW_ROWS * device_cu_count() && fw_lds_bytes(topk_kcap(k)) <= 64 * 1024;
}

bool topk_use_wide(const onng_vectors *Q, int64_t nb, int32_t k) {
    return Q->dtype == ONNG_U8 && nch_for(ONNG_U8, Q->dim) <= 2 && nb >= 16 * BN &&
           Q->n >= (int64_t)WIDE_ROWS * device_cu_count() &&
           wide_lds_bytes(lds_pitch_for(ONNG_U8, Q->dim), topk_kcap(k)) <= 64 * 1024;
}

}  // namespace

size_t topk_ws_size(const onng_vectors *Q, const onng_vectors *B, int64_t n_cand, int32_t k) {
    Carver c(nullptr);
    int64_t nb = n_cand > 0 ? n_cand : B->n;
    c.take<float>(Q->n);
    c.take<float>(nb);
    if (n_cand > 0) c.take<uint8_t>((size_t)nb * B->pitch_bytes);
    if (topk_use_wide(Q, nb, k)) {
        c.take<uint64_t>((size_t)Q->n * topk_kcap(k));
        c.take<uint64_t>((size_t)Q->n * WIDE_CB);
        return c.size() + 256;
    }
    if (topk_use_wide_f32(Q, nb, k)) {
        c.take<uint8_t>((size_t)nb * FW_NCH * 64);
        c.take<uint8_t>((size_t)Q->n * FW_NCH * 64);
        c.take<uint32_t>(1);
        c.take<uint64_t>((size_t)Q->n * topk_kcap(k));
        c.take<uint32_t>((size_t)Q->n * FW_CB);
        return c.size() + 256;
    }
    const int sp = topk_splits(Q->n, nb, topk_bm(k, Q->dtype, Q->dim, topk_side_words(Q->dtype, Q->metric, n_cand > 0)));
    if (sp > 1) c.take<uint64_t>((size_t)Q->n * sp * k);
    return c.size() + 256;
}

onng_status launch_topk(const onng_vectors *Q, const onng_vectors *B, const int32_t *cand,
                        int64_t n_cand, int32_t k, int32_t exclude_self, int32_t *ids,
                        void *dists, void *ws, size_t ws_bytes, hipStream_t st) {
    if (!(Q->dtype == B->dtype && (Q->dtype == ONNG_U8 || Q->dtype == ONNG_F32))) {
        set_error("onng_topk: queries and base must both be u8 or both f32");
        return ONNG_ERR_UNSUPPORTED;
    }
    if (Q->dtype == ONNG_U8 && Q->metric != ONNG_L2SQ) {
        set_error("onng_topk: u8 data supports squared L2 only");
        return ONNG_ERR_UNSUPPORTED;
    }
    if (ws_bytes < topk_ws_size(Q, B, cand ? n_cand : 0, k)) {
        set_error("onng_topk: workspace too small");
        return ONNG_ERR_WORKSPACE;
    }
    if (Q->dim != B->dim || Q->dim > (Q->dtype == ONNG_U8 ? 512 : 256)) {
        set_error("onng_topk: dims differ, or above 512 (u8) / 256 (f32)");
        return ONNG_ERR_UNSUPPORTED;
    }
    const bool u8 = Q->dtype == ONNG_U8;
    const int64_t nb = cand ? n_cand : B->n;
    const bool wide = topk_use_wide(Q, nb, k);
    const bool wide_f32 = !wide && topk_use_wide_f32(Q, nb, k);
    Carver c(ws);
    void *qn = c.take<float>(Q->n);
    void *bn = c.take<float>(nb);
    const int sp = (wide || wide_f32) ? 1 : topk_splits(Q->n, nb, topk_bm(k, Q->dtype, Q->dim, topk_side_words(Q->dtype, Q->metric, cand != nullptr)));
    uint64_t *part = sp > 1 ? c.take<uint64_t>((size_t)Q->n * sp * k) : nullptr;
    const uint8_t *brows = static_cast<const uint8_t *>(B->data);
    if (cand && nb > 0) {
        uint8_t *g = c.take<uint8_t>((size_t)nb * B->pitch_bytes);
        hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)nb), dim3(64), 0, st, brows,
                           B->pitch_bytes, cand, nb, g);
        brows = g;
    }
    uint64_t *glist = wide ? c.take<uint64_t>((size_t)Q->n * topk_kcap(k)) : nullptr;
    uint64_t *gcand = wide ? c.take<uint64_t>((size_t)Q->n * WIDE_CB) : nullptr;
    uint8_t *fbh = nullptr, *fqh = nullptr;
    uint32_t *fymax = nullptr, *fcand = nullptr;
    uint64_t *flist = nullptr;
    if (wide_f32) {
        fbh = c.take<uint8_t>((size_t)nb * FW_NCH * 64);
        fqh = c.take<uint8_t>((size_t)Q->n * FW_NCH * 64);
        fymax = c.take<uint32_t>(1);
        flist = c.take<uint64_t>((size_t)Q->n * topk_kcap(k));
        fcand = c.take<uint32_t>((size_t)Q->n * FW_CB);
    }
    if (Q->n > 0) {
        if (u8)
            hipLaunchKernelGGL(norms_u8_kernel, dim3((unsigned)((Q->n + 3) / 4)), dim3(256), 0, st,
                               static_cast<const uint8_t *>(Q->data), Q->pitch_bytes, Q->n, Q->dim,
                               static_cast<int32_t *>(qn));
        else
            hipLaunchKernelGGL(norms_f32_kernel, dim3((unsigned)((Q->n + 3) / 4)), dim3(256), 0,
                               st, static_cast<const uint8_t *>(Q->data), Q->pitch_bytes, Q->n,
                               Q->dim, static_cast<float *>(qn));
    }
    if (nb > 0) {
        if (u8)
            hipLaunchKernelGGL(norms_u8_kernel, dim3((unsigned)((nb + 3) / 4)), dim3(256), 0, st,
                               brows, B->pitch_bytes, nb, B->dim, static_cast<int32_t *>(bn));
        else
            hipLaunchKernelGGL(norms_f32_kernel, dim3((unsigned)((nb + 3) / 4)), dim3(256), 0, st,
                               brows, B->pitch_bytes, nb, B->dim, static_cast<float *>(bn));
    }
    ONNG_HIP(hipGetLastError());
    if (Q->n == 0) return ONNG_OK;

    TopkArgs a;
    a.q = static_cast<const uint8_t *>(Q->data);
    a.q_pitch = Q->pitch_bytes;
    a.nq = Q->n;
    a.b = brows;
    a.b_pitch = B->pitch_bytes;
    a.nb = nb;
    a.b_ids = cand;
    a.qn = qn;
    a.bn = bn;
    a.dim = Q->dim;
    a.k = k;
    a.kcap = topk_kcap(k);
    a.cb = topk_cb(k);
    const int side_words = topk_side_words(Q->dtype, Q->metric, cand != nullptr);
    a.side_norms = Q->dtype == ONNG_U8 || Q->metric == ONNG_L2SQ;
    a.bm = topk_bm(k, Q->dtype, Q->dim, side_words);
    a.exclude_self = exclude_self;
    a.rotate = 0;   // set below once the split count is known
    // the staged tile holds a row's components (zero-extended), not its padding
    a.lds_pitch = lds_pitch_for(Q->dtype, B->dim);
    a.out_ids = ids;
    a.out_d = dists;
    if (wide_f32) {
        a.splits = 1;
        a.tiles_per_split = (int)((nb + FW_BN - 1) / FW_BN);
        a.part = nullptr;
        const bool same = !cand && Q->data == B->data && Q->n == B->n &&
                          Q->pitch_bytes == B->pitch_bytes;
        a.rotate = same ? 1 : 0;
        return launch_topk_wide_f32(a, Q, same, fqh, fbh, fymax, flist, fcand, st);
    }
    if (wide) {
        a.splits = 1;
        a.tiles_per_split = (int)((nb + BN - 1) / BN);
        a.part = nullptr;
        a.rotate = (!cand && Q->data == B->data && Q->n == B->n) ? 1 : 0;
        return launch_topk_wide(a, nch_for(ONNG_U8, Q->dim), glist, gcand, st);
    }
    size_t lds = topk_lds_bytes(a.bm, a.kcap, a.cb, a.lds_pitch, side_words);
    if (lds > 160 * 1024) {
        set_error("onng_topk: k or dim too large for the on-chip tile");
        return ONNG_ERR_UNSUPPORTED;
    }
    const int nch = nch_for(Q->dtype, Q->dim);
    const void *fn;
    if (u8) fn = topk_fn_for<ONNG_U8, ONNG_L2SQ>(nch);
    else if (Q->metric == ONNG_L2SQ) fn = topk_fn_for<ONNG_F32, ONNG_L2SQ>(nch);
    else fn = topk_fn_for<ONNG_F32, ONNG_COSINE>(nch);
    ONNG_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    const int ntiles = (int)((nb + BN - 1) / BN);
    a.splits = sp;
    a.rotate = (!cand && sp == 1 && Q->data == B->data && Q->n == B->n) ? 1 : 0;
    a.tiles_per_split = (ntiles + sp - 1) / sp;
    a.part = part;
    dim3 grid((unsigned)((Q->n + a.bm - 1) / a.bm), (unsigned)sp),
        block((unsigned)(a.bm / 16 * 64));
    void *args[] = {&a};
    ONNG_HIP(hipLaunchKernel(fn, grid, block, args, lds, st));
    if (sp > 1) {
        const int wpb = 4;
        const size_t mlds = (size_t)wpb * (a.kcap + WAVE) * 8;
        const void *mf = u8 ? (const void *)merge_parts_kernel<true>
                            : (const void *)merge_parts_kernel<false>;
        ONNG_HIP(hipFuncSetAttribute(mf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)mlds));
        int64_t nq = Q->n;
        int splits = sp, kk = k, kcap = a.kcap;
        void *margs[] = {&part, &nq, &splits, &kk, &kcap, &ids, &dists};
        ONNG_HIP(hipLaunchKernel(mf, dim3((unsigned)((Q->n + wpb - 1) / wpb)), dim3(wpb * WAVE),
                                 margs, mlds, st));
    }
    return ONNG_OK;
}

}  // namespace onng
