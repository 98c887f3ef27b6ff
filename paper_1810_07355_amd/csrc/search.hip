// Batched best-first k-nearest-neighbour search over an adjusted kNN graph:
// KnnSearch (Algorithm 1) of Iwasaki & Miyazaki, one 64-lane wavefront per query.
//
// Per query the wave keeps, in LDS:
//   pool   the best `pool_q` (distance, id) keys seen so far, sorted.  Its first
//          k entries are the result set R of Algorithm 1; r is the k-th
//          distance once k entries exist.  With a rerank, pool_q = pool_factor*k
//          candidates are kept for the exact pass.
//   S      the candidate set, a sorted array [head, size) of keys that are
//          still within the search range; entries that no longer pass
//          d <= r(1+eps) are cut from its tail (they can never be expanded).
//          Keys that do not fit spill to a per-slot global array and come back
//          when the on-chip part runs below their minimum, so S is exact.
//   vis    the visited set C, on chip for a window of consecutive ids around
//          the first seed (one bit per id; the rows are in locality order, so
//          much of a query's neighbourhood falls in it), and a per-slot
//          global bitset (atomic OR) for the other ids.  A query logs every
//          word it turns non-zero and clears those words when it ends, so
//          the bitset is all zero between queries; it is zeroed as a whole
//          only when the workspace's tag says its state is unknown.
//
// One expansion (pop of s, scan of its first e_p edges) is processed as one
// batch: the unvisited neighbours are marked, their distances computed by the
// whole wave, R updated with all of them, then the ones within the updated
// range inserted into S.  Algorithm 1 interleaves these per neighbour; the
// batch gives the same R, visited set, distance count and pop sequence,
// because r never grows: a neighbour Algorithm 1 would insert with an older,
// larger r but the batch rejects is beyond every later range and could only
// end the search when popped, at a pop where the batch's next candidate ends
// it too.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "dist.h"
#include "onng_internal.h"
#include "search_args.h"
#include "wave.h"

namespace onng {

namespace {

constexpr float F_INF = __builtin_inff();

// (1+eps)^2 for squared L2, 1+eps for cosine, rounded to f32; +inf stays +inf.
__device__ __forceinline__ float range_factor(float eps, int metric) {
    if (__builtin_isinf(eps)) return F_INF;
    double t = __dadd_rn(1.0, (double)eps);
    return metric == ONNG_L2SQ ? (float)__dmul_rn(t, t) : (float)t;
}

// Equation 1 for a predicted eps, in f32 (the value used is reported per
// query, so a replay uses the same integer).
__device__ __forceinline__ uint32_t dynamic_ep(float eps, float e0, float we) {
    float v = floorf(exp10f(we * eps) + e0);
    if (!(v < 4294967040.0f)) return 0xffffffffu;
    return v < 1.0f ? 1u : (uint32_t)v;
}

template <int DT, int MT>
struct Q;

// ----------------------------------------------------------- u8, L2^2 ----
template <>
struct Q<ONNG_U8, ONNG_L2SQ> {
    static constexpr int PPL = 2;
    static constexpr bool INT = true;
    u32x4 q[PPL];
    uint32_t qq;
    __device__ void load(const uint8_t *row, int p, int L, int n16) {
        qq = 0;
#pragma unroll
        for (int t = 0; t < PPL; t++) {
            int pc = p + t * L;
            if (pc < n16) {
                q[t] = load16(row + pc * 16);
                qq += u8_norm_piece(q[t]);
            } else {
                q[t] = u32x4{0, 0, 0, 0};
            }
        }
    }
    // this lane's pieces of a row (zero where the lane has none)
    __device__ void fetch(const uint8_t *row, int p, int L, int n16, u32x4 *x) const {
#pragma unroll
        for (int t = 0; t < PPL; t++) {
            int pc = p + t * L;
            x[t] = pc < n16 ? load16(row + pc * 16) : u32x4{0, 0, 0, 0};
        }
    }
    // sum over this lane's pieces of (x - q)^2
    __device__ uint32_t fold(const u32x4 *x, float) const {
        uint32_t s = qq;
#pragma unroll
        for (int t = 0; t < PPL; t++) s += u8_piece(x[t], q[t]);
        return s;
    }
};

// ------------------------------------------------------ float storage ----
template <int DT, int MT>
struct Q {
    static constexpr int PPL = 2;
    static constexpr int N = Piece<DT>::N;
    static constexpr bool INT = false;
    float q[PPL][N];
    // the query is always f32: its piece t of the stored layout covers
    // components [pc*N, pc*N + N)
    __device__ void load_f32(const float *qrow, int dim, int p, int L, int n16) {
#pragma unroll
        for (int t = 0; t < PPL; t++) {
            int pc = p + t * L;
#pragma unroll
            for (int e = 0; e < N; e++) {
                int c = pc * N + e;
                q[t][e] = (pc < n16 && c < dim) ? qrow[c] : 0.0f;
            }
        }
    }
    __device__ void fetch(const uint8_t *row, int p, int L, int n16, u32x4 *x) const {
#pragma unroll
        for (int t = 0; t < PPL; t++) {
            int pc = p + t * L;
            x[t] = pc < n16 ? load16(row + pc * 16) : u32x4{0, 0, 0, 0};
        }
    }
    // this lane's part of sum (x - q)^2, or of <x, q> for cosine
    __device__ float fold(const u32x4 *x, float sc) const {
        // two accumulation chains (even / odd components) halve the
        // dependent-FMA latency
        float acc[2] = {0.0f, 0.0f};
#pragma unroll
        for (int t = 0; t < PPL; t++) {
            float v[N];
            Piece<DT>::decode(x[t], v);
#pragma unroll
            for (int e = 0; e < N; e++) {
                float xv = v[e];
                // fp8 rows carry a per-row scale: applied per component for
                // L2, once to the dot product for cosine
                if constexpr (DT == ONNG_FP8_E4M3 && MT == ONNG_L2SQ) xv *= sc;
                if constexpr (MT == ONNG_L2SQ) {
                    float df = xv - q[t][e];
                    acc[e & 1] = fmaf(df, df, acc[e & 1]);
                } else {
                    acc[e & 1] = fmaf(xv, q[t][e], acc[e & 1]);
                }
            }
        }
        if constexpr (DT == ONNG_FP8_E4M3 && MT != ONNG_L2SQ) return (acc[0] + acc[1]) * sc;
        return acc[0] + acc[1];
    }
};

template <bool INT>
__device__ __forceinline__ float key_dist(uint64_t key) {
    uint32_t hi = (uint32_t)(key >> 32);
    if constexpr (INT) return (float)hi;
    else return unord_f32(hi);
}

__device__ __forceinline__ float threshold(bool rfull, float r, float f) {
    if (!rfull || __builtin_isinf(f)) return F_INF;
    return __fmul_rn(r, f);
}

struct LdsWave {
    uint64_t *pool;
    uint64_t *S;
    uint64_t *stage;
    uint64_t *stage2;
    uint32_t *ids;
    uint32_t *vis;
    float *misc;
};

}  // namespace

template <int DT, int MT>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(3, 8)))
search_kernel(SearchKArgs a) {
    typedef Q<DT, MT> QT;
    constexpr bool INT = QT::INT;
    extern __shared__ __attribute__((aligned(16))) char smem[];
    const int lane = lane_id();
    const int wib = uni(threadIdx.x / WAVE);   // wave-uniform: derived pointers stay scalar
    const int slot = blockIdx.x * a.waves_per_block + wib;

    char *w = smem + (size_t)wib * a.lds_per_wave;
    LdsWave lds;
    lds.pool = reinterpret_cast<uint64_t *>(w + a.off_pool);
    lds.S = reinterpret_cast<uint64_t *>(w + a.off_s);
    lds.stage = reinterpret_cast<uint64_t *>(w + a.off_stage);
    lds.stage2 = reinterpret_cast<uint64_t *>(w + a.off_stage2);
    lds.ids = reinterpret_cast<uint32_t *>(w + a.off_ids);
    lds.vis = reinterpret_cast<uint32_t *>(w + a.off_vis);
    lds.misc = reinterpret_cast<float *>(w + a.off_misc);
    // 128 keys: the two 64-key stages are adjacent
    uint64_t *const kbuf = lds.stage;

    uint32_t *gbits = a.gbits + (size_t)slot * a.gbits_words;
    int32_t *vlog = a.vlog + (size_t)slot * a.vlog_cap;
    uint64_t *spill0 = a.spill + (size_t)slot * 2 * a.spill_cap;
    // Every launch leaves each slot's bitset all zero (queries clear the words
    // they set).  The workspace tag, written by the last wave of a launch,
    // records the layout that state belongs to; when the caller does not vouch
    // for the workspace or the tag differs, each slot zeroes its bitset first.
    const bool ws_known =
        a.ws_reuse && __hip_atomic_load(a.ws_tag_at, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
                          a.ws_tag;
    if (!ws_known) {
        u32x4 *g4 = reinterpret_cast<u32x4 *>(gbits);
        for (int64_t i = lane; i < a.gbits_words / 4; i += WAVE) g4[i] = u32x4{0, 0, 0, 0};
        __threadfence();
    }

    const int L = a.lanes_per_row;
    const int p = lane & (L - 1);
    const int grp = lane / L;
    const int rpp = WAVE / L;   // rows per pass
    // on-chip visited bits: 2^vis_log2 words, one bit per id of a window of
    // W consecutive ids (the rows are in locality order, so a query's
    // neighbourhood has nearby ids); other ids use the global bitset
    const uint32_t W = a.vis_log2 > 0 ? (32u << a.vis_log2) : 0u;

    for (;;) {
        int ticket = 0;
        if (lane == 0) ticket = atomicAdd(a.counter, 1);
        ticket = uni(__shfl(ticket, 0));
        if (ticket >= a.nq) break;
        const int qi = a.order ? uni(a.order[ticket]) : ticket;
        const uint64_t t_start = wall_clock64();

        // ---------------------------------------------- per-query setup --
        const int k = a.k_pq ? min(max(uni(a.k_pq[qi]), 1), a.k_stride) : a.k;
        float eps = a.eps_pq ? unif(a.eps_pq[qi]) : a.eps;
        uint32_t ep = a.ep_pq ? uniu(a.ep_pq[qi]) : a.ep;
        if (a.range_from) {
            eps = unif(a.range_from[qi].eps);
            ep = uniu(a.range_from[qi].e_p);
        }
        float cost = eps;
        float f = range_factor(eps, MT);
        if (a.two_phase) {
            f = F_INF;
            ep = a.ep_first;
        }
        const int pool_q = a.has_rr ? min(a.pool_cap, max(k, a.pool_factor * k)) : k;
        int max_dc = a.max_dc_pq ? uni(a.max_dc_pq[qi]) : a.max_dc;
        if (max_dc <= 0) max_dc = INT32_MAX;
        // budget relative to the predicted cost of the chosen range
        auto cost_budget = [&](float c) {
            if (a.max_dc_factor > 0.0f) {
                float b = fminf(a.max_dc_factor * c, 2.0e9f);
                max_dc = min(max_dc, max(64, (int)b));
            }
        };
        if (a.range_from) cost_budget(unif(a.range_from[qi].cost));

        QT qr;
        const uint8_t *qrow = a.qry + (size_t)qi * a.q_pitch;
        if constexpr (INT) qr.load(qrow, p, L, a.n16);
        else qr.load_f32(reinterpret_cast<const float *>(qrow), a.dim, p, L, a.n16);

        // state
        int npool = 0;
        int head = 0, size = 0;
        int spill_n = 0, spill_sel = 0;
        uint64_t spill_min = KEY_MAX;
        int log_n = 0;          // words of the global bitset this query made non-zero
        int dc = 0, hops = 0;
        int scanned = 0;   // adjacency entries read (sum of min(deg, e_p) over expansions)
        int flags = 0;
        bool rfull = false;
        float r = F_INF;
        // guessed next expansion (see the expansion loop)
        constexpr uint32_t NO_SPEC = 0xFFFFFFFFu;
        uint32_t spec_id = NO_SPEC;
        int64_t spec_e0 = 0, spec_deg = 0;
        uint32_t spec_nb = 0, spec_nb1 = 0;
        bool spec_vis = false;
        // per guessed id, read ahead: its visited bit, and whether its bitset word was zero
        bool spec_bit = false, spec_bit1 = false, spec_wz = false, spec_wz1 = false;

        // the on-chip window: W ids around the first seed, within [0, n)
        uint32_t w0 = 0;
        if (W) {
            const int32_t s0 = a.n_seeds > 0 ? a.seeds[(size_t)qi * a.n_seeds] : -1;
            int64_t c = (s0 >= 0 && (int64_t)s0 < a.n_base) ? (int64_t)s0 - (int64_t)(W / 2) : 0;
            const int64_t hi = a.n_base > (int64_t)W ? a.n_base - (int64_t)W : 0;
            c = c < 0 ? 0 : (c > hi ? hi : c);
            w0 = (uint32_t)uni((int)(c & ~31LL));
            for (int i = lane; i < (1 << a.vis_log2); i += WAVE) lds.vis[i] = 0u;
        }
        wave_sync();

        // -------------------------------------------------- helpers ------
        // Mark a batch of ids visited; returns whether this lane's id is new.
        // known_ok: the caller read this id's bitset word after every earlier
        // mark of the query (known_bit: the id's bit, known_zero: the whole
        // word was zero); the mark then needs no reply, and *from_known tells
        // the caller the answer came from that word (an id repeated in one
        // list looks new in each copy: see dedupe_known).
        auto visit = [&](bool valid, uint32_t id, bool known_ok = false, bool known_bit = false,
                         bool known_zero = false, bool *from_known = nullptr) -> bool {
            const uint32_t off = id - w0;   // wraps below the window
            const bool inw = valid && off < W;
            const bool outw = valid && !inw;
            bool isnew = false, first = false;
            if (inw) {
                const uint32_t bit = 1u << (off & 31);
                isnew = (atomicOr(&lds.vis[off >> 5], bit) & bit) == 0u;
            } else if (outw) {
                const uint32_t bit = 1u << (id & 31);
                if (known_ok) {
                    isnew = !known_bit;
                    first = known_zero;
                    if (isnew)
                        __hip_atomic_fetch_or(&gbits[id >> 5], bit, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
                    if (from_known) *from_known = isnew;
                } else {
                    const uint32_t old = atomicOr(&gbits[id >> 5], bit);
                    isnew = (old & bit) == 0u;
                    first = old == 0u;
                }
            }
            // log each word when this query turns it non-zero
            const bool logged = isnew && first;
            const uint64_t m = ballot(logged);
            if (logged && log_n + mbcnt(m) < a.vlog_cap) vlog[log_n + mbcnt(m)] = (int32_t)(id >> 5);
            log_n += __popcll(m);
            return isnew;
        };

        // Ids of chunk 0 and chunk 1 of a guessed expansion that were found new
        // from words read before it (k0/k1 set) are new in every copy when the
        // list repeats an id.  Keep the first copy in list order (chunk 0
        // before chunk 1, lower lane first), as Algorithm 1's visited set does:
        // a bitmap of 8192 id hashes in LDS finds the lanes whose hash was
        // already taken, and only for those the wave compares ids exactly.
        // The bitmap lives in the distance-key buffer, unused until the batch.
        auto dedupe_known = [&](uint32_t id0, bool &n0, bool k0, uint32_t id1, bool &n1,
                                bool k1) {
            uint32_t *bm = reinterpret_cast<uint32_t *>(kbuf);   // 1 KiB
            reinterpret_cast<u32x4 *>(bm)[lane] = u32x4{0, 0, 0, 0};
            wave_sync();
            bool c0 = false, c1 = false;
            if (k0) {
                const uint32_t h = id0 & 8191u, b = 1u << (h & 31);
                c0 = (atomicOr(&bm[h >> 5], b) & b) != 0u;
            }
            if (k1) {
                const uint32_t h = id1 & 8191u, b = 1u << (h & 31);
                c1 = (atomicOr(&bm[h >> 5], b) & b) != 0u;
            }
            uint64_t cm0 = ballot(c0), cm1 = ballot(c1);
            uint64_t drop0 = 0, drop1 = 0;
            while (cm0 | cm1) {
                uint32_t cid;
                if (cm0) {
                    const int src = (int)__builtin_ctzll(cm0);
                    cm0 &= cm0 - 1;
                    cid = (uint32_t)__builtin_amdgcn_readlane((int)id0, src);
                } else {
                    const int src = (int)__builtin_ctzll(cm1);
                    cm1 &= cm1 - 1;
                    cid = (uint32_t)__builtin_amdgcn_readlane((int)id1, src);
                }
                uint64_t e0 = ballot(k0 && id0 == cid), e1 = ballot(k1 && id1 == cid);
                if (e0) e0 &= e0 - 1;   // the first copy stays new
                else e1 &= e1 - 1;
                drop0 |= e0;
                drop1 |= e1;
            }
            n0 = n0 && !((drop0 >> lane) & 1u);
            n1 = n1 && !((drop1 >> lane) & 1u);
            wave_sync();
        };

        // Distances of rows lds.ids[0..u) -> kbuf[i] as keys (u <= 128).  A lane
        // group of L lanes takes one row; the loads of UP row passes are
        // issued together so that several rows per lane are in flight.
        auto batch_keys = [&](int u) {
            constexpr int UP = DT == ONNG_FP8_E4M3 ? 2 : 4;
            for (int r0 = 0; r0 < u; r0 += rpp * UP) {
                u32x4 x[UP][QT::PPL];
                uint32_t rid[UP];
                float sc[UP];
#pragma unroll
                for (int up = 0; up < UP; up++) {
                    int row = r0 + up * rpp + grp;
                    rid[up] = row < u ? lds.ids[row] : 0u;
                }
#pragma unroll
                for (int up = 0; up < UP; up++) {
                    int row = r0 + up * rpp + grp;
                    const uint8_t *rp = a.base + (size_t)rid[up] * a.base_pitch;
                    qr.fetch(rp, p, L, row < u ? a.n16 : 0, x[up]);
                    sc[up] = 1.0f;
                    if constexpr (DT == ONNG_FP8_E4M3) {
                        // the row's scale (in its own line when the rows carry
                        // it); the lanes of a row read one address
                        float v = 1.0f;
                        if (row < u)
                            v = a.scale_in_row ? *reinterpret_cast<const float *>(rp + a.base_pitch - 4)
                                               : a.base_scale[rid[up]];
                        sc[up] = v;
                    }
                }
#pragma unroll
                for (int up = 0; up < UP; up++) {
                    int row = r0 + up * rpp + grp;
                    typename DistTraits<DT>::acc_t acc = qr.fold(x[up], sc[up]);
                    // sum over the L lanes of the row (DPP, no LDS round trip)
                    acc = group_sum_rt(acc, L);
                    if (row < u && p == 0) {
                        uint32_t dord;
                        if constexpr (INT) dord = acc;
                        else dord = ord_f32(MT == ONNG_COSINE ? 1.0f - acc : acc);
                        kbuf[row] = make_key(dord, rid[up]);
                    }
                }
            }
            wave_sync();
        };

        // spill a key that fell past the on-chip capacity of S; spilled keys
        // arrive in ascending order, so index 0 is the smallest of this merge
        uint64_t first_spilled = KEY_MAX;
        auto spill_put = [&](int idx, uint64_t key) {
            int pos = spill_n + idx;
            if (idx == 0) first_spilled = key;
            if (pos < a.spill_cap) spill0[(size_t)spill_sel * a.spill_cap + pos] = key;
        };

        // Merge sorted batch (lane j < nb holds j-th key) into S.
        auto s_insert = [&](uint64_t key, int nb) {
            if (nb == 0) return;
            if (size + nb > a.s_cap && head > 0) {
                // compact the live part to the front
                int live = size - head;
                for (int c0 = 0; c0 < live; c0 += WAVE) {
                    uint64_t v = 0;
                    if (c0 + lane < live) v = lds.S[head + c0 + lane];
                    wave_sync();
                    if (c0 + lane < live) lds.S[c0 + lane] = v;
                    wave_sync();
                }
                size = live;
                head = 0;
            }
            first_spilled = KEY_MAX;
            int total = merge_sorted(lds.S, head, size - head, key, nb, a.s_cap - head, lds.stage,
                                     spill_put);
            int over = total - (a.s_cap - head);
            if (over > 0) {
                uint64_t mn = first_spilled;
                for (int m = 32; m >= 1; m >>= 1) {
                    uint64_t o = shfl_xor64(mn, m);
                    mn = o < mn ? o : mn;
                }
                mn = uni64(mn);
                spill_min = mn < spill_min ? mn : spill_min;
                if (spill_n + over > a.spill_cap) flags |= ONNG_QF_CAPACITY;
                spill_n = min(spill_n + over, (int)a.spill_cap);
                flags |= ONNG_QF_SPILLED;
                size = a.s_cap;
            } else {
                size = head + total;
            }
        };

        // Drop S entries beyond the range (a suffix of the sorted array).
        auto s_prune = [&](float thr) {
            if (size == head || __builtin_isinf(thr)) return;
            if (key_dist<INT>(lds.S[size - 1]) <= thr) return;   // all within range
            // first index with d > thr: every stride-th entry first, then the
            // entries between the last sample within range and the next one
            const int n = size - head;
            const int stride = (n + WAVE - 1) / WAVE;
            const int i1 = head + lane * stride;
            uint64_t m = ballot(i1 < size && key_dist<INT>(lds.S[i1]) > thr);
            const int ns = (n + stride - 1) / stride;
            const int b = m ? (int)__builtin_ctzll(m) : ns;
            if (b == 0) {
                size = head;
                return;
            }
            const int lo = head + (b - 1) * stride + 1;
            const int hi = min(head + b * stride, size);
            int cut = hi;
            for (int c = lo; c < hi; c += WAVE) {
                const int i2 = c + lane;
                uint64_t m2 = ballot(i2 < hi && key_dist<INT>(lds.S[i2]) > thr);
                if (m2) {
                    cut = c + (int)__builtin_ctzll(m2);
                    break;
                }
            }
            size = uni(cut);
        };

        // Merge sorted keys into the pool (R and rerank candidates).
        auto pool_insert = [&](uint64_t key, int nb) {
            // a full pool only takes keys below its last one (a sorted prefix)
            if (npool == pool_q) nb = __popcll(ballot(lane < nb && key < lds.pool[pool_q - 1]));
            if (nb == 0) return;
            int total = merge_sorted(lds.pool, 0, npool, key, nb, pool_q, lds.stage, NoSpill());
            npool = min(total, pool_q);
            if (npool >= k) {
                rfull = true;
                r = key_dist<INT>(lds.pool[k - 1]);
                r = unif(r);
            }
        };

        // Process a sorted batch: R first (absorb_pool), then the range test
        // with the new r and the insertion into S (absorb_s).
        auto absorb_pool = [&](uint64_t key, int u) { pool_insert(key, u); };
        auto absorb_s = [&](uint64_t key, int u, bool to_s) {
            float thr = threshold(rfull, r, f);
            // the batch is sorted, so the keys within range are a prefix
            bool keep = lane < u && key_dist<INT>(key) <= thr;
            if (!to_s) keep = lane < u;
            const int nk = __popcll(ballot(keep));
            const uint64_t ck = lane < nk ? key : KEY_MAX;
            s_prune(thr);
            s_insert(ck, nk);
        };
        auto absorb = [&](uint64_t key, int u, bool to_s) {
            absorb_pool(key, u);
            absorb_s(key, u, to_s);
        };

        // Bring spilled keys back: merge every live spilled key into S, the
        // ones that do not fit go to the other spill buffer.
        auto refill = [&]() {
            __threadfence_block();   // spilled keys were stored by other lanes
            float thr = threshold(rfull, r, f);
            int n_old = spill_n;
            int sel_old = spill_sel;
            spill_sel ^= 1;
            spill_n = 0;
            spill_min = KEY_MAX;
            for (int c0 = 0; c0 < n_old; c0 += WAVE) {
                uint64_t v = KEY_MAX;
                if (c0 + lane < n_old) {
                    v = spill0[(size_t)sel_old * a.spill_cap + c0 + lane];
                    if (key_dist<INT>(v) > thr) v = KEY_MAX;   // dead
                }
                uint64_t m = ballot(v != KEY_MAX);
                int nb = __popcll(m);
                if (nb == 0) continue;
                v = wave_sort(v, WAVE);
                s_prune(thr);
                s_insert(v, nb);
            }
        };

        // ------------------------------------------------------ seeds ----
        {
            bool valid = false;
            uint32_t sid = 0;
            if (lane < a.n_seeds) {
                int32_t s = a.seeds[(size_t)qi * a.n_seeds + lane];
                valid = s >= 0 && (int64_t)s < a.n_base;
                sid = valid ? (uint32_t)s : 0u;
            }
            bool isnew = visit(valid, sid);
            uint64_t m = ballot(isnew);
            int u = __popcll(m);
            if (isnew) lds.ids[mbcnt(m)] = sid;
            wave_sync();
            batch_keys(u);
            dc += u;
            uint64_t key = lane < u ? kbuf[lane] : KEY_MAX;
            wave_sync();
            key = wave_sort(key, pow2_at_least(u));
            if (a.two_phase) lds.misc[lane] = lane < u ? key_dist<INT>(key) : 0.0f;
            if (a.two_phase && lane == 0) lds.misc[64] = (float)u;
            // every seed enters S (no range test) and is offered to R
            absorb(key, u, false);
        }

        // ------------------------------------------------- main loop -----
        for (;;) {
            if (head == size && spill_n == 0) break;                  // S empty
            if (dc >= max_dc) {                                       // budget spent
                flags |= ONNG_QF_BUDGET;
                break;
            }
            if (spill_n > 0 && (head == size || uni64(lds.S[head]) > spill_min)) {
                refill();
                if (head == size) break;
            }
            uint64_t sk = uni64(lds.S[head]);
            head++;
            float thr = threshold(rfull, r, f);
            if (key_dist<INT>(sk) > thr) break;                        // d(s,q) > r(1+eps)
            hops++;
            const uint32_t s = (uint32_t)sk;
            // adjacency of s: prefetched during the previous expansion when
            // that one guessed this pop, else read now
            const bool hit = s == spec_id;
            spec_id = NO_SPEC;
            int64_t e0, deg;
            if (hit) {
                e0 = spec_e0;
                deg = spec_deg;
            } else {
                e0 = a.offsets[s];
                deg = a.offsets[s + 1] - e0;
            }
            const int64_t np = (int64_t)ep < deg ? (int64_t)ep : deg;
            scanned += (int)np;
            // The edges in groups of up to two 64-edge chunks: ids and visited
            // marks of the group, then one distance batch for its new nodes.
            for (int64_t g0 = 0; g0 < np; g0 += 2 * WAVE) {
                int u = 0;
                const bool pre = hit && g0 == 0;
                if (pre && spec_vis) {
                    // both chunks read ahead, with their visited words
                    const bool v0 = lane < np && (int64_t)spec_nb < a.n_base;
                    const bool v1 = WAVE + lane < np && (int64_t)spec_nb1 < a.n_base;
                    bool k0 = false, k1 = false;
                    bool n0 = visit(v0, spec_nb, true, spec_bit, spec_wz, &k0);
                    bool n1 = false;
                    if (WAVE < np) n1 = visit(v1, spec_nb1, true, spec_bit1, spec_wz1, &k1);
                    dedupe_known(spec_nb, n0, k0, spec_nb1, n1, k1);
                    uint64_t m = ballot(n0);
                    if (n0) lds.ids[mbcnt(m)] = spec_nb;
                    u = __popcll(m);
                    m = ballot(n1);
                    if (n1) lds.ids[u + mbcnt(m)] = spec_nb1;
                    u += __popcll(m);
                } else {
#pragma unroll
                    for (int cc = 0; cc < 2; cc++) {
                        const int64_t c0 = g0 + cc * WAVE;
                        if (c0 >= np) break;
                        const int64_t j = c0 + lane;
                        uint32_t id;
                        if (pre) id = j < np ? (cc == 0 ? spec_nb : spec_nb1) : 0u;
                        else id = j < np ? (uint32_t)a.nbrs[e0 + j] : 0u;
                        bool valid = j < np && (int64_t)id < a.n_base;
                        bool isnew = visit(valid, id);
                        uint64_t m = ballot(isnew);
                        if (isnew) lds.ids[u + mbcnt(m)] = id;
                        u += __popcll(m);
                    }
                }
                if (u == 0) continue;
                wave_sync();
                batch_keys(u);
                dc += u;
                uint64_t k0 = lane < u ? kbuf[lane] : KEY_MAX;
                uint64_t k1 = lane + WAVE < u ? kbuf[lane + WAVE] : KEY_MAX;
                wave_sync();
                // Keys that can neither enter S (beyond the current range,
                // which only shrinks) nor the pool (beyond its last key when
                // full) are dropped before sorting.
                int nk;
                {
                    const float thr0 = threshold(rfull, r, f);
                    const uint64_t plast = npool == pool_q ? lds.pool[pool_q - 1] : KEY_MAX;
                    bool keep0 = lane < u && (key_dist<INT>(k0) <= thr0 || k0 < plast);
                    bool keep1 = lane + WAVE < u && (key_dist<INT>(k1) <= thr0 || k1 < plast);
                    uint64_t m0 = ballot(keep0), m1 = ballot(keep1);
                    const int n0 = __popcll(m0);
                    nk = n0 + __popcll(m1);
                    if (nk < u) {
                        if (keep0) kbuf[mbcnt(m0)] = k0;
                        if (keep1) kbuf[n0 + mbcnt(m1)] = k1;
                        wave_sync();
                        k0 = lane < nk ? kbuf[lane] : KEY_MAX;
                        k1 = lane + WAVE < nk ? kbuf[lane + WAVE] : KEY_MAX;
                        wave_sync();
                    }
                }
                const int na = min(nk, WAVE), nb2 = nk - na;
                // Guess the next pop (the smaller of S's head and this group's
                // minimum, when within range and no spilled key is smaller)
                // and start reading its adjacency (two chunks) and visited bits
                // while the batch is sorted and merged.  A wrong guess only
                // wastes the reads.
                bool go = false;
                int64_t spec_ofs = 0;
                if (g0 + 2 * WAVE >= np) {
                    uint64_t bmin = nk > 0 ? wave_min64(k0 < k1 ? k0 : k1) : KEY_MAX;
                    uint64_t smin = head < size ? lds.S[head] : KEY_MAX;
                    uint64_t cand = uni64(bmin < smin ? bmin : smin);
                    go = cand != KEY_MAX && !(spill_n > 0 && spill_min < cand) &&
                         key_dist<INT>(cand) <= threshold(rfull, r, f);
                    if (go) {
                        spec_id = (uint32_t)cand;
                        // lanes 0 and 1 read the two offsets with a vector load,
                        // which the sort's LDS traffic does not wait for
                        spec_ofs = a.offsets[spec_id + (lane & 1)];
                    }
                }
                if (na > 0) k0 = wave_sort(k0, pow2_at_least(na));
                // The guess's reads form a dependent chain (offsets, then
                // adjacency, then visited bits); each step is issued one
                // merge after the previous one so that its latency overlaps it.
                if (na > 0) absorb_pool(k0, na);
                int nl0 = 0, nl1 = 0;
                if (go) {
                    spec_e0 = readlane64(spec_ofs, 0);
                    spec_deg = readlane64(spec_ofs, 1) - spec_e0;
                    nl0 = (int)(spec_deg < WAVE ? spec_deg : WAVE);
                    nl1 = (int)(spec_deg < 2 * WAVE ? spec_deg - nl0 : WAVE);
                    spec_nb = lane < nl0 ? (uint32_t)a.nbrs[spec_e0 + lane] : 0u;
                    spec_nb1 = lane < nl1 ? (uint32_t)a.nbrs[spec_e0 + WAVE + lane] : 0u;
                }
                if (na > 0) absorb_s(k0, na, true);
                spec_vis = go;
                if (spec_vis) {
                    // the marks of this expansion are complete before the
                    // visited words of the guess are read (those outside the
                    // window: the others are on chip)
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                    uint32_t wd = 0u, wd1 = 0u;
                    if (lane < nl0 && (int64_t)spec_nb < a.n_base && spec_nb - w0 >= W)
                        wd = __hip_atomic_load(&gbits[spec_nb >> 5], __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
                    if (lane < nl1 && (int64_t)spec_nb1 < a.n_base && spec_nb1 - w0 >= W)
                        wd1 = __hip_atomic_load(&gbits[spec_nb1 >> 5], __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
                    spec_bit = (wd >> (spec_nb & 31)) & 1u;
                    spec_bit1 = (wd1 >> (spec_nb1 & 31)) & 1u;
                    spec_wz = wd == 0u;
                    spec_wz1 = wd1 == 0u;
                }
                if (nb2 > 0) {
                    k1 = wave_sort(k1, pow2_at_least(nb2));
                    absorb(k1, nb2, true);
                }
            }

            if (a.two_phase && hops == (int)a.probe_hops) {
                // ---- state after the probe expansions -> search range ----
                if (spill_n > 0) refill();   // the smallest keys of S on chip
                int nseed = (int)lds.misc[64];
                int ns = size - head + spill_n;
                int m = min(size - head, 64);
                float rmax = npool > 0 ? key_dist<INT>(lds.pool[min(npool, k) - 1]) : 0.0f;
                // lane t < 14 computes feature t
                float fv = 0.0f;
                if (lane < 8) fv = nseed == 0 ? 0.0f : lds.misc[lane < nseed ? lane : nseed - 1];
                else if (lane == 8) fv = (float)ns;
                else if (lane == 9) fv = m > 0 ? key_dist<INT>(lds.S[head]) : rmax;
                else if (lane == 10) fv = m > 0 ? key_dist<INT>(lds.S[head + (m + 1) / 2 - 1]) : rmax;
                else if (lane == 11) fv = m > 0 ? key_dist<INT>(lds.S[head + m - 1]) : rmax;
                else if (lane == 12) fv = rmax;
                else if (lane == 13) fv = (float)dc;
                if (a.feat_out && lane < ONNG_NFEAT) a.feat_out[(size_t)qi * ONNG_NFEAT + lane] = fv;
                if (a.has_pred) {
                    eps = predict_eps(a.pred, fv, MT, qi, lane, lds.misc + 72, &cost);
                    eps = unif(eps);
                    cost = unif(cost);
                    if (a.pred.mode == ONNG_PRED_CURVE) cost_budget(cost);
                    ep = a.pred.we >= 0.0f ? dynamic_ep(eps, a.pred.e0, a.pred.we)
                                           : (a.ep_pq ? uniu(a.ep_pq[qi]) : a.ep);
                } else {
                    eps = a.eps_pq ? unif(a.eps_pq[qi]) : a.eps;
                    ep = a.ep_pq ? uniu(a.ep_pq[qi]) : a.ep;
                }
                f = range_factor(eps, MT);
                s_prune(threshold(rfull, r, f));
                if (a.predict_only) break;   // the range is all this pass reports
            }
        }

        // ---------------------------------------------- rerank, output ---
        int nout = min(npool, k);
        if (a.predict_only) {
            // no result rows in a predict-only pass
        } else if (a.has_rr && npool > 0) {
            // exact f32 distances of the pool from the f32 rows
            for (int c0 = 0; c0 < npool; c0 += WAVE) {
                if (c0 + lane < npool) lds.ids[lane] = (uint32_t)lds.pool[c0 + lane];
                wave_sync();
                int u = min(WAVE, npool - c0);
                // 16 rows per pass, 4 lanes per row; a lane reads 16-byte
                // pieces pp, pp + 4, ... of its row, up to 8 at once, so that a
                // pass waits for memory once (rows of up to 128 components)
                const int pp = lane & 3;
                const int n4 = (a.dim + 3) >> 2;
                const float4 *qf4 = reinterpret_cast<const float4 *>(qrow);
                for (int r0 = 0; r0 < u; r0 += 16) {
                    const int row = r0 + (lane >> 2);
                    const bool rv = row < u;
                    const uint32_t id = rv ? lds.ids[row] : 0u;
                    const float4 *xr4 =
                        reinterpret_cast<const float4 *>(a.rr_base + (size_t)id * a.rr_pitch);
                    float acc = 0.0f;
                    for (int j0 = 0; j0 < n4; j0 += 32) {
                        float4 xv[8], qv[8];
#pragma unroll
                        for (int t = 0; t < 8; t++) {
                            const int c4 = j0 + pp + 4 * t;
                            const bool in = rv && c4 < n4;
                            xv[t] = in ? xr4[c4] : float4{0.0f, 0.0f, 0.0f, 0.0f};
                            qv[t] = in ? qf4[c4] : float4{0.0f, 0.0f, 0.0f, 0.0f};
                        }
#pragma unroll
                        for (int t = 0; t < 8; t++) {
                            const int c = 4 * (j0 + pp + 4 * t);
                            const float xs[4] = {xv[t].x, xv[t].y, xv[t].z, xv[t].w};
                            const float qs[4] = {qv[t].x, qv[t].y, qv[t].z, qv[t].w};
#pragma unroll
                            for (int e = 0; e < 4; e++) {
                                // components past dim (a row's padding) count as zero
                                const float xe = c + e < a.dim ? xs[e] : 0.0f;
                                const float qe = c + e < a.dim ? qs[e] : 0.0f;
                                if constexpr (MT == ONNG_L2SQ) {
                                    const float df = xe - qe;
                                    acc = fmaf(df, df, acc);
                                } else {
                                    acc = fmaf(xe, qe, acc);
                                }
                            }
                        }
                    }
                    acc += __shfl_xor(acc, 1);
                    acc += __shfl_xor(acc, 2);
                    if (rv && pp == 0) {
                        float d = MT == ONNG_COSINE ? 1.0f - acc : acc;
                        lds.stage2[row] = make_key(ord_f32(d), id);
                    }
                }
                wave_sync();
                uint64_t key = lane < u ? lds.stage2[lane] : KEY_MAX;
                wave_sync();
                key = wave_sort(key, pow2_at_least(u));
                // reuse S as the top-k accumulator of the reranked keys
                int cur = c0 == 0 ? 0 : min(c0, k);
                merge_sorted(lds.S, 0, cur, key, u, k, lds.stage, NoSpill());
            }
            nout = min(npool, k);
            for (int i = lane; i < a.k_stride; i += WAVE) {
                int32_t id = -1;
                float d = F_INF;
                if (i < nout) {
                    uint64_t key = lds.S[i];
                    id = (int32_t)(uint32_t)key;
                    d = unord_f32((uint32_t)(key >> 32));
                    if (a.id_map) id = a.id_map[id];
                }
                a.out_ids[(size_t)qi * a.k_stride + i] = id;
                reinterpret_cast<float *>(a.out_d)[(size_t)qi * a.k_stride + i] = d;
            }
        } else {
            for (int i = lane; i < a.k_stride; i += WAVE) {
                int32_t id = -1;
                uint64_t key = i < nout ? lds.pool[i] : KEY_MAX;
                if (i < nout) id = (int32_t)(uint32_t)key;
                if (i < nout && a.id_map) id = a.id_map[id];
                a.out_ids[(size_t)qi * a.k_stride + i] = id;
                if constexpr (INT) {
                    reinterpret_cast<int32_t *>(a.out_d)[(size_t)qi * a.k_stride + i] =
                        i < nout ? (int32_t)(key >> 32) : INT32_MAX;
                } else {
                    reinterpret_cast<float *>(a.out_d)[(size_t)qi * a.k_stride + i] =
                        i < nout ? unord_f32((uint32_t)(key >> 32)) : F_INF;
                }
            }
        }
        if (nout < k && !a.predict_only) flags |= ONNG_QF_PADDED;
        if (lane == 0) {
            onng_query_stats st;
            st.dc = dc;
            st.hops = hops;
            st.flags = flags;
            st.e_p = ep;
            st.eps = eps;
            st.scanned = scanned;
            st.cost = cost;
            st.us = (float)(wall_clock64() - t_start) * a.us_per_tick;
            a.stats[qi] = st;
        }

        // leave the global visited bitset clean for the next query
        if (log_n > 0) {
            __threadfence_block();   // the log was written by other lanes
            if (log_n <= a.vlog_cap) {
                // eight log entries per lane in flight, then their stores
                for (int i0 = 0; i0 < log_n; i0 += 8 * WAVE) {
                    int32_t wd[8];
#pragma unroll
                    for (int t = 0; t < 8; t++) {
                        const int i = i0 + t * WAVE + lane;
                        wd[t] = i < log_n ? vlog[i] : -1;
                    }
#pragma unroll
                    for (int t = 0; t < 8; t++)
                        if (wd[t] >= 0) gbits[(uint32_t)wd[t]] = 0u;
                }
            } else {
                u32x4 *g4 = reinterpret_cast<u32x4 *>(gbits);
                for (int64_t i = lane; i < a.gbits_words / 4; i += WAVE) g4[i] = u32x4{0, 0, 0, 0};
            }
            __threadfence_block();
        }
        wave_sync();
    }

    // The last wave of the launch records the layout whose bitsets are now
    // all zero.
    if (lane == 0) {
        __threadfence();
        const int total = (int)gridDim.x * a.waves_per_block;
        if (atomicAdd(a.counter + 1, 1) == total - 1)
            __hip_atomic_store(a.ws_tag_at, a.ws_tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Dispatch -----------------------------------------------------------------

#define ONNG_SEARCH_INST(DT, MT)                                                      \
    template __global__ void search_kernel<DT, MT>(SearchKArgs);

ONNG_SEARCH_INST(ONNG_U8, ONNG_L2SQ)
ONNG_SEARCH_INST(ONNG_F32, ONNG_L2SQ)
ONNG_SEARCH_INST(ONNG_F32, ONNG_COSINE)
ONNG_SEARCH_INST(ONNG_F16, ONNG_L2SQ)
ONNG_SEARCH_INST(ONNG_F16, ONNG_COSINE)
ONNG_SEARCH_INST(ONNG_BF16, ONNG_L2SQ)
ONNG_SEARCH_INST(ONNG_BF16, ONNG_COSINE)
ONNG_SEARCH_INST(ONNG_FP8_E4M3, ONNG_L2SQ)
ONNG_SEARCH_INST(ONNG_FP8_E4M3, ONNG_COSINE)

// work ticket (c[0]) and finished-wave count (c[1]) of a search launch
__global__ void reset_counter_kernel(int32_t *c) {
    c[0] = 0;
    c[1] = 0;
}

const void *search_kernel_ptr(int dtype, int metric) {
    switch (dtype) {
    case ONNG_U8: return metric == ONNG_L2SQ ? (const void *)search_kernel<ONNG_U8, ONNG_L2SQ> : nullptr;
    case ONNG_F32:
        return metric == ONNG_L2SQ ? (const void *)search_kernel<ONNG_F32, ONNG_L2SQ>
                                   : (const void *)search_kernel<ONNG_F32, ONNG_COSINE>;
    case ONNG_F16:
        return metric == ONNG_L2SQ ? (const void *)search_kernel<ONNG_F16, ONNG_L2SQ>
                                   : (const void *)search_kernel<ONNG_F16, ONNG_COSINE>;
    case ONNG_BF16:
        return metric == ONNG_L2SQ ? (const void *)search_kernel<ONNG_BF16, ONNG_L2SQ>
                                   : (const void *)search_kernel<ONNG_BF16, ONNG_COSINE>;
    case ONNG_FP8_E4M3:
        return metric == ONNG_L2SQ ? (const void *)search_kernel<ONNG_FP8_E4M3, ONNG_L2SQ>
                                   : (const void *)search_kernel<ONNG_FP8_E4M3, ONNG_COSINE>;
    }
    return nullptr;
}

// forget the workspace tag, so that the next launch zeroes the bitsets
__global__ void clear_tag_kernel(uint64_t *tag) { *tag = 0; }

const void *reset_counter_kernel_ptr() { return (const void *)reset_counter_kernel; }
const void *clear_tag_kernel_ptr() { return (const void *)clear_tag_kernel; }

}  // namespace onng
