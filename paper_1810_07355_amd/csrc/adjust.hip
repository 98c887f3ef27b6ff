// Graph adjustment on the GPU:
//   static degree adjustment, ConstructAdjustedGraph (Algorithm 2),
//   the same with constraints, ConstructAdjustedGraphWithConstraint
//   (Algorithm 3), and path adjustment, AdjustPath with HasPath (Algorithms 4 and 5).
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <type_traits>
#include <cstdint>
#include <vector>

#include "onng_internal.h"
#include "wave.h"

namespace onng {

namespace {

template <typename LenT>
__device__ __forceinline__ uint32_t len_ord(LenT v) {
    if constexpr (std::is_integral<LenT>::value) return (uint32_t)v;   // int32 lengths
    else return ord_f32((float)v);
}

// ------------------------------------------------------------ Algorithm 2 --
// Row o of the kNN table gives, in order, the edges S of Algorithm 2.  With the
// loop guard "p <= e_o or p <= e_i", step p of node o adds o -> n (p <= e_o) and
// n -> o (p <= e_i).  As sets: N(o) = F(o) u Rv(o), F(o) = first e_o of row o,
// Rv(o) = {m : o among the first e_i of row m}.  An edge present in both
// ways is inserted once, by whichever step comes first in the loop (node
// ascending, then p): the reverse copy when the far end has the smaller id,
// and it keeps that copy's length.

__device__ __forceinline__ int row_len(const int32_t *row, int k) {
    int l = 0;
    while (l < k && row[l] >= 0) l++;
    return l;
}

// position of `x` among the first `lim` ids of `row`, or -1
__device__ __forceinline__ int find_in(const int32_t *row, int lim, int32_t x) {
    for (int t = 0; t < lim; t++)
        if (row[t] == x) return t;
    return -1;
}

__global__ void sa_count_kernel(const int32_t *knn, int64_t n, int k, int eo, int ei,
                                int64_t *count) {
    int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    const int32_t *row = knn + m * k;
    int len = row_len(row, k);
    atomicAdd((unsigned long long *)&count[m], (unsigned long long)min(eo, len));
    int lim = min(ei, len);
    for (int t = 0; t < lim; t++) {
        int32_t o = row[t];
        if (o >= n) continue;
        const int32_t *orow = knn + (int64_t)o * k;
        int olen = row_len(orow, k);
        // reverse edge o -> m, unless m is already a forward edge of o
        if (find_in(orow, min(eo, olen), (int32_t)m) < 0)
            atomicAdd((unsigned long long *)&count[o], 1ull);
    }
}

template <typename LenT>
__global__ void sa_scatter_kernel(const int32_t *knn, const LenT *kd, int64_t n, int k, int eo,
                                  int ei, const int64_t *off, int32_t *cursor, uint64_t *keys) {
    int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    const int32_t *row = knn + m * k;
    int len = row_len(row, k);
    // forward edges of m
    int fwd = min(eo, len);
    for (int t = 0; t < fwd; t++) {
        int32_t nn = row[t];
        LenT l = kd[m * k + t];
        if (nn < m && nn < n) {
            // also a reverse edge inserted earlier (while processing nn)?
            const int32_t *nrow = knn + (int64_t)nn * k;
            int pos = find_in(nrow, min(ei, row_len(nrow, k)), (int32_t)m);
            if (pos >= 0) l = kd[(int64_t)nn * k + pos];
        }
        keys[off[m] + t] = make_key(len_ord(l), (uint32_t)nn);
    }
    // reverse edges o -> m
    int lim = min(ei, len);
    for (int t = 0; t < lim; t++) {
        int32_t o = row[t];
        if (o >= n) continue;
        const int32_t *orow = knn + (int64_t)o * k;
        int olen = row_len(orow, k);
        if (find_in(orow, min(eo, olen), (int32_t)m) >= 0) continue;   // forward edge of o
        int ofwd = min(eo, olen);
        int slot = atomicAdd(&cursor[o], 1);
        keys[off[o] + ofwd + slot] = make_key(len_ord(kd[m * k + t]), (uint32_t)m);
    }
}

// Sort each list by (length, id): rank of every key among the keys of its list.
template <typename LenT>
__global__ void __launch_bounds__(256) segment_rank_sort_kernel(const int64_t *off, int64_t n,
                                                                const uint64_t *keys,
                                                                int32_t *nbrs, LenT *lens) {
    extern __shared__ uint64_t sk[];
    int64_t v = blockIdx.x;
    if (v >= n) return;
    int64_t b = off[v], e = off[v + 1];
    int m = (int)(e - b);
    const int cap = 4096;
    const uint64_t *src = keys + b;
    if (m <= cap) {
        for (int i = threadIdx.x; i < m; i += blockDim.x) sk[i] = src[i];
        __syncthreads();
        src = sk;
    }
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
        uint64_t x = src[i];
        int rank = 0;
        for (int j = 0; j < m; j++) rank += src[j] < x;
        nbrs[b + rank] = (int32_t)(uint32_t)x;
        uint32_t lo = (uint32_t)(x >> 32);
        if constexpr (std::is_integral<LenT>::value) lens[b + rank] = (LenT)lo;
        else lens[b + rank] = unord_f32(lo);
    }
}

// ------------------------------------------------------------ Algorithm 3 --
// G_t = ConstructAdjustedGraph(G, 0, e_i): N(G_t, o) = {m : o among the first
// e_i of row m}, each edge with row m's length.  The first loop's in-degree
// bound never binds: only the (at most e_i) nodes of row n's head can add an
// edge into n, each of them considers n once, so whenever one does, fewer
// than e_i have added it before.  What remains decides every edge on its own:
// the first of row n's head in processing order (ascending (|N(G_t, x)|, x))
// meets n with in-degree 0 and adds it; any later one adds it only while its
// own out-degree is below e_o, i.e. for the first e_o members of N(G_t, o) in
// (length, id) order, all of which the loop keeps.  So o -> n is kept iff n is
// among those first e_o or o is n's first source.  The fill loop matters only
// for nodes with |N(G_t, o)| < e_o, whose first loop kept all of N(G_t, o): it
// appends the members of row o not already present, nearest first, up to e_o.

__global__ void sac_rcount_kernel(const int32_t *knn, int64_t n, int k, int ei, int64_t *cnt) {
    int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    const int32_t *row = knn + m * k;
    int lim = min(ei, row_len(row, k));
    for (int t = 0; t < lim; t++) {
        int32_t o = row[t];
        if (o < n) atomicAdd((unsigned long long *)&cnt[o], 1ull);
    }
}

// reverse keys of G_t into each node's segment, and every node's first source
template <typename LenT>
__global__ void sac_scatter_kernel(const int32_t *knn, const LenT *kd, int64_t n, int k, int ei,
                                   const int64_t *rev_off, int32_t *cursor, uint64_t *keys,
                                   int32_t *first_src) {
    int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n) return;
    const int32_t *row = knn + m * k;
    int lim = min(ei, row_len(row, k));
    int32_t best = -1;
    int64_t bestc = 0;
    for (int t = 0; t < lim; t++) {
        int32_t o = row[t];
        if (o >= n) continue;
        int slot = atomicAdd(&cursor[o], 1);
        keys[rev_off[o] + slot] = make_key(len_ord(kd[m * k + t]), (uint32_t)m);
        int64_t c = rev_off[o + 1] - rev_off[o];
        if (best < 0 || c < bestc || (c == bestc && o < best)) {
            best = o;
            bestc = c;
        }
    }
    first_src[m] = best;
}

// One wave per node o over its sorted N(G_t, o) (rv_nb/rv_len at rev_off):
// counts the kept edges (WRITE false) or writes their keys at out_off[o].
template <typename LenT, bool WRITE>
__global__ void __launch_bounds__(256) sac_select_kernel(
    const int64_t *rev_off, const int32_t *rv_nb, const LenT *rv_len, const int32_t *first_src,
    const int32_t *knn, const LenT *kd, int64_t n, int k, int eo, int64_t *out_cnt,
    const int64_t *out_off, uint64_t *keys) {
    const int64_t o = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const int lane = lane_id();
    if (o >= n) return;
    const int64_t b = rev_off[o];
    const int m = (int)(rev_off[o + 1] - b);
    const int head = min(m, eo);
    const int64_t w = WRITE ? out_off[o] : 0;
    if (WRITE)
        for (int p = lane; p < head; p += WAVE)
            keys[w + p] = make_key(len_ord(rv_len[b + p]), (uint32_t)rv_nb[b + p]);
    int c = head;
    for (int p0 = head; p0 < m; p0 += WAVE) {
        const int p = p0 + lane;
        const bool keep = p < m && first_src[rv_nb[b + p]] == (int32_t)o;
        const uint64_t bal = ballot(keep);
        if (WRITE && keep)
            keys[w + c + mbcnt(bal)] = make_key(len_ord(rv_len[b + p]), (uint32_t)rv_nb[b + p]);
        c += __popcll(bal);
    }
    if (m < eo) {
        const int32_t *row = knn + o * k;
        const LenT *rd = kd + o * k;
        for (int t0 = 0; t0 < k && c < eo; t0 += WAVE) {
            const int t = t0 + lane;
            const int32_t id = t < k ? row[t] : -1;
            bool add = id >= 0;
            for (int p = 0; add && p < m; p++) add = rv_nb[b + p] != id;
            const uint64_t bal = ballot(add);
            const int r = c + mbcnt(bal);
            if (WRITE && add && r < eo) keys[w + r] = make_key(len_ord(rd[t]), (uint32_t)id);
            c = min(eo, c + __popcll(bal));
        }
    }
    if (!WRITE && lane == 0) out_cnt[o] = c;
}

// --------------------------------------------------------- Algorithms 4/5 --
// Round j visits every node with more than j edges.  Node n's j-th edge
// n -> nd (length L) is removed when HasPath finds c in N(G_p, n) with
// nd in N(G_p, c) and len(c, nd) < L.  In Algorithm 4 nodes are visited in
// ascending id and G_p changes immediately, so G_p at n's turn is the graph
// at the start of round j plus the round-j edges kept by nodes c < n.  The
// GPU evaluates the start-of-round graph for all nodes at once (Jacobi
// kernel), then settles the remaining dependence — a node c < n in
// N(G_p, n) whose own round-j edge also goes to nd, is shorter than L and was
// kept — by repeated passes in which a node is decided as soon as all such
// c are (the smallest undecided node always is).

constexpr int8_t ST_UNDECIDED = 0, ST_KEPT = 1, ST_REMOVED = 2;

// Witness test of the start-of-round graph: c in N(G_p, n) is a witness
// when c's edge to nd exists, was kept in an earlier round (its rank in c's
// list is below j) and is shorter than L.  The edge is found by binary
// search in c's edges sorted by id (sid_nb, with their edge index sid_e),
// instead of scanning c's kept edges by length.
template <typename LenT>
__global__ void pa_jacobi_kernel(const int64_t *off, const int32_t *nbrs, const LenT *lens,
                                 const int32_t *active, int64_t n_active, int j,
                                 const int32_t *gp_nb, const int32_t *gp_cnt,
                                 const int32_t *sid_nb, const int32_t *sid_e, const int8_t *kept,
                                 int8_t *status) {
    int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    int lane = lane_id();
    if (w >= n_active) return;
    int32_t v = active[w];
    int64_t e = off[v] + j;
    int32_t nd = nbrs[e];
    LenT L = lens[e];
    int cn = gp_cnt[v];
    bool found = false;
    for (int c0 = 0; c0 < cn && !found; c0 += WAVE) {
        bool hit = false;
        if (c0 + lane < cn) {
            const int32_t c = gp_nb[off[v] + c0 + lane];
            const int64_t cb = off[c], ce = off[c + 1];
            int64_t lo = cb, hi = ce;
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if (sid_nb[mid] < nd) lo = mid + 1;
                else hi = mid;
            }
            // (a list may hold nd more than once: every copy is a candidate)
            for (; lo < ce && sid_nb[lo] == nd && !hit; lo++) {
                const int64_t ec = sid_e[lo];
                hit = ec - cb < j && kept[ec] && lens[ec] < L;
            }
        }
        found = ballot(hit) != 0;
    }
    if (lane == 0) status[v] = found ? ST_REMOVED : ST_UNDECIDED;
}

// edge index of every edge (the values sorted along with the ids)
__global__ void iota_kernel(int64_t n, int32_t *out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (int32_t)i;
}

template <typename LenT>
__global__ void pa_settle_kernel(const int64_t *off, const int32_t *nbrs, const LenT *lens,
                                 const int32_t *active, int64_t n_active, int j,
                                 const int32_t *gp_nb, const int32_t *gp_cnt, int8_t *status,
                                 int32_t *undecided) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_active) return;
    int32_t v = active[i];
    if (status[v] != ST_UNDECIDED) return;
    int64_t e = off[v] + j;
    int32_t nd = nbrs[e];
    LenT L = lens[e];
    int cn = gp_cnt[v];
    bool kept_witness = false, pending = false;
    for (int t = 0; t < cn; t++) {
        int32_t c = gp_nb[off[v] + t];
        if (c >= v) continue;
        int64_t cdeg = off[c + 1] - off[c];
        if (cdeg <= j) continue;
        int64_t ce = off[c] + j;
        if (nbrs[ce] != nd || !(lens[ce] < L)) continue;
        int8_t sc = __atomic_load_n(&status[c], __ATOMIC_RELAXED);
        if (sc == ST_KEPT) { kept_witness = true; break; }
        if (sc == ST_UNDECIDED) pending = true;
    }
    if (kept_witness) status[v] = ST_REMOVED;
    else if (!pending) status[v] = ST_KEPT;
    else atomicAdd(undecided, 1);
}

template <typename LenT>
__global__ void pa_apply_kernel(const int64_t *off, const int32_t *nbrs, const LenT *lens,
                                const int32_t *active, int64_t n_active, int j,
                                int32_t *gp_nb, LenT *gp_len, int32_t *gp_cnt,
                                const int8_t *status, int8_t *kept) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_active) return;
    int32_t v = active[i];
    if (status[v] != ST_KEPT) return;
    int64_t e = off[v] + j;
    kept[e] = 1;
    int c = gp_cnt[v];
    gp_nb[off[v] + c] = nbrs[e];
    gp_len[off[v] + c] = lens[e];
    gp_cnt[v] = c + 1;
}

__global__ void degree_hist_kernel(const int64_t *off, int64_t n, int32_t *deg,
                                   unsigned long long *hist) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    int64_t d64 = off[v + 1] - off[v];
    int d = d64 < (1 << 20) - 1 ? (int)d64 : (1 << 20) - 1;   // last bin flags overflow
    deg[v] = d;
    atomicAdd(&hist[d], 1ull);
}

// nodes by degree, descending: position = (#nodes with larger degree) + slot
__global__ void order_by_degree_kernel(const int32_t *deg, int64_t n, const int64_t *start,
                                       int32_t *cursor, int32_t *order) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    int d = deg[v];
    int slot = atomicAdd(&cursor[d], 1);
    order[start[d] + slot] = (int32_t)v;
}

template <typename LenT>
__global__ void pa_compact_kernel(const int64_t *off, const int64_t *out_off, int64_t n,
                                  const int32_t *gp_nb, const LenT *gp_len,
                                  int32_t *out_nb, LenT *out_len) {
    int64_t v = blockIdx.x;
    if (v >= n) return;
    int64_t b = off[v], ob = out_off[v], m = out_off[v + 1] - ob;
    for (int64_t t = threadIdx.x; t < m; t += blockDim.x) {
        out_nb[ob + t] = gp_nb[b + t];
        out_len[ob + t] = gp_len[b + t];
    }
}

__global__ void cnt_to_i64_kernel(const int32_t *c, int64_t n, int64_t *o) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) o[v] = c[v];
    if (v == n) o[n] = 0;
}

inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

size_t segsort_temp_bytes(int64_t nnz, int64_t n) {
    size_t bytes = 0;
    (void)hipcub::DeviceSegmentedRadixSort::SortPairs(
        nullptr, bytes, (const int32_t *)nullptr, (int32_t *)nullptr, (const int32_t *)nullptr,
        (int32_t *)nullptr, (int)nnz, (int)n, (const int64_t *)nullptr, (const int64_t *)nullptr);
    return bytes;
}

size_t scan_temp_bytes(int64_t n) {
    size_t bytes = 0;
    (void)hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, (int64_t *)nullptr, (int64_t *)nullptr,
                                     (int)n);
    return bytes;
}

// ------------------------------------------------------ graph statistics --
// Degree shape and incoming-edge lengths of a graph (Table 4).

__global__ void gs_degree_kernel(const int64_t *off, const int32_t *nbrs, int64_t n,
                                 int32_t *outdeg, int32_t *indeg) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    outdeg[v] = (int32_t)(off[v + 1] - off[v]);
    for (int64_t e = off[v]; e < off[v + 1]; e++) {
        const int32_t t = nbrs[e];
        if (t >= 0 && t < n) atomicAdd(&indeg[t], 1);   // ids outside the graph count nowhere
    }
}

// every edge's length key into its target's segment of the transposed graph
template <typename LenT>
__global__ void gs_transpose_kernel(const int64_t *off, const int32_t *nbrs, const LenT *lens,
                                    int64_t n, const int64_t *toff, int32_t *cursor,
                                    uint32_t *tkeys) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    for (int64_t e = off[v]; e < off[v + 1]; e++) {
        const int32_t t = nbrs[e];
        if (t < 0 || t >= n) continue;
        const int slot = atomicAdd(&cursor[t], 1);
        tkeys[toff[t] + slot] = len_ord(lens[e]);
    }
}

// per node: the sum of its `keep` shortest incoming lengths, as distances
template <typename LenT, bool SQRT>
__global__ void gs_keep_kernel(const int64_t *toff, const uint32_t *sorted, int64_t n, int keep,
                               double *psum, double *pcnt) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    int64_t b = toff[v];
    int c = (int)min<int64_t>(keep, toff[v + 1] - b);
    double s = 0.0;
    for (int i = 0; i < c; i++) {
        uint32_t key = sorted[b + i];
        double x;
        if constexpr (std::is_integral<LenT>::value) x = (double)key;
        else x = (double)unord_f32(key);
        s += SQRT ? sqrt(x) : x;
    }
    psum[v] = s;
    pcnt[v] = (double)c;
}

// one block: out[slot] = sum of a[0 .. cnt) in double, in a fixed order
template <typename T>
__global__ void __launch_bounds__(1024) gs_sum_kernel(const T *a, int64_t cnt, double *out,
                                                      int slot) {
    __shared__ double part[1024];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < cnt; i += blockDim.x) s += (double)a[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[slot] = part[0];
}

__global__ void gs_final_kernel(const double *sums, double t, double *res) {
    res[0] = t > 0 ? sums[0] / t : 0.0;
    res[1] = t > 0 ? sums[1] / t : 0.0;
    res[2] = sums[3] > 0 ? sums[2] / sums[3] : 0.0;
}

// ------------------------------------------------------- edge insertion --
// Graph plus new edges (src, dst, length): per-node counts, offsets, keys of
// the old and new edges in each node's segment, then the (length, id) sort.

__global__ void ae_count_kernel(const int64_t *off, int64_t n, const int32_t *src,
                                const int32_t *dst, int64_t m, int64_t *cnt) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) atomicAdd((unsigned long long *)&cnt[i], (unsigned long long)(off[i + 1] - off[i]));
    if (i < m && src[i] >= 0 && src[i] < n && dst[i] >= 0 && dst[i] < n)
        atomicAdd((unsigned long long *)&cnt[src[i]], 1ull);
}

template <typename LenT>
__global__ void ae_scatter_kernel(const int64_t *off, const int32_t *nbrs, const LenT *lens,
                                  int64_t n, const int32_t *src, const int32_t *dst,
                                  const LenT *len, int64_t m, const int64_t *out_off,
                                  int32_t *cursor, uint64_t *keys) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const int64_t b = off[i], e = off[i + 1];
        const int64_t w = out_off[i];
        for (int64_t t = b; t < e; t++) keys[w + (t - b)] = make_key(len_ord(lens[t]), (uint32_t)nbrs[t]);
        cursor[i] = (int32_t)(e - b);
    }
}

template <typename LenT>
__global__ void ae_new_kernel(int64_t n, const int32_t *src, const int32_t *dst, const LenT *len,
                              int64_t m, const int64_t *out_off, int32_t *cursor, uint64_t *keys) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const int32_t s = src[i], d = dst[i];
    if (s < 0 || s >= n || d < 0 || d >= n) return;
    const int slot = atomicAdd(&cursor[s], 1);
    keys[out_off[s] + slot] = make_key(len_ord(len[i]), (uint32_t)d);
}

}  // namespace

// ------------------------------------------------------------- host side --

size_t adjust_degree_ws(int64_t n, int32_t k, int32_t e_o, int32_t e_i) {
    int64_t cap = n * (int64_t)(std::min(e_o, k) + std::min(e_i, k));
    Carver c(nullptr);
    c.take<int64_t>(n + 1);            // counts / offsets
    c.take<int32_t>(n);                // cursors
    c.take<uint64_t>(cap);             // keys
    c.take<char>(scan_temp_bytes(n + 1));
    return c.size() + 256;
}

template <typename LenT>
static onng_status adjust_degree_impl(const int32_t *knn, const LenT *kd, int64_t n, int32_t k,
                                      int32_t e_o, int32_t e_i, int64_t *offsets, int32_t *nbrs,
                                      LenT *lens, int64_t nnz_cap, int64_t *nnz_out, void *ws,
                                      hipStream_t st) {
    int eo = std::min(e_o, k), ei = std::min(e_i, k);
    int64_t cap = n * (int64_t)(eo + ei);
    Carver c(ws);
    int64_t *cnt = c.take<int64_t>(n + 1);
    int32_t *cursor = c.take<int32_t>(n);
    uint64_t *keys = c.take<uint64_t>(cap);
    size_t tb = scan_temp_bytes(n + 1);
    void *tmp = c.take<char>(tb);
    ONNG_HIP(hipMemsetAsync(cnt, 0, sizeof(int64_t) * (n + 1), st));
    ONNG_HIP(hipMemsetAsync(cursor, 0, sizeof(int32_t) * n, st));
    hipLaunchKernelGGL(sa_count_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, knn, n, k, eo,
                       ei, cnt);
    ONNG_HIP(hipcub::DeviceScan::ExclusiveSum(tmp, tb, cnt, offsets, (int)(n + 1), st));
    ONNG_HIP(hipMemcpyAsync(nnz_out, offsets + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    ONNG_HIP(hipStreamSynchronize(st));
    if (*nnz_out > nnz_cap) {
        set_error("onng_adjust_degree: nnz_capacity too small");
        return ONNG_ERR_CAPACITY;
    }
    hipLaunchKernelGGL((sa_scatter_kernel<LenT>), dim3(blocks_for(n, 256)), dim3(256), 0, st, knn,
                       kd, n, k, eo, ei, offsets, cursor, keys);
    if (n > 0)
        hipLaunchKernelGGL((segment_rank_sort_kernel<LenT>), dim3((unsigned)n), dim3(256),
                           4096 * sizeof(uint64_t), st, offsets, n, keys, nbrs, lens);
    ONNG_HIP(hipGetLastError());
    ONNG_HIP(hipStreamSynchronize(st));
    return ONNG_OK;
}

onng_status adjust_degree_launch(const int32_t *knn, const void *kd, int64_t n, int32_t k,
                                 bool int_len, int32_t e_o, int32_t e_i, int64_t *offsets,
                                 int32_t *nbrs, void *lens, int64_t nnz_cap, int64_t *nnz_out,
                                 void *ws, hipStream_t st) {
    if (int_len)
        return adjust_degree_impl<int32_t>(knn, static_cast<const int32_t *>(kd), n, k, e_o, e_i,
                                           offsets, nbrs, static_cast<int32_t *>(lens), nnz_cap,
                                           nnz_out, ws, st);
    return adjust_degree_impl<float>(knn, static_cast<const float *>(kd), n, k, e_o, e_i, offsets,
                                     nbrs, static_cast<float *>(lens), nnz_cap, nnz_out, ws, st);
}

size_t adjust_degree_constrained_ws(int64_t n, int32_t k, int32_t e_o, int32_t e_i) {
    const int64_t nrev = n * (int64_t)std::min(e_i, k);
    const int64_t cap = nrev + n * (int64_t)std::min(e_o, k);
    Carver c(nullptr);
    c.take<int64_t>(n + 1);            // |N(G_t, o)|
    c.take<int64_t>(n + 1);            // G_t offsets
    c.take<int32_t>(n);                // cursors
    c.take<int32_t>(n);                // first source per node
    c.take<uint64_t>(nrev);            // G_t keys
    c.take<int32_t>(nrev);             // G_t ids, sorted per node
    c.take<int32_t>(nrev);             // G_t lengths (4 bytes)
    c.take<int64_t>(n + 1);            // kept counts
    c.take<uint64_t>(cap);             // kept keys
    c.take<char>(scan_temp_bytes(n + 1));
    return c.size() + 256;
}

template <typename LenT>
static onng_status adjust_degree_constrained_impl(const int32_t *knn, const LenT *kd, int64_t n,
                                                  int32_t k, int32_t e_o, int32_t e_i,
                                                  int64_t *offsets, int32_t *nbrs, LenT *lens,
                                                  int64_t nnz_cap, int64_t *nnz_out, void *ws,
                                                  hipStream_t st) {
    const int ei = std::min(e_i, k);
    const int eo = e_o;
    const int64_t nrev = n * (int64_t)ei;
    const int64_t cap = nrev + n * (int64_t)std::min(e_o, k);
    Carver c(ws);
    int64_t *cnt = c.take<int64_t>(n + 1);
    int64_t *rev_off = c.take<int64_t>(n + 1);
    int32_t *cursor = c.take<int32_t>(n);
    int32_t *first_src = c.take<int32_t>(n);
    uint64_t *rkeys = c.take<uint64_t>(nrev);
    int32_t *rv_nb = c.take<int32_t>(nrev);
    LenT *rv_len = reinterpret_cast<LenT *>(c.take<int32_t>(nrev));
    int64_t *ocnt = c.take<int64_t>(n + 1);
    uint64_t *okeys = c.take<uint64_t>(cap);
    size_t tb = scan_temp_bytes(n + 1);
    void *tmp = c.take<char>(tb);
    ONNG_HIP(hipMemsetAsync(cnt, 0, sizeof(int64_t) * (n + 1), st));
    ONNG_HIP(hipMemsetAsync(ocnt, 0, sizeof(int64_t) * (n + 1), st));
    ONNG_HIP(hipMemsetAsync(cursor, 0, sizeof(int32_t) * n, st));
    if (n > 0) {
        hipLaunchKernelGGL(sac_rcount_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, knn, n,
                           k, ei, cnt);
        ONNG_HIP(hipcub::DeviceScan::ExclusiveSum(tmp, tb, cnt, rev_off, (int)(n + 1), st));
        hipLaunchKernelGGL((sac_scatter_kernel<LenT>), dim3(blocks_for(n, 256)), dim3(256), 0, st,
                           knn, kd, n, k, ei, rev_off, cursor, rkeys, first_src);
        hipLaunchKernelGGL((segment_rank_sort_kernel<LenT>), dim3((unsigned)n), dim3(256),
                           4096 * sizeof(uint64_t), st, rev_off, n, rkeys, rv_nb, rv_len);
        hipLaunchKernelGGL((sac_select_kernel<LenT, false>), dim3(blocks_for(n * WAVE, 256)),
                           dim3(256), 0, st, rev_off, rv_nb, rv_len, first_src, knn, kd, n, k, eo,
                           ocnt, nullptr, nullptr);
        ONNG_HIP(hipGetLastError());
    }
    ONNG_HIP(hipcub::DeviceScan::ExclusiveSum(tmp, tb, ocnt, offsets, (int)(n + 1), st));
    ONNG_HIP(hipMemcpyAsync(nnz_out, offsets + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    ONNG_HIP(hipStreamSynchronize(st));
    if (*nnz_out > nnz_cap) {
        set_error("onng_adjust_degree_constrained: nnz_capacity too small");
        return ONNG_ERR_CAPACITY;
    }
    if (*nnz_out > cap) {
        set_error("onng_adjust_degree_constrained: more edges than the workspace bound");
        return ONNG_ERR_CAPACITY;
    }
    if (n > 0) {
        hipLaunchKernelGGL((sac_select_kernel<LenT, true>), dim3(blocks_for(n * WAVE, 256)),
                           dim3(256), 0, st, rev_off, rv_nb, rv_len, first_src, knn, kd, n, k, eo,
                           nullptr, offsets, okeys);
        hipLaunchKernelGGL((segment_rank_sort_kernel<LenT>), dim3((unsigned)n), dim3(256),
                           4096 * sizeof(uint64_t), st, offsets, n, okeys, nbrs, lens);
    }
    ONNG_HIP(hipGetLastError());
    ONNG_HIP(hipStreamSynchronize(st));
    return ONNG_OK;
}

onng_status adjust_degree_constrained_launch(const int32_t *knn, const void *kd, int64_t n,
                                             int32_t k, bool int_len, int32_t e_o, int32_t e_i,
                                             int64_t *offsets, int32_t *nbrs, void *lens,
                                             int64_t nnz_cap, int64_t *nnz_out, void *ws,
                                             hipStream_t st) {
    if (int_len)
        return adjust_degree_constrained_impl<int32_t>(
            knn, static_cast<const int32_t *>(kd), n, k, e_o, e_i, offsets, nbrs,
            static_cast<int32_t *>(lens), nnz_cap, nnz_out, ws, st);
    return adjust_degree_constrained_impl<float>(knn, static_cast<const float *>(kd), n, k, e_o,
                                                 e_i, offsets, nbrs, static_cast<float *>(lens),
                                                 nnz_cap, nnz_out, ws, st);
}

static size_t gs_sort_temp_bytes(int64_t n, int64_t nnz) {
    size_t a = 0, b = 0, d = 0;
    (void)hipcub::DeviceRadixSort::SortKeys(nullptr, a, (const int32_t *)nullptr,
                                            (int32_t *)nullptr, (int)n);
    (void)hipcub::DeviceRadixSort::SortKeysDescending(nullptr, d, (const int32_t *)nullptr,
                                                      (int32_t *)nullptr, (int)n);
    a = std::max(a, d);
    (void)hipcub::DeviceSegmentedRadixSort::SortKeys(
        nullptr, b, (const uint32_t *)nullptr, (uint32_t *)nullptr, (int)nnz, (int)n,
        (const int64_t *)nullptr, (const int64_t *)nullptr);
    return std::max(std::max(a, b), scan_temp_bytes(n + 1));
}

size_t graph_stats_ws(int64_t n, int64_t nnz) {
    Carver c(nullptr);
    c.take<int32_t>(n);          // out-degrees
    c.take<int32_t>(n);          // in-degrees
    c.take<int32_t>(n);          // sorted degrees
    c.take<int32_t>(n);          // cursors
    c.take<int64_t>(n + 1);      // in-degrees as int64
    c.take<int64_t>(n + 1);      // transposed offsets
    c.take<uint32_t>(nnz);       // incoming length keys
    c.take<uint32_t>(nnz);       // the same, sorted per node
    c.take<double>(n);           // per-node sums
    c.take<double>(n);           // per-node counts
    c.take<double>(8);           // sums and results
    c.take<char>(gs_sort_temp_bytes(n, nnz));
    return c.size() + 256;
}

template <typename LenT>
static onng_status graph_stats_impl(const onng_graph *g, bool sqrt_len, double frac, int keep,
                                    double *out, void *ws, hipStream_t st) {
    const int64_t n = g->n, nnz = g->nnz;
    Carver c(ws);
    int32_t *outdeg = c.take<int32_t>(n);
    int32_t *indeg = c.take<int32_t>(n);
    int32_t *sdeg = c.take<int32_t>(n);
    int32_t *cursor = c.take<int32_t>(n);
    int64_t *in64 = c.take<int64_t>(n + 1);
    int64_t *toff = c.take<int64_t>(n + 1);
    uint32_t *tkeys = c.take<uint32_t>(nnz);
    uint32_t *tsorted = c.take<uint32_t>(nnz);
    double *psum = c.take<double>(n);
    double *pcnt = c.take<double>(n);
    double *sums = c.take<double>(8);
    size_t tb = gs_sort_temp_bytes(n, nnz);
    void *tmp = c.take<char>(tb);
    const int64_t t = n > 0 ? std::max<int64_t>(1, (int64_t)std::floor(frac * (double)n)) : 0;
    ONNG_HIP(hipMemsetAsync(indeg, 0, sizeof(int32_t) * n, st));
    ONNG_HIP(hipMemsetAsync(cursor, 0, sizeof(int32_t) * n, st));
    ONNG_HIP(hipMemsetAsync(sums, 0, sizeof(double) * 8, st));
    if (n > 0) {
        const unsigned nb = blocks_for(n, 256);
        hipLaunchKernelGGL(gs_degree_kernel, dim3(nb), dim3(256), 0, st, g->offsets, g->nbrs, n,
                           outdeg, indeg);
        size_t b = tb;
        ONNG_HIP(hipcub::DeviceRadixSort::SortKeysDescending(tmp, b, outdeg, sdeg, (int)n, 0, 32,
                                                             st));
        hipLaunchKernelGGL((gs_sum_kernel<int32_t>), dim3(1), dim3(1024), 0, st, sdeg, t, sums, 0);
        b = tb;
        ONNG_HIP(hipcub::DeviceRadixSort::SortKeys(tmp, b, indeg, sdeg, (int)n, 0, 32, st));
        hipLaunchKernelGGL((gs_sum_kernel<int32_t>), dim3(1), dim3(1024), 0, st, sdeg, t, sums, 1);
        hipLaunchKernelGGL(cnt_to_i64_kernel, dim3(blocks_for(n + 1, 256)), dim3(256), 0, st,
                           indeg, n, in64);
        b = tb;
        ONNG_HIP(hipcub::DeviceScan::ExclusiveSum(tmp, b, in64, toff, (int)(n + 1), st));
        hipLaunchKernelGGL((gs_transpose_kernel<LenT>), dim3(nb), dim3(256), 0, st, g->offsets,
                           g->nbrs, static_cast<const LenT *>(g->lens), n, toff, cursor, tkeys);
        if (nnz > 0) {
            b = tb;
            ONNG_HIP(hipcub::DeviceSegmentedRadixSort::SortKeys(
                tmp, b, tkeys, tsorted, (int)nnz, (int)n, toff, toff + 1, 0, 32, st));
        }
        if (sqrt_len)
            hipLaunchKernelGGL((gs_keep_kernel<LenT, true>), dim3(nb), dim3(256), 0, st, toff,
                               tsorted, n, keep, psum, pcnt);
        else
            hipLaunchKernelGGL((gs_keep_kernel<LenT, false>), dim3(nb), dim3(256), 0, st, toff,
                               tsorted, n, keep, psum, pcnt);
        hipLaunchKernelGGL((gs_sum_kernel<double>), dim3(1), dim3(1024), 0, st, psum, n, sums, 2);
        hipLaunchKernelGGL((gs_sum_kernel<double>), dim3(1), dim3(1024), 0, st, pcnt, n, sums, 3);
    }
    hipLaunchKernelGGL(gs_final_kernel, dim3(1), dim3(1), 0, st, sums, (double)t, sums + 4);
    ONNG_HIP(hipGetLastError());
    ONNG_HIP(hipMemcpyAsync(out, sums + 4, 3 * sizeof(double), hipMemcpyDeviceToHost, st));
    ONNG_HIP(hipStreamSynchronize(st));
    return ONNG_OK;
}

onng_status graph_stats_launch(const onng_graph *g, bool int_len, bool sqrt_len, double frac,
                               int keep, double *out, void *ws, hipStream_t st) {
    if (int_len) return graph_stats_impl<int32_t>(g, sqrt_len, frac, keep, out, ws, st);
    return graph_stats_impl<float>(g, sqrt_len, frac, keep, out, ws, st);
}

// ---------------------------------------------- first k edges of a graph --

namespace {

// Row v of the table: the first min(k, deg(v)) edges of v's list (sorted by
// (length, id)), then padding (-1, INT32_MAX or +inf).  One lane per entry.
template <typename LT>
__global__ void graph_head_kernel(const int64_t *off, const int32_t *nb, const LT *len, int64_t n,
                                  int32_t k, LT pad, int32_t *ids, LT *dists) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * (int64_t)k) return;
    const int64_t v = t / k;
    const int32_t j = (int32_t)(t - v * k);
    const int64_t e = off[v] + j;
    const bool has = e < off[v + 1];
    ids[t] = has ? nb[e] : -1;
    dists[t] = has ? len[e] : pad;
}

}  // namespace

onng_status graph_head_launch(const onng_graph *g, bool int_len, int32_t k, int32_t *ids,
                              void *dists, hipStream_t st) {
    const int64_t total = g->n * (int64_t)k;
    if (total == 0) return ONNG_OK;
    const unsigned blocks = (unsigned)((total + 255) / 256);
    if (int_len)
        hipLaunchKernelGGL(graph_head_kernel<int32_t>, dim3(blocks), dim3(256), 0, st, g->offsets,
                           g->nbrs, static_cast<const int32_t *>(g->lens), g->n, k, INT32_MAX, ids,
                           static_cast<int32_t *>(dists));
    else
        hipLaunchKernelGGL(graph_head_kernel<float>, dim3(blocks), dim3(256), 0, st, g->offsets,
                           g->nbrs, static_cast<const float *>(g->lens), g->n, k,
                           __builtin_huge_valf(), ids, static_cast<float *>(dists));
    ONNG_HIP(hipGetLastError());
    return ONNG_OK;
}

size_t add_edges_ws(int64_t n, int64_t nnz, int64_t m) {
    Carver c(nullptr);
    c.take<int64_t>(n + 1);
    c.take<int32_t>(n);
    c.take<uint64_t>(nnz + m);
    c.take<char>(scan_temp_bytes(n + 1));
    return c.size() + 256;
}

template <typename LenT>
static onng_status add_edges_impl(const onng_graph *g, const int32_t *src, const int32_t *dst,
                                  const LenT *len, int64_t m, int64_t *out_off, int32_t *out_nb,
                                  LenT *out_len, int64_t nnz_cap, int64_t *nnz_out, void *ws,
                                  hipStream_t st) {
    const int64_t n = g->n, nnz = g->nnz;
    Carver c(ws);
    int64_t *cnt = c.take<int64_t>(n + 1);
    int32_t *cursor = c.take<int32_t>(n);
    uint64_t *keys = c.take<uint64_t>(nnz + m);
    size_t tb = scan_temp_bytes(n + 1);
    void *tmp = c.take<char>(tb);
    ONNG_HIP(hipMemsetAsync(cnt, 0, sizeof(int64_t) * (n + 1), st));
    ONNG_HIP(hipMemsetAsync(cursor, 0, sizeof(int32_t) * n, st));
    const int64_t big = std::max(n, m);
    if (big > 0)
        hipLaunchKernelGGL(ae_count_kernel, dim3(blocks_for(big, 256)), dim3(256), 0, st,
                           g->offsets, n, src, dst, m, cnt);
    ONNG_HIP(hipcub::DeviceScan::ExclusiveSum(tmp, tb, cnt, out_off, (int)(n + 1), st));
    ONNG_HIP(hipMemcpyAsync(nnz_out, out_off + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    ONNG_HIP(hipStreamSynchronize(st));
    if (*nnz_out > nnz_cap) {
        set_error("onng_graph_add_edges: nnz_capacity too small");
        return ONNG_ERR_CAPACITY;
    }
    if (n > 0) {
        hipLaunchKernelGGL((ae_scatter_kernel<LenT>), dim3(blocks_for(n, 256)), dim3(256), 0, st,
                           g->offsets, g->nbrs, static_cast<const LenT *>(g->lens), n, src, dst,
                           len, m, out_off, cursor, keys);
        if (m > 0)
            hipLaunchKernelGGL((ae_new_kernel<LenT>), dim3(blocks_for(m, 256)), dim3(256), 0, st,
                               n, src, dst, len, m, out_off, cursor, keys);
        hipLaunchKernelGGL((segment_rank_sort_kernel<LenT>), dim3((unsigned)n), dim3(256),
                           4096 * sizeof(uint64_t), st, out_off, n, keys, out_nb, out_len);
    }
    ONNG_HIP(hipGetLastError());
    ONNG_HIP(hipStreamSynchronize(st));
    return ONNG_OK;
}

onng_status add_edges_launch(const onng_graph *g, const int32_t *src, const int32_t *dst,
                             const void *len, int64_t m, bool int_len, int64_t *out_off,
                             int32_t *out_nb, void *out_len, int64_t nnz_cap, int64_t *nnz_out,
                             void *ws, hipStream_t st) {
    if (int_len)
        return add_edges_impl<int32_t>(g, src, dst, static_cast<const int32_t *>(len), m, out_off,
                                       out_nb, static_cast<int32_t *>(out_len), nnz_cap, nnz_out,
                                       ws, st);
    return add_edges_impl<float>(g, src, dst, static_cast<const float *>(len), m, out_off, out_nb,
                                 static_cast<float *>(out_len), nnz_cap, nnz_out, ws, st);
}

size_t adjust_path_ws(int64_t n, int64_t nnz) {
    Carver c(nullptr);
    c.take<int32_t>(nnz);          // gp_nb
    c.take<int32_t>(nnz);          // gp_len (4-byte lengths)
    c.take<int32_t>(n);            // gp_cnt
    c.take<int8_t>(n);             // status
    c.take<int32_t>(n);            // degrees
    c.take<int32_t>(n);            // order
    c.take<int32_t>(4);            // undecided counter
    c.take<unsigned long long>(1 << 20);   // degree histogram (max degree < 2^20)
    c.take<int64_t>(1 << 20);      // start per degree
    c.take<int32_t>(1 << 20);      // cursor per degree
    c.take<int64_t>(n + 1);        // out counts
    c.take<char>(scan_temp_bytes(n + 1));
    c.take<int32_t>(nnz);          // edge index
    c.take<int32_t>(nnz);          // ids sorted per node
    c.take<int32_t>(nnz);          // their edge index
    c.take<int8_t>(nnz);           // kept flag per edge
    c.take<char>(segsort_temp_bytes(nnz, n));
    return c.size() + 256;
}

template <typename LenT>
static onng_status adjust_path_impl(const onng_graph *g, int64_t *out_off, int32_t *out_nb,
                                    LenT *out_len, int64_t *nnz_out, void *ws, hipStream_t st) {
    const int64_t n = g->n, nnz = g->nnz;
    const LenT *lens = static_cast<const LenT *>(g->lens);
    constexpr int MAXD = 1 << 20;
    Carver c(ws);
    int32_t *gp_nb = c.take<int32_t>(nnz);
    LenT *gp_len = reinterpret_cast<LenT *>(c.take<int32_t>(nnz));
    int32_t *gp_cnt = c.take<int32_t>(n);
    int8_t *status = c.take<int8_t>(n);
    int32_t *deg = c.take<int32_t>(n);
    int32_t *order = c.take<int32_t>(n);
    int32_t *undecided = c.take<int32_t>(4);
    unsigned long long *hist = c.take<unsigned long long>(MAXD);
    int64_t *start = c.take<int64_t>(MAXD);
    int32_t *cursor = c.take<int32_t>(MAXD);
    int64_t *ocnt = c.take<int64_t>(n + 1);
    size_t tb = scan_temp_bytes(n + 1);
    void *tmp = c.take<char>(tb);
    int32_t *eidx = c.take<int32_t>(nnz);
    int32_t *sid_nb = c.take<int32_t>(nnz);
    int32_t *sid_e = c.take<int32_t>(nnz);
    int8_t *kept = c.take<int8_t>(nnz);
    size_t sb = segsort_temp_bytes(nnz, n);
    void *stmp = c.take<char>(sb);
    // every node's edges sorted by id, for the witness lookups
    ONNG_HIP(hipMemsetAsync(kept, 0, (size_t)nnz, st));
    if (nnz > 0) {
        hipLaunchKernelGGL(iota_kernel, dim3(blocks_for(nnz, 256)), dim3(256), 0, st, nnz, eidx);
        ONNG_HIP(hipcub::DeviceSegmentedRadixSort::SortPairs(
            stmp, sb, g->nbrs, sid_nb, eidx, sid_e, (int)nnz, (int)n, g->offsets, g->offsets + 1,
            0, 32, st));
    }

    ONNG_HIP(hipMemsetAsync(gp_cnt, 0, sizeof(int32_t) * n, st));
    ONNG_HIP(hipMemsetAsync(hist, 0, sizeof(unsigned long long) * MAXD, st));
    ONNG_HIP(hipMemsetAsync(cursor, 0, sizeof(int32_t) * MAXD, st));
    hipLaunchKernelGGL(degree_hist_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, g->offsets,
                       n, deg, hist);
    std::vector<unsigned long long> h(MAXD);
    ONNG_HIP(hipMemcpyAsync(h.data(), hist, sizeof(unsigned long long) * MAXD,
                            hipMemcpyDeviceToHost, st));
    ONNG_HIP(hipStreamSynchronize(st));
    if (h[MAXD - 1]) {
        set_error("onng_adjust_path: a node has 2^20 - 1 or more edges");
        return ONNG_ERR_UNSUPPORTED;
    }
    int maxdeg = 0;
    for (int d = 0; d < MAXD; d++)
        if (h[d]) maxdeg = d;
    // start[d] = number of nodes with degree > d; active(j) = start[j] nodes
    std::vector<int64_t> s(MAXD, 0);
    int64_t acc = 0;
    for (int d = maxdeg; d >= 0; d--) {
        s[d] = acc;
        acc += (int64_t)h[d];
    }
    ONNG_HIP(hipMemcpyAsync(start, s.data(), sizeof(int64_t) * (maxdeg + 1), hipMemcpyHostToDevice,
                            st));
    hipLaunchKernelGGL(order_by_degree_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, deg, n,
                       start, cursor, order);
    for (int j = 0; j < maxdeg; j++) {
        int64_t n_act = s[j];    // nodes with degree > j
        if (n_act == 0) break;
        hipLaunchKernelGGL((pa_jacobi_kernel<LenT>), dim3(blocks_for(n_act * WAVE, 256)),
                           dim3(256), 0, st, g->offsets, g->nbrs, lens, order, n_act, j, gp_nb,
                           gp_cnt, sid_nb, sid_e, kept, status);
        for (int it = 0;; it++) {
            ONNG_HIP(hipMemsetAsync(undecided, 0, sizeof(int32_t), st));
            hipLaunchKernelGGL((pa_settle_kernel<LenT>), dim3(blocks_for(n_act, 256)), dim3(256),
                               0, st, g->offsets, g->nbrs, lens, order, n_act, j, gp_nb, gp_cnt,
                               status, undecided);
            int32_t und = 0;
            ONNG_HIP(hipMemcpyAsync(&und, undecided, sizeof(int32_t), hipMemcpyDeviceToHost, st));
            ONNG_HIP(hipStreamSynchronize(st));
            if (und == 0) break;
            if (it > n_act + 2) {
                set_error("onng_adjust_path: same-round dependences did not settle");
                return ONNG_ERR_DEVICE;
            }
        }
        hipLaunchKernelGGL((pa_apply_kernel<LenT>), dim3(blocks_for(n_act, 256)), dim3(256), 0, st,
                           g->offsets, g->nbrs, lens, order, n_act, j, gp_nb, gp_len, gp_cnt,
                           status, kept);
    }
    hipLaunchKernelGGL(cnt_to_i64_kernel, dim3(blocks_for(n + 1, 256)), dim3(256), 0, st, gp_cnt,
                       n, ocnt);
    ONNG_HIP(hipcub::DeviceScan::ExclusiveSum(tmp, tb, ocnt, out_off, (int)(n + 1), st));
    if (n > 0)
        hipLaunchKernelGGL((pa_compact_kernel<LenT>), dim3((unsigned)n), dim3(64), 0, st,
                           g->offsets, out_off, n, gp_nb, gp_len, out_nb, out_len);
    ONNG_HIP(hipGetLastError());
    ONNG_HIP(hipMemcpyAsync(nnz_out, out_off + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    ONNG_HIP(hipStreamSynchronize(st));
    return ONNG_OK;
}

onng_status adjust_path_launch(const onng_graph *g, bool int_len, int64_t *offsets,
                               int32_t *nbrs, void *lens, int64_t *nnz_out, void *ws,
                               hipStream_t st) {
    if (int_len)
        return adjust_path_impl<int32_t>(g, offsets, nbrs, static_cast<int32_t *>(lens), nnz_out,
                                         ws, st);
    return adjust_path_impl<float>(g, offsets, nbrs, static_cast<float *>(lens), nnz_out, ws, st);
}

}  // namespace onng
