// Entry seeds from a 4-way vantage-point tree (Section 3.2, Table 5).
//
// A node of m > leaf_size rows takes its row of lowest (priority, id) as
// vantage point v; the other m-1 rows, sorted by (d(v, x), x), are cut at
// floor(c (m-1) / 4), c = 0..4, into four children, and mu[c-1] is the
// distance of child c's first row.  A node of at most leaf_size rows is a
// leaf whose seeds are its n_seeds rows nearest its own vantage point.  A
// query descends by one distance computation per inner node, taking child
// #{c : d(q, v) >= mu[c]}, and returns its leaf's seeds.  With leaves of at
// most 100 rows the depth is 6-8 at 1M-10M rows, the count Table 5 reports.
//
// The build is level-synchronous: every inner node of a level picks its
// vantage point (one block per node), every row of those nodes gets its key
// (distance, id), one segmented radix sort orders all of the level's nodes,
// and the cut positions give the thresholds.  Nodes are numbered breadth
// first.  Tree distances use one fixed arithmetic, since they decide
// branches: exact integers on u8 rows; on f32 rows fp32 in coordinate order
// with every product and sum rounded on its own.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cstdint>
#include <vector>

#include "onng_internal.h"
#include "wave.h"

namespace onng {

namespace {

struct Seg {
    int64_t begin, size;
    int32_t node, aux;    // aux: first child (inner node) or leaf index (leaf)
};

template <bool U8, bool COS>
struct VDist {
    using T = typename std::conditional<U8, int32_t, float>::type;
    static __device__ T d(const uint8_t *a, const uint8_t *b, int dim) {
#pragma clang fp contract(off)
        if constexpr (U8) {
            int32_t s = 0;
            for (int t = 0; t < dim; t++) {
                int32_t df = (int32_t)a[t] - (int32_t)b[t];
                s += df * df;
            }
            return s;
        } else {
            const float *x = reinterpret_cast<const float *>(a);
            const float *y = reinterpret_cast<const float *>(b);
            float s = 0.0f;
            for (int t = 0; t < dim; t++) {
                if constexpr (COS) {
                    float pr = x[t] * y[t];
                    s = s + pr;
                } else {
                    float df = x[t] - y[t];
                    float sq = df * df;
                    s = s + sq;
                }
            }
            if constexpr (COS) return 1.0f - s;
            else return s;
        }
    }
    static __device__ uint32_t ord(T v) {
        if constexpr (U8) return (uint32_t)v;
        else return ord_f32(v);
    }
};

__global__ void vp_iota_kernel(int32_t *perm, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) perm[i] = (int32_t)i;
}

// one block per inner node: its lowest (priority, id) row moves to the front
__global__ void __launch_bounds__(256) vp_pick_kernel(int32_t *perm, const Seg *segs,
                                                      const uint32_t *prio, int32_t *node_vp) {
    __shared__ uint64_t best[256];
    __shared__ int64_t bpos[256];
    const Seg s = segs[blockIdx.x];
    uint64_t b = ~0ull;
    int64_t bp = 0;
    for (int64_t i = threadIdx.x; i < s.size; i += blockDim.x) {
        const int32_t x = perm[s.begin + i];
        const uint64_t k = ((uint64_t)prio[x] << 32) | (uint32_t)x;
        if (k < b) {
            b = k;
            bp = i;
        }
    }
    best[threadIdx.x] = b;
    bpos[threadIdx.x] = bp;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w && best[threadIdx.x + w] < best[threadIdx.x]) {
            best[threadIdx.x] = best[threadIdx.x + w];
            bpos[threadIdx.x] = bpos[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int64_t p = s.begin + bpos[0];
        const int32_t v = perm[p];
        perm[p] = perm[s.begin];
        perm[s.begin] = v;
        node_vp[s.node] = v;
    }
}

// the segment (of a begin-sorted list) holding position p
__device__ __forceinline__ int seg_of(const Seg *segs, int nseg, int64_t p) {
    int a = 0, b = nseg - 1;
    while (a < b) {
        const int m = (a + b + 1) >> 1;
        if (segs[m].begin <= p) a = m;
        else b = m - 1;
    }
    return a;
}

// key (distance to the node's vantage point, id) of every other row of the inner nodes
template <bool U8, bool COS>
__global__ void vp_keys_kernel(const int32_t *perm, const Seg *segs, int nseg, const uint8_t *base,
                               int64_t pitch, int dim, int64_t lo, int64_t hi, uint64_t *keys) {
    const int64_t p = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= hi) return;
    const Seg s = segs[seg_of(segs, nseg, p)];
    if (p <= s.begin || p >= s.begin + s.size) return;
    const int32_t v = perm[s.begin], x = perm[p];
    const auto d = VDist<U8, COS>::d(base + (int64_t)v * pitch, base + (int64_t)x * pitch, dim);
    keys[p] = make_key(VDist<U8, COS>::ord(d), (uint32_t)x);
}

// sorted rows back into place; each inner node's thresholds and children
template <bool U8>
__global__ void vp_place_kernel(int32_t *perm, const Seg *segs, int nseg, const uint64_t *sorted,
                                int64_t lo, int64_t hi, int32_t *node_child, void *node_mu) {
    const int64_t p = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= hi) return;
    const Seg s = segs[seg_of(segs, nseg, p)];
    if (p <= s.begin || p >= s.begin + s.size) return;
    const uint64_t k = sorted[p];
    perm[p] = (int32_t)(uint32_t)k;
    const int64_t m1 = s.size - 1, r = p - s.begin - 1;
    if (r == 0) node_child[s.node] = s.aux;
    for (int c = 1; c < 4; c++) {
        if (r != c * m1 / 4) continue;
        const uint32_t hi32 = (uint32_t)(k >> 32);
        if constexpr (U8) static_cast<int32_t *>(node_mu)[3 * (int64_t)s.node + c - 1] = (int32_t)hi32;
        else static_cast<float *>(node_mu)[3 * (int64_t)s.node + c - 1] = unord_f32(hi32);
    }
}

// one wave per leaf: vantage point and its n_seeds nearest rows (leaf_size <= 256)
template <bool U8, bool COS>
__global__ void __launch_bounds__(64) vp_leaf_kernel(const int32_t *perm, const Seg *segs,
                                                     const uint32_t *prio, const uint8_t *base,
                                                     int64_t pitch, int dim, int n_seeds,
                                                     int32_t *node_vp, int32_t *node_child,
                                                     int32_t *leaf_seeds) {
    __shared__ uint64_t k[256];
    const Seg s = segs[blockIdx.x];
    const int m = (int)s.size;
    const int lane = threadIdx.x;
    uint64_t b = ~0ull;
    for (int i = lane; i < m; i += 64) {
        const int32_t x = perm[s.begin + i];
        b = min(b, ((uint64_t)prio[x] << 32) | (uint32_t)x);
    }
    b = wave_min64(b);
    const int32_t v = (int32_t)(uint32_t)b;
    for (int i = lane; i < m; i += 64) {
        const int32_t x = perm[s.begin + i];
        const auto d = VDist<U8, COS>::d(base + (int64_t)v * pitch, base + (int64_t)x * pitch, dim);
        k[i] = make_key(VDist<U8, COS>::ord(d), (uint32_t)x);
    }
    __syncthreads();
    int32_t *out = leaf_seeds + (int64_t)s.aux * n_seeds;
    for (int i = lane; i < m; i += 64) {
        int rank = 0;
        for (int j = 0; j < m; j++) rank += k[j] < k[i];
        if (rank < n_seeds) out[rank] = (int32_t)(uint32_t)k[i];
    }
    for (int r = m + lane; r < n_seeds; r += 64) out[r] = -1;
    if (lane == 0) {
        node_vp[s.node] = v;
        node_child[s.node] = -1 - s.aux;
    }
}

// one thread per query
template <bool U8, bool COS>
__global__ void vp_descend_kernel(const uint8_t *base, int64_t bpitch, const uint8_t *qs,
                                  int64_t qpitch, int64_t nq, int dim, const int32_t *node_vp,
                                  const int32_t *node_child, const void *node_mu,
                                  const int32_t *leaf_seeds, int n_seeds, int64_t n_nodes,
                                  int64_t n_leaves, int64_t n_base, int32_t *seeds, int32_t *dc) {
    using T = typename VDist<U8, COS>::T;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq) return;
    const T *mu = static_cast<const T *>(node_mu);
    int64_t node = 0;
    int cnt = 0;
    bool bad = false;
    // every index is checked against the tree's counts, and the depth is
    // bounded, so a tree not made by the build cannot fault or loop
    while (!bad && node_child[node] >= 0 && cnt < 64) {
        const int32_t v = node_vp[node];
        bad = v < 0 || v >= n_base;
        if (bad) break;
        const T d = VDist<U8, COS>::d(qs + q * qpitch, base + (int64_t)v * bpitch, dim);
        const int c = (d >= mu[3 * node]) + (d >= mu[3 * node + 1]) + (d >= mu[3 * node + 2]);
        node = (int64_t)node_child[node] + c;
        bad = node >= n_nodes;
        cnt++;
    }
    int32_t *out = seeds + q * n_seeds;
    const int64_t leaf = bad ? -1 : -1 - (int64_t)node_child[node];
    if (bad || leaf < 0 || leaf >= n_leaves) {
        for (int r = 0; r < n_seeds; r++) out[r] = -1;
        dc[q] = -1;
        return;
    }
    const int32_t *src = leaf_seeds + leaf * n_seeds;
    for (int r = 0; r < n_seeds; r++) out[r] = src[r];
    dc[q] = cnt;
}

inline unsigned blocks_of(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

size_t vp_sort_temp(int64_t n) {
    size_t bytes = 0;
    (void)hipcub::DeviceSegmentedRadixSort::SortKeys(nullptr, bytes, (const uint64_t *)nullptr,
                                                     (uint64_t *)nullptr, (int)n, (int)n,
                                                     (const int64_t *)nullptr,
                                                     (const int64_t *)nullptr);
    return bytes;
}

template <bool U8, bool COS>
onng_status vptree_build_impl(const onng_vectors *base, const uint32_t *prio, onng_vptree *t,
                              void *ws, hipStream_t st) {
    const int64_t n = base->n;
    const uint8_t *B = static_cast<const uint8_t *>(base->data);
    const int64_t pitch = base->pitch_bytes;
    const int dim = base->dim;
    Carver c(ws);
    int32_t *perm = c.take<int32_t>(n);
    uint64_t *keys = c.take<uint64_t>(n);
    uint64_t *sorted = c.take<uint64_t>(n);
    Seg *dinner = c.take<Seg>(n);
    Seg *dleaf = c.take<Seg>(n);
    int64_t *sb = c.take<int64_t>(n);
    int64_t *se = c.take<int64_t>(n);
    size_t tb = vp_sort_temp(n);
    void *tmp = c.take<char>(tb);
    hipLaunchKernelGGL(vp_iota_kernel, dim3(blocks_of(n, 256)), dim3(256), 0, st, perm, n);
    std::vector<Seg> level{Seg{0, n, 0, 0}}, inner, leaves, nextl;
    std::vector<int64_t> hb, he;
    int64_t next = 1, nleaf = 0;
    while (!level.empty()) {
        inner.clear();
        leaves.clear();
        for (Seg s : level) {
            if (s.size > t->leaf_size) {
                s.aux = (int32_t)next;
                next += 4;
                inner.push_back(s);
            } else {
                s.aux = (int32_t)nleaf++;
                leaves.push_back(s);
            }
        }
        if (next > t->node_capacity || nleaf > t->leaf_capacity) {
            set_error("onng_vptree_build: node or leaf capacity too small");
            return ONNG_ERR_CAPACITY;
        }
        if (!inner.empty()) {
            const int ni = (int)inner.size();
            hb.resize(ni);
            he.resize(ni);
            for (int i = 0; i < ni; i++) {
                hb[i] = inner[i].begin + 1;
                he[i] = inner[i].begin + inner[i].size;
            }
            ONNG_HIP(hipMemcpyAsync(dinner, inner.data(), sizeof(Seg) * ni, hipMemcpyHostToDevice, st));
            ONNG_HIP(hipMemcpyAsync(sb, hb.data(), sizeof(int64_t) * ni, hipMemcpyHostToDevice, st));
            ONNG_HIP(hipMemcpyAsync(se, he.data(), sizeof(int64_t) * ni, hipMemcpyHostToDevice, st));
            hipLaunchKernelGGL(vp_pick_kernel, dim3(ni), dim3(256), 0, st, perm, dinner, prio,
                               t->node_vp);
            const int64_t lo = inner.front().begin, hi = inner.back().begin + inner.back().size;
            hipLaunchKernelGGL((vp_keys_kernel<U8, COS>), dim3(blocks_of(hi - lo, 256)), dim3(256),
                               0, st, perm, dinner, ni, B, pitch, dim, lo, hi, keys);
            size_t b = tb;
            ONNG_HIP(hipcub::DeviceSegmentedRadixSort::SortKeys(tmp, b, keys, sorted, (int)n, ni,
                                                                sb, se, 0, 64, st));
            hipLaunchKernelGGL((vp_place_kernel<U8>), dim3(blocks_of(hi - lo, 256)), dim3(256), 0,
                               st, perm, dinner, ni, sorted, lo, hi, t->node_child, t->node_mu);
        }
        if (!leaves.empty()) {
            const int nl = (int)leaves.size();
            ONNG_HIP(hipMemcpyAsync(dleaf, leaves.data(), sizeof(Seg) * nl, hipMemcpyHostToDevice, st));
            hipLaunchKernelGGL((vp_leaf_kernel<U8, COS>), dim3(nl), dim3(64), 0, st, perm, dleaf,
                               prio, B, pitch, dim, t->n_seeds, t->node_vp, t->node_child,
                               t->leaf_seeds);
        }
        ONNG_HIP(hipGetLastError());
        ONNG_HIP(hipStreamSynchronize(st));    // host segment lists are reused next level
        nextl.clear();
        for (const Seg &s : inner) {
            const int64_t m1 = s.size - 1;
            for (int k = 0; k < 4; k++) {
                const int64_t r0 = k * m1 / 4, r1 = (k + 1) * m1 / 4;
                nextl.push_back(Seg{s.begin + 1 + r0, r1 - r0, s.aux + k, 0});
            }
        }
        level.swap(nextl);
    }
    t->n_nodes = next;
    t->n_leaves = nleaf;
    return ONNG_OK;
}

template <bool U8, bool COS>
void vptree_seeds_impl(const onng_vectors *base, const onng_vptree *t, const onng_vectors *q,
                       int32_t *seeds, int32_t *dc, hipStream_t st) {
    if (q->n == 0) return;
    hipLaunchKernelGGL((vp_descend_kernel<U8, COS>), dim3(blocks_of(q->n, 256)), dim3(256), 0, st,
                       static_cast<const uint8_t *>(base->data), base->pitch_bytes,
                       static_cast<const uint8_t *>(q->data), q->pitch_bytes, q->n, base->dim,
                       t->node_vp, t->node_child, t->node_mu, t->leaf_seeds, t->n_seeds,
                       t->n_nodes, t->n_leaves, base->n, seeds, dc);
}

}  // namespace

size_t vptree_ws(int64_t n) {
    Carver c(nullptr);
    c.take<int32_t>(n);
    c.take<uint64_t>(n);
    c.take<uint64_t>(n);
    c.take<Seg>(n);
    c.take<Seg>(n);
    c.take<int64_t>(n);
    c.take<int64_t>(n);
    c.take<char>(vp_sort_temp(n));
    return c.size() + 256;
}

onng_status vptree_build_launch(const onng_vectors *base, const uint32_t *prio, onng_vptree *t,
                                void *ws, hipStream_t st) {
    if (base->dtype == ONNG_U8) return vptree_build_impl<true, false>(base, prio, t, ws, st);
    if (base->metric == ONNG_COSINE) return vptree_build_impl<false, true>(base, prio, t, ws, st);
    return vptree_build_impl<false, false>(base, prio, t, ws, st);
}

onng_status vptree_seeds_launch(const onng_vectors *base, const onng_vptree *t,
                                const onng_vectors *q, int32_t *seeds, int32_t *dc,
                                hipStream_t st) {
    if (base->dtype == ONNG_U8) vptree_seeds_impl<true, false>(base, t, q, seeds, dc, st);
    else if (base->metric == ONNG_COSINE) vptree_seeds_impl<false, true>(base, t, q, seeds, dc, st);
    else vptree_seeds_impl<false, false>(base, t, q, seeds, dc, st);
    ONNG_HIP(hipGetLastError());
    return ONNG_OK;
}

}  // namespace onng
