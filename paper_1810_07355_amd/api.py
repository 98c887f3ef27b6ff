"""Python binding of libonng.so: argument marshalling only.

Torch tensors provide device memory and the current HIP stream; every step of
the path runs in the library's kernels.  Function names follow the C-ABI
(include/onng.h) without the `onng_` prefix."""
from __future__ import annotations

import ctypes as C
import dataclasses
import math

import numpy as np
import torch

from . import _lib as L

_DTYPE_BYTES = {L.U8: 1, L.F32: 4, L.F16: 2, L.BF16: 2, L.FP8_E4M3: 1}


def _ptr(t):
    return None if t is None else t.data_ptr()


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def row_pitch(dim: int, dtype: int, align: int = 16) -> int:
    """Smallest multiple of `align` bytes holding `dim` elements of `dtype`."""
    return (dim * _DTYPE_BYTES[dtype] + align - 1) // align * align


class Vectors:
    """Device rows of one storage type.  `data` is a uint8/float tensor
    [n, pitch_bytes / element size]; `scale` the FP8 per-row scale."""

    def __init__(self, data: torch.Tensor, dtype: int, metric: int, dim: int,
                 scale: torch.Tensor | None = None):
        assert data.is_cuda and data.is_contiguous()
        self.data = data
        self.dtype = dtype
        self.metric = metric
        self.dim = dim
        self.n = data.shape[0]
        self.pitch = data.shape[1] * data.element_size() if data.dim() == 2 else 0
        self.scale = scale
        self._s = L.Vectors_t(data.data_ptr(), _ptr(scale), self.n, dim, dtype, self.pitch,
                              metric, 0)

    @property
    def ref(self):
        return C.byref(self._s)

    @property
    def dist_dtype(self):
        return torch.int32 if (self.dtype == L.U8 and self.metric == L.L2SQ) else torch.float32

    @staticmethod
    def from_tensor(x: torch.Tensor, metric: int, pitch: int | None = None) -> "Vectors":
        """u8 or f32 rows, padded with zeros to a 16-byte pitch (or to
        `pitch` bytes, e.g. whole 128-byte cache lines)."""
        n, dim = x.shape
        dtype = L.U8 if x.dtype == torch.uint8 else L.F32
        esz = _DTYPE_BYTES[dtype]
        cols = max(row_pitch(dim, dtype), pitch or 0) // esz
        if cols != dim:
            buf = torch.zeros((n, cols), dtype=x.dtype, device=x.device)
            buf[:, :dim] = x
            x = buf
        return Vectors(x.contiguous(), dtype, metric, dim)


@dataclasses.dataclass
class Graph:
    offsets: torch.Tensor
    nbrs: torch.Tensor
    lens: torch.Tensor | None

    @property
    def n(self):
        return self.offsets.numel() - 1

    @property
    def nnz(self):
        return self.nbrs.numel()

    def struct(self):
        return L.Graph_t(self.offsets.data_ptr(), self.nbrs.data_ptr(), _ptr(self.lens), self.n,
                         self.nnz)


# ------------------------------------------------------------------ top-k --

def topk(queries: Vectors, base: Vectors, k: int, cand: torch.Tensor | None = None,
         exclude_self: bool = False):
    dev = queries.data.device
    ids = torch.empty((queries.n, k), dtype=torch.int32, device=dev)
    d = torch.empty((queries.n, k), dtype=queries.dist_dtype, device=dev)
    nc = 0 if cand is None else cand.numel()
    ws_n = L.load().onng_topk_workspace_size(queries.ref, base.ref, nc, k)
    ws = _workspace(ws_n, dev)
    L.call("onng_topk", queries.ref, base.ref, _ptr(cand), nc, k, int(exclude_self),
           ids.data_ptr(), d.data_ptr(), ws.data_ptr(), ws.numel(), _stream())
    return ids, d


def build_knn(base: Vectors, k: int):
    dev = base.data.device
    ids = torch.empty((base.n, k), dtype=torch.int32, device=dev)
    d = torch.empty((base.n, k), dtype=base.dist_dtype, device=dev)
    ws_n = L.load().onng_topk_workspace_size(base.ref, base.ref, 0, k)
    ws = _workspace(ws_n, dev)
    L.call("onng_build_knn", base.ref, k, ids.data_ptr(), d.data_ptr(), ws.data_ptr(),
           ws.numel(), _stream())
    return ids, d


# ------------------------------------------------------------ adjustments --

def adjust_degree(knn_ids: torch.Tensor, knn_d: torch.Tensor, dtype: int, metric: int, e_o: int,
                  e_i: int) -> Graph:
    n, k = knn_ids.shape
    dev = knn_ids.device
    cap = n * (min(e_o, k) + min(e_i, k))
    off = torch.empty(n + 1, dtype=torch.int64, device=dev)
    nb = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    ln = torch.empty(max(cap, 1), dtype=knn_d.dtype, device=dev)
    ws = _workspace(L.load().onng_adjust_degree_workspace_size(n, k, e_o, e_i), dev)
    nnz = C.c_int64(0)
    L.call("onng_adjust_degree", knn_ids.data_ptr(), knn_d.data_ptr(), n, k, dtype, metric, e_o,
           e_i, off.data_ptr(), nb.data_ptr(), ln.data_ptr(), cap, C.byref(nnz), ws.data_ptr(),
           ws.numel(), _stream())
    return Graph(off, nb[:nnz.value].clone(), ln[:nnz.value].clone())


def adjust_degree_constrained(knn_ids: torch.Tensor, knn_d: torch.Tensor, dtype: int,
                              metric: int, e_o: int, e_i: int) -> Graph:
    n, k = knn_ids.shape
    dev = knn_ids.device
    cap = n * (min(e_o, k) + min(e_i, k))
    off = torch.empty(n + 1, dtype=torch.int64, device=dev)
    nb = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    ln = torch.empty(max(cap, 1), dtype=knn_d.dtype, device=dev)
    ws = _workspace(L.load().onng_adjust_degree_constrained_workspace_size(n, k, e_o, e_i), dev)
    nnz = C.c_int64(0)
    L.call("onng_adjust_degree_constrained", knn_ids.data_ptr(), knn_d.data_ptr(), n, k, dtype,
           metric, e_o, e_i, off.data_ptr(), nb.data_ptr(), ln.data_ptr(), cap, C.byref(nnz),
           ws.data_ptr(), ws.numel(), _stream())
    return Graph(off, nb[:nnz.value].clone(), ln[:nnz.value].clone())


def graph_stats(g: Graph, dtype: int, metric: int, frac: float = 0.05, keep: int = 10):
    """(mean top-frac out-degree, mean bottom-frac in-degree, mean length of
    every node's `keep` shortest incoming edges) of a graph, as in Table 4."""
    ws = _workspace(L.load().onng_graph_stats_workspace_size(g.n, g.nnz), g.offsets.device)
    out = (C.c_double * 3)()
    L.call("onng_graph_stats", C.byref(g.struct()), dtype, metric, frac, keep, out,
           ws.data_ptr(), ws.numel(), _stream())
    return tuple(out)


def graph_add_edges(g: Graph, src: torch.Tensor, dst: torch.Tensor, lens: torch.Tensor,
                    dtype: int, metric: int) -> Graph:
    """g plus the edges src -> dst (ids outside [0, n) skipped), lists sorted
    by (length, id)."""
    dev = g.offsets.device
    m = src.numel()
    cap = g.nnz + m
    off = torch.empty_like(g.offsets)
    nb = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    ln = torch.empty(max(cap, 1), dtype=lens.dtype, device=dev)
    ws = _workspace(L.load().onng_graph_add_edges_workspace_size(g.n, g.nnz, m), dev)
    nnz = C.c_int64(0)
    L.call("onng_graph_add_edges", C.byref(g.struct()), _ptr(src), _ptr(dst), _ptr(lens), m,
           dtype, metric, off.data_ptr(), nb.data_ptr(), ln.data_ptr(), cap, C.byref(nnz),
           ws.data_ptr(), ws.numel(), _stream())
    return Graph(off, nb[:nnz.value].clone(), ln[:nnz.value].clone())


def graph_head(g: Graph, k: int, dtype: int, metric: int):
    """Algorithm 8's first step: every node's k shortest edges as a padded
    table (ids [n][k], dists [n][k]), the AKNNG of an ANNG."""
    dev = g.offsets.device
    ids = torch.empty((g.n, k), dtype=torch.int32, device=dev)
    dt = torch.int32 if (dtype == L.U8 and metric == L.L2SQ) else torch.float32
    d = torch.empty((g.n, k), dtype=dt, device=dev)
    L.call("onng_graph_head", C.byref(g.struct()), dtype, metric, k, ids.data_ptr(), d.data_ptr(),
           _stream())
    return ids, d


class VPTree:
    """A 4-way vantage-point tree for entry seeds (Section 3.2, Table 5);
    built by vptree_build, its arrays live on the device."""

    def __init__(self, n: int, device, int_dist: bool, leaf_size: int, n_seeds: int):
        self.node_vp = torch.empty(n, dtype=torch.int32, device=device)
        self.node_child = torch.empty(n, dtype=torch.int32, device=device)
        self.node_mu = torch.empty(3 * n, dtype=torch.int32 if int_dist else torch.float32,
                                   device=device)
        self.leaf_seeds = torch.empty(n * n_seeds, dtype=torch.int32, device=device)
        self.t = L.VPTree_t(self.node_vp.data_ptr(), self.node_child.data_ptr(),
                            self.node_mu.data_ptr(), self.leaf_seeds.data_ptr(), n, n,
                            leaf_size, n_seeds, 0, 0)

    @property
    def n_nodes(self):
        return self.t.n_nodes

    @property
    def n_leaves(self):
        return self.t.n_leaves

    @property
    def n_seeds(self):
        return self.t.n_seeds


def vptree_build(base: Vectors, priority: torch.Tensor, leaf_size: int = 100,
                 n_seeds: int = 10) -> VPTree:
    dev = priority.device
    tree = VPTree(base.n, dev, base.dtype == L.U8, leaf_size, n_seeds)
    ws = _workspace(L.load().onng_vptree_build_workspace_size(base.n), dev)
    L.call("onng_vptree_build", base.ref, priority.data_ptr(), C.byref(tree.t),
           ws.data_ptr(), ws.numel(), _stream())
    return tree


def vptree_seeds(base: Vectors, tree: VPTree, queries: Vectors):
    """(seeds [nq][n_seeds] int32, distance computations [nq] int32)."""
    dev = tree.node_vp.device
    seeds = torch.empty((queries.n, tree.n_seeds), dtype=torch.int32, device=dev)
    dc = torch.empty(queries.n, dtype=torch.int32, device=dev)
    L.call("onng_vptree_seeds", base.ref, C.byref(tree.t), queries.ref,
           seeds.data_ptr(), dc.data_ptr(), _stream())
    return seeds, dc


def adjust_path(g: Graph, dtype: int, metric: int) -> Graph:
    dev = g.offsets.device
    off = torch.empty_like(g.offsets)
    nb = torch.empty(max(g.nnz, 1), dtype=torch.int32, device=dev)
    ln = torch.empty(max(g.nnz, 1), dtype=g.lens.dtype, device=dev)
    ws = _workspace(L.load().onng_adjust_path_workspace_size(g.n, g.nnz), dev)
    gs = g.struct()
    nnz = C.c_int64(0)
    L.call("onng_adjust_path", C.byref(gs), dtype, metric, off.data_ptr(), nb.data_ptr(),
           ln.data_ptr(), C.byref(nnz), ws.data_ptr(), ws.numel(), _stream())
    return Graph(off, nb[:nnz.value].clone(), ln[:nnz.value].clone())


# ----------------------------------------------------------------- search --

@dataclasses.dataclass
class Predictor:
    """Weights of the search-range predictor (bf16 matrices, f32 vectors).
    mode L.PRED_LOG_EPS: head `head` predicts log10(eps + 0.01) (+ shift).
    mode L.PRED_CURVE: heads [0, G) recall and [G, 2G) log(1 + cost) at
    eps_cand[g] (the cost in distance-computation units: the count itself, or
    the query's search time scaled to it); the query takes argmax recall -
    lambda*cost."""
    w1_bf16: torch.Tensor
    b1: torch.Tensor
    w2_bf16: torch.Tensor
    b2: torch.Tensor
    mean: torch.Tensor
    std: torch.Tensor
    shift: torch.Tensor | None = None
    head: int = 0
    head_per_query: torch.Tensor | None = None
    eps_min: float = 0.0
    eps_max: float = 0.5
    e0: float = 30.0
    we: float = -1.0
    mode: int = L.PRED_LOG_EPS
    eps_cand: torch.Tensor | None = None
    lam: float = 0.0
    lambda_per_query: torch.Tensor | None = None

    def struct(self):
        return L.Predictor_t(self.w1_bf16.data_ptr(), self.b1.data_ptr(), self.w2_bf16.data_ptr(),
                             self.b2.data_ptr(), self.mean.data_ptr(), self.std.data_ptr(),
                             _ptr(self.shift), _ptr(self.head_per_query), self.head, L.NFEAT,
                             self.b1.numel(), self.b2.numel(), self.eps_min, self.eps_max,
                             self.e0, self.we, self.mode,
                             0 if self.eps_cand is None else self.eps_cand.numel(),
                             _ptr(self.eps_cand), self.lam, _ptr(self.lambda_per_query))


def launch_config(waves_per_block=0, lanes_per_row=0, s_capacity=0, visited_log2=0,
                  pool_capacity=0, blocks=0):
    return L.LaunchConfig_t(waves_per_block, lanes_per_row, s_capacity, visited_log2,
                            pool_capacity, blocks)


class SearchRequest:
    """Holds the C parameter block and every buffer it points to."""

    def __init__(self, base: Vectors, graph: Graph, queries: Vectors, seeds: torch.Tensor, k=10,
                 k_stride=None, eps=0.0, ep=L.EP_INF, two_phase=False, ep_first=L.EP_INF,
                 predictor: Predictor | None = None, want_features=False,
                 rerank_base: Vectors | None = None, pool_factor=4, launch=None, probe_hops=1,
                 predict_only=False, range_from: torch.Tensor | None = None,
                 order: torch.Tensor | None = None, max_dc=0, max_dc_factor=0.0,
                 id_map: torch.Tensor | None = None, single_pass=False, static_scratch=False):
        """static_scratch: run through onng_search_static (the library's
        static device scratch; no workspace is allocated)."""
        dev = queries.data.device
        nq = queries.n
        self.base, self.graph, self.queries = base, graph, queries
        self.seeds = seeds.contiguous()
        self._keep = []
        kq = None
        if torch.is_tensor(k):
            kq = k.to(device=dev, dtype=torch.int32).contiguous()
            kmax = int(kq.max()) if nq else 1
            k = kmax
        self.k_stride = k_stride or int(k)
        epsq = None
        if torch.is_tensor(eps):
            epsq = eps.to(device=dev, dtype=torch.float32).contiguous()
            eps = 0.0
        epq = None
        if torch.is_tensor(ep):
            epq = ep.to(device=dev, dtype=torch.int64).to(torch.int32).contiguous()
            ep = 1
        mdq = None
        if torch.is_tensor(max_dc):
            mdq = max_dc.to(device=dev, dtype=torch.int32).contiguous()
            max_dc = 0
        self._keep += [kq, epsq, epq, mdq]
        self.predictor = predictor
        self._pred_s = predictor.struct() if predictor else None
        self.features = (torch.zeros((nq, L.NFEAT), dtype=torch.float32, device=dev)
                         if want_features else None)
        self.rerank_base = rerank_base
        self._launch = launch
        self.params = L.SearchParams_t(
            int(k), self.k_stride, _ptr(kq), float(eps), _ptr(epsq), int(ep) & 0xFFFFFFFF,
            _ptr(epq), int(two_phase), int(ep_first) & 0xFFFFFFFF,
            C.cast(C.byref(self._pred_s), C.c_void_p) if predictor else None,
            _ptr(self.features),
            C.cast(rerank_base.ref, C.c_void_p) if rerank_base else None,
            int(pool_factor), C.cast(C.byref(launch), C.c_void_p) if launch is not None else None,
            int(probe_hops), int(predict_only), _ptr(range_from), _ptr(order), int(max_dc),
            _ptr(mdq), float(max_dc_factor), _ptr(id_map), int(single_pass), 0)
        self._keep += [range_from, order, id_map]
        self.gs = graph.struct()
        out_dt = torch.float32 if rerank_base is not None else base.dist_dtype
        self.ids = torch.empty((nq, self.k_stride), dtype=torch.int32, device=dev)
        self.dists = torch.empty((nq, self.k_stride), dtype=out_dt, device=dev)
        self.stats = torch.empty((nq, 8), dtype=torch.int32, device=dev)
        self.static_scratch = bool(static_scratch)
        self.ws = None
        if self.static_scratch:
            return
        self.ws_bytes = L.load().onng_search_workspace_size(base.ref, nq, C.byref(self.params))
        if self.ws_bytes == 0:
            raise L.OnngError("onng_search_workspace_size", L.ERR_INVALID_ARG,
                              L.load().onng_last_error().decode())
        self.ws = _workspace(self.ws_bytes, dev)

    def run(self):
        if self.static_scratch:
            L.call("onng_search_static", self.base.ref, C.byref(self.gs), self.queries.ref,
                   self.seeds.data_ptr(), self.seeds.shape[1], C.byref(self.params),
                   self.ids.data_ptr(), self.dists.data_ptr(), self.stats.data_ptr(), _stream())
            return self
        L.call("onng_search", self.base.ref, C.byref(self.gs), self.queries.ref,
               self.seeds.data_ptr(), self.seeds.shape[1], C.byref(self.params),
               self.ids.data_ptr(), self.dists.data_ptr(), self.stats.data_ptr(),
               self.ws.data_ptr(), self.ws.numel(), _stream())
        # the workspace is this request's: later runs reuse its zeroed bitsets
        self.params.ws_reuse = 1
        return self

    def autotune(self):
        best = L.LaunchConfig_t()
        L.call("onng_autotune_search", self.base.ref, C.byref(self.gs), self.queries.ref,
               self.seeds.data_ptr(), self.seeds.shape[1], C.byref(self.params),
               self.ids.data_ptr(), self.dists.data_ptr(), self.stats.data_ptr(),
               self.ws.data_ptr(), self.ws.numel(), _stream(), C.byref(best))
        # the tuned shape may need a different workspace
        self.ws_bytes = L.load().onng_search_workspace_size(self.base.ref, self.queries.n,
                                                            C.byref(self.params))
        if self.ws_bytes > self.ws.numel():
            self.ws = _workspace(self.ws_bytes, self.ws.device)
            self.params.ws_reuse = 0
        return best

    @property
    def dc(self):
        return self.stats[:, 0]

    @property
    def hops(self):
        return self.stats[:, 1]

    @property
    def flags(self):
        return self.stats[:, 2]

    @property
    def ep_used(self):
        return self.stats[:, 3].to(torch.int64) & 0xFFFFFFFF

    @property
    def eps_used(self):
        return self.stats[:, 4].view(torch.float32)

    @property
    def scanned(self):
        return self.stats[:, 5]

    @property
    def cost(self):
        return self.stats[:, 6].view(torch.float32)

    @property
    def us(self):
        """Per-query device wall time in microseconds."""
        return self.stats[:, 7].view(torch.float32)


def locality_order(base: Vectors, pivots: torch.Tensor) -> torch.Tensor:
    """Permutation grouping the rows by nearest pivot (see onng_locality_order)."""
    pivots = pivots.contiguous().to(torch.int32)
    perm = torch.empty(base.n, dtype=torch.int32, device=base.data.device)
    n_ws = L.load().onng_locality_order_workspace_size(base.ref, pivots.numel())
    ws = _workspace(n_ws, base.data.device)
    L.call("onng_locality_order", base.ref, pivots.data_ptr(), pivots.numel(), perm.data_ptr(),
           ws.data_ptr(), ws.numel(), _stream())
    return perm


def gather_rows(x: torch.Tensor, ids: torch.Tensor) -> torch.Tensor:
    """Rows of a device tensor [n, ...] in the order `ids` (library kernel)."""
    x = x.contiguous()
    ids = ids.contiguous().to(torch.int32)
    out = torch.empty((ids.numel(),) + tuple(x.shape[1:]), dtype=x.dtype, device=x.device)
    pitch = x[0].numel() * x.element_size() if x.shape[0] else 16
    L.call("onng_gather_rows", x.data_ptr(), pitch, ids.data_ptr(), ids.numel(),
           out.data_ptr(), _stream())
    return out


def order_by_cost(stats: torch.Tensor, order: torch.Tensor | None = None) -> torch.Tensor:
    """Query indices by descending predicted cost (longest first)."""
    n = stats.shape[0]
    order = torch.empty(n, dtype=torch.int32, device=stats.device) if order is None else order
    ws = _workspace(L.load().onng_order_by_cost_workspace_size(n), stats.device)
    L.call("onng_order_by_cost", stats.data_ptr(), n, order.data_ptr(), ws.data_ptr(), ws.numel(),
           _stream())
    return order


class LearnedSearch:
    """Search with a learned range, scheduled longest first: a predict-only
    pass chooses each query's range and cost, the queries are ordered by
    that cost, and the search runs with the chosen ranges in that order."""

    def __init__(self, base, graph, queries, seeds, predictor: Predictor, ep_first=L.EP_INF,
                 probe_hops=1, **kw):
        kw.pop("two_phase", None)
        kw.pop("eps", None)
        kw.pop("ep", None)
        self.pre = SearchRequest(base, graph, queries, seeds, two_phase=True, ep_first=ep_first,
                                 probe_hops=probe_hops, predictor=predictor, predict_only=True,
                                 **{k: v for k, v in kw.items() if k != "want_features"})
        self.order = torch.empty(queries.n, dtype=torch.int32, device=queries.data.device)
        self.ows = _workspace(L.load().onng_order_by_cost_workspace_size(queries.n),
                              queries.data.device)
        self.req = SearchRequest(base, graph, queries, seeds, range_from=self.pre.stats,
                                 order=self.order, **kw)

    def run(self):
        self.pre.run()
        L.call("onng_order_by_cost", self.pre.stats.data_ptr(), self.order.numel(),
               self.order.data_ptr(), self.ows.data_ptr(), self.ows.numel(), _stream())
        self.req.run()
        return self.req

    # result accessors of the final pass
    def __getattr__(self, name):
        return getattr(self.__dict__["req"], name)


def search(base, graph, queries, seeds, **kw) -> SearchRequest:
    return SearchRequest(base, graph, queries, seeds, **kw).run()


# ------------------------------------------------------ codecs and rerank --

def fp8_inrow_pitch(dim: int) -> int:
    """Smallest pitch of FP8 rows that carry their scale in the last 4 bytes."""
    return (dim + 15) // 16 * 16 + 16


def encode(x: torch.Tensor, dtype: int, metric: int, pitch: int | None = None,
           scale_in_row: bool = False) -> Vectors:
    """f32 rows -> stored rows of `dtype` (Vectors with uint8 storage).
    FP8 rows keep their per-row scale in a separate array, or with
    scale_in_row in the last 4 bytes of the row (one cache line per row for
    up to 112 components at a 128-byte pitch)."""
    x = x.contiguous().to(torch.float32)
    n, dim = x.shape
    inrow = scale_in_row and dtype == L.FP8_E4M3
    pitch = pitch or (fp8_inrow_pitch(dim) if inrow else row_pitch(dim, dtype))
    out = torch.empty((n, pitch), dtype=torch.uint8, device=x.device)
    scale = (torch.empty(n, dtype=torch.float32, device=x.device)
             if dtype == L.FP8_E4M3 and not inrow else None)
    L.call("onng_encode", x.data_ptr(), n, dim, dtype, out.data_ptr(), pitch, _ptr(scale),
           _stream())
    return Vectors(out, dtype, metric, dim, scale)


def rerank(queries: Vectors, base: Vectors, pool: torch.Tensor, k: int, use_f64=False):
    pool = pool.contiguous().to(torch.int32)
    nq, psz = pool.shape
    ids = torch.empty((nq, k), dtype=torch.int32, device=pool.device)
    d = torch.empty((nq, k), dtype=torch.float64 if use_f64 else torch.float32,
                    device=pool.device)
    L.call("onng_rerank", queries.ref, base.ref, pool.data_ptr(), psz, k, int(use_f64),
           ids.data_ptr(), d.data_ptr(), _stream())
    return ids, d


def ground_truth(queries: Vectors, base: Vectors, k: int, screen: int = 64):
    """Exact top-k: u8 directly; float by f32 screening of k+screen, then f64."""
    if base.dtype == L.U8:
        return topk(queries, base, k)
    kk = min(k + screen, 256, base.n)
    pool, _ = topk(queries, base, kk)
    return rerank(queries, base, pool, k, use_f64=True)


# -------------------------------------------------------------------- MLP --

def mlp_forward(X, W1, b1, W2, b2, want_hidden=False):
    B, F = X.shape
    H, T = W1.shape[0], W2.shape[0]
    Y = torch.empty((B, T), dtype=torch.float32, device=X.device)
    hid = torch.empty((B, H), dtype=torch.float32, device=X.device) if want_hidden else None
    L.call("onng_mlp_forward", X.data_ptr(), B, F, W1.data_ptr(), b1.data_ptr(), H,
           W2.data_ptr(), b2.data_ptr(), T, _ptr(hid), Y.data_ptr(), _stream())
    return (Y, hid) if want_hidden else Y


def mlp_backward(X, target, W1, b1, W2, b2, w=None):
    B, F = X.shape
    H, T = W1.shape[0], W2.shape[0]
    g = [torch.empty_like(t) for t in (W1, b1, W2, b2)]
    loss = torch.empty(1, dtype=torch.float32, device=X.device)
    ws = _workspace(L.load().onng_mlp_backward_workspace_size(B, H, T), X.device)
    L.call("onng_mlp_backward", X.data_ptr(), target.data_ptr(), _ptr(w), B, F, W1.data_ptr(),
           b1.data_ptr(), H, W2.data_ptr(), b2.data_ptr(), T, *[t.data_ptr() for t in g],
           loss.data_ptr(), ws.data_ptr(), ws.numel(), _stream())
    return loss, g


def adam_step(p, g, m, v, lr, t, beta1=0.9, beta2=0.999, eps=1e-8):
    L.call("onng_adam_step", p.data_ptr(), g.data_ptr(), m.data_ptr(), v.data_ptr(), p.numel(),
           lr, beta1, beta2, eps, t, _stream())


def feature_transform(raw: torch.Tensor, metric: int) -> torch.Tensor:
    out = torch.empty_like(raw)
    L.call("onng_feature_transform", raw.data_ptr(), raw.shape[0], metric, out.data_ptr(),
           _stream())
    return out


def column_stats(x: torch.Tensor, w: torch.Tensor | None = None):
    """(mean, std) of the columns of x [n][cols] (f32, device), weighted by w."""
    x = x.contiguous()
    n, cols = x.shape
    mean = torch.empty(cols, dtype=torch.float32, device=x.device)
    std = torch.empty(cols, dtype=torch.float32, device=x.device)
    wp = None if w is None else w.contiguous()
    L.call("onng_column_stats", x.data_ptr(), None if wp is None else wp.data_ptr(), n, cols,
           mean.data_ptr(), std.data_ptr(), _stream())
    return mean, std


def standardize(x: torch.Tensor, mean: torch.Tensor, std: torch.Tensor) -> torch.Tensor:
    x = x.contiguous()
    out = torch.empty_like(x)
    L.call("onng_standardize", x.data_ptr(), x.shape[0], x.shape[1], mean.data_ptr(),
           std.data_ptr(), out.data_ptr(), _stream())
    return out


def mlp_fold_output(W2: torch.Tensor, b2: torch.Tensor, scale: torch.Tensor,
                    shift: torch.Tensor) -> None:
    """In place: the output layer of a network trained on (y - shift) / scale
    becomes the same network on y."""
    L.call("onng_mlp_fold_output", W2.data_ptr(), b2.data_ptr(), W2.shape[0], W2.shape[1],
           scale.data_ptr(), shift.data_ptr(), _stream())


def degree_loss_from_samples(p, c) -> float:
    """Equation 2's L from (precision, distance computations) samples (host)."""
    pa = np.ascontiguousarray(p, dtype=np.float64)
    ca = np.ascontiguousarray(c, dtype=np.float64)
    out = C.c_double(0.0)
    L.call("onng_degree_loss", pa.ctypes.data, ca.ctypes.data, len(pa), C.byref(out))
    return out.value


def to_bf16_bits(w: torch.Tensor) -> torch.Tensor:
    """f32 weights -> bf16 bit patterns (round to nearest even) via onng_encode."""
    flat = w.reshape(1, -1).contiguous().to(torch.float32)
    v = encode(flat, L.BF16, L.L2SQ, pitch=row_pitch(flat.shape[1], L.BF16))
    return v.data.view(torch.int16)[0, :flat.shape[1]].contiguous().view(w.shape)


# --------------------------------------------------------------- pipeline --

class Pipeline:
    """Seeding (nearest pivots) + search (+ predictor, + rerank) captured once
    into a HIP graph and replayed."""

    def __init__(self, base: Vectors, graph: Graph, queries: Vectors, pivots: torch.Tensor,
                 n_seeds: int, seed_base: Vectors | None = None, **kw):
        dev = queries.data.device
        self.seeds = torch.empty((queries.n, n_seeds), dtype=torch.int32, device=dev)
        self.req = SearchRequest(base, graph, queries, self.seeds, **kw)
        self.pivots = pivots.contiguous()
        n_bytes = L.load().onng_pipeline_workspace_size(base.ref, queries.ref,
                                                        self.pivots.numel(), n_seeds,
                                                        C.byref(self.req.params))
        if n_bytes == 0:
            raise L.OnngError("onng_pipeline_workspace_size", L.ERR_INVALID_ARG,
                              L.load().onng_last_error().decode())
        self.ws = _workspace(n_bytes, dev)
        self.stream = torch.cuda.Stream(device=dev)
        self.handle = C.c_void_p()
        torch.cuda.synchronize()
        L.call("onng_pipeline_create", base.ref, C.byref(self.req.gs), queries.ref,
               self.pivots.data_ptr(), self.pivots.numel(), n_seeds, self.seeds.data_ptr(),
               C.byref(self.req.params), self.req.ids.data_ptr(), self.req.dists.data_ptr(),
               self.req.stats.data_ptr(), self.ws.data_ptr(), self.ws.numel(),
               self.stream.cuda_stream, C.byref(self.handle))

    def launch(self):
        L.call("onng_pipeline_launch", self.handle, _stream())
        return self.req

    def close(self):
        if self.handle:
            L.load().onng_pipeline_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
