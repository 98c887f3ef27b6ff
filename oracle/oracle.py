"""NumPy-facing wrapper of the plain C oracle (onng_oracle.c) plus the oracle's
own small helpers (search-range factor, e_p of dynamic degree adjustment,
recall, predictor features, label generation).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
benchmark's CPU-baseline leg.  Nothing in the product package imports it.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libonng_oracle.so")

U8, F32, F16, BF16, FP8 = 0, 1, 2, 3, 4
L2SQ, COS = 0, 1
NFEAT = 14
INF_EP = 0xFFFFFFFF


class _Vecs(C.Structure):
    _fields_ = [("data", C.c_void_p), ("scale", C.c_void_p), ("n", C.c_int64),
                ("dim", C.c_int32), ("pitch", C.c_int64), ("dtype", C.c_int32),
                ("metric", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build_oracle  # noqa: F401  (package-relative when imported as oracle.oracle)
            build_oracle.build()
        _lib = C.CDLL(LIB_PATH)
        P = C.c_void_p
        _lib.or_decode.restype = C.c_double
        _lib.or_decode.argtypes = [C.c_int32, C.c_uint32]
        for nm in ("or_encode_f16", "or_encode_bf16", "or_encode_fp8"):
            getattr(_lib, nm).restype = C.c_uint32
            getattr(_lib, nm).argtypes = [C.c_float]
        _lib.or_encode_rows.argtypes = [P, C.c_int64, C.c_int32, C.c_int32, P, C.c_int64, P]
        _lib.or_dist.restype = C.c_double
        _lib.or_dist.argtypes = [P, C.c_int64, P, C.c_int64]
        _lib.or_topk.argtypes = [P, P, C.c_int64, P, P, C.c_int64, C.c_int32, C.c_int32, P, P,
                                 C.c_int32]
        _lib.or_adjust_degree.argtypes = [P, P, C.c_int64, C.c_int32, C.c_int32, C.c_int32, P,
                                          P, P, C.c_int64, P]
        _lib.or_adjust_degree_constrained.argtypes = [P, P, C.c_int64, C.c_int32, C.c_int32,
                                                      C.c_int32, P, P, P, C.c_int64, P]
        _lib.or_adjust_path.argtypes = [P, P, P, C.c_int64, P, P, P, P]
        _lib.or_vptree_build.argtypes = [P, P, C.c_int32, C.c_int32, P, P, P, P, P, P]
        _lib.or_vptree_seeds.argtypes = [P, P, C.c_int64, P, P, P, P, C.c_int32, P, P]
        _lib.or_search.argtypes = [P, P, P, C.c_int64, P, C.c_int64, P, C.c_int32, P, P, P, P,
                                   P, C.c_int32, P, C.c_int32, P, P, P, P, P, P, C.c_int32, P, P,
                                   P, C.c_int32, C.c_int32]
        _lib.or_hash_size.restype = C.c_int64
        _lib.or_hash_size.argtypes = [C.c_int64, C.c_int32]
        _lib.or_visited_replay.argtypes = [C.c_int64, P, C.c_int64, P]
        _lib.or_rerank.argtypes = [P, P, P, C.c_int32, C.c_int64, C.c_int32, P, P]
        _lib.or_mlp_forward.argtypes = [P, C.c_int32, C.c_int32, P, P, C.c_int32, P, P,
                                        C.c_int32, P, P]
        _lib.or_mlp_loss_grad.restype = C.c_double
        _lib.or_mlp_loss_grad.argtypes = [P, P, P, C.c_int32, C.c_int32, P, P, C.c_int32, P, P,
                                          C.c_int32, P, P, P, P]
        _lib.or_adam_step.argtypes = [P, P, P, P, C.c_int64, C.c_double, C.c_double,
                                      C.c_double, C.c_double, C.c_int32]
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def nthreads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


class Vectors:
    """Rows as stored (u8 / f32 / f16 / bf16 / fp8 codes) plus the metric."""

    def __init__(self, data: np.ndarray, dtype: int, metric: int, dim: int | None = None,
                 scale: np.ndarray | None = None):
        data = np.ascontiguousarray(data)
        self.data = data
        self.dtype = dtype
        self.metric = metric
        esz = {U8: 1, F32: 4, F16: 2, BF16: 2, FP8: 1}[dtype]
        self.pitch = data.shape[1] * data.dtype.itemsize
        self.dim = dim if dim is not None else self.pitch // esz
        self.n = data.shape[0]
        self.scale = None if scale is None else np.ascontiguousarray(scale, dtype=np.float32)
        self._s = _Vecs(data.ctypes.data, _ptr(self.scale), self.n, self.dim, self.pitch, dtype,
                        metric)

    @property
    def ref(self):
        return C.byref(self._s)

    @staticmethod
    def from_array(x: np.ndarray, metric: int) -> "Vectors":
        if x.dtype == np.uint8:
            return Vectors(x, U8, metric)
        return Vectors(np.ascontiguousarray(x, dtype=np.float32), F32, metric)


# ---------------------------------------------------------------- codecs --

def decode(dtype: int, code: int) -> float:
    return lib().or_decode(dtype, code)


def encode_scalar(dtype: int, x: float) -> int:
    fn = {F16: lib().or_encode_f16, BF16: lib().or_encode_bf16, FP8: lib().or_encode_fp8}[dtype]
    return fn(float(x))


def encode_rows(x: np.ndarray, dtype: int, pitch: int | None = None):
    """fp32 rows -> stored rows of `dtype` (uint8 view, `pitch` bytes), fp8 scales."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    n, dim = x.shape
    esz = {F32: 4, F16: 2, BF16: 2, FP8: 1}[dtype]
    pitch = dim * esz if pitch is None else pitch
    out = np.zeros((n, pitch), dtype=np.uint8)
    scale = np.zeros(n, dtype=np.float32) if dtype == FP8 else None
    rc = lib().or_encode_rows(x.ctypes.data, n, dim, dtype, out.ctypes.data, pitch, _ptr(scale))
    assert rc == 0
    return out, scale


# --------------------------------------------------------------- top-k ----

def topk(Q: Vectors, B: Vectors, k: int, q_rows=None, cand=None, exclude_self=False,
         threads: int | None = None):
    nq = Q.n if q_rows is None else len(q_rows)
    qr = None if q_rows is None else np.ascontiguousarray(q_rows, dtype=np.int64)
    cd = None if cand is None else np.ascontiguousarray(cand, dtype=np.int32)
    ids = np.empty((nq, k), dtype=np.int32)
    ds = np.empty((nq, k), dtype=np.float64)
    rc = lib().or_topk(Q.ref, _ptr(qr), nq, B.ref, _ptr(cd), 0 if cd is None else len(cd), k,
                       int(exclude_self), ids.ctypes.data, ds.ctypes.data,
                       threads or nthreads())
    assert rc == 0
    return ids, ds


def knn_graph(B: Vectors, k: int, rows=None, threads=None):
    """Exact kNN of base rows among the base, self excluded by index."""
    return topk(B, B, k, q_rows=rows, exclude_self=True, threads=threads)


# ----------------------------------------------------- graph adjustment ---

def adjust_degree(knn_ids, knn_d, e_o: int, e_i: int):
    knn_ids = np.ascontiguousarray(knn_ids, dtype=np.int32)
    knn_d = np.ascontiguousarray(knn_d, dtype=np.float64)
    n, k = knn_ids.shape
    nnz = C.c_int64(0)
    rc = lib().or_adjust_degree(knn_ids.ctypes.data, knn_d.ctypes.data, n, k, e_o, e_i, None,
                                None, None, 0, C.byref(nnz))
    assert rc == 0
    off = np.empty(n + 1, dtype=np.int64)
    nb = np.empty(max(1, nnz.value), dtype=np.int32)
    ln = np.empty(max(1, nnz.value), dtype=np.float64)
    rc = lib().or_adjust_degree(knn_ids.ctypes.data, knn_d.ctypes.data, n, k, e_o, e_i,
                                off.ctypes.data, nb.ctypes.data, ln.ctypes.data, nnz.value,
                                C.byref(nnz))
    assert rc == 0
    return off, nb[:nnz.value], ln[:nnz.value]


def adjust_degree_constrained(knn_ids, knn_d, e_o: int, e_i: int):
    """Algorithm 3 (static degree adjustment with constraints) on a k-NN table
    whose rows are sorted by (d, id).  Returns CSR (offsets, nbrs, lens), each
    list in (len, id) order."""
    knn_ids = np.ascontiguousarray(knn_ids, dtype=np.int32)
    knn_d = np.ascontiguousarray(knn_d, dtype=np.float64)
    n, k = knn_ids.shape
    nnz = C.c_int64(0)
    rc = lib().or_adjust_degree_constrained(knn_ids.ctypes.data, knn_d.ctypes.data, n, k, e_o,
                                            e_i, None, None, None, 0, C.byref(nnz))
    assert rc == 0
    off = np.empty(n + 1, dtype=np.int64)
    nb = np.empty(max(1, nnz.value), dtype=np.int32)
    ln = np.empty(max(1, nnz.value), dtype=np.float64)
    rc = lib().or_adjust_degree_constrained(knn_ids.ctypes.data, knn_d.ctypes.data, n, k, e_o,
                                            e_i, off.ctypes.data, nb.ctypes.data,
                                            ln.ctypes.data, nnz.value, C.byref(nnz))
    assert rc == 0
    return off, nb[:nnz.value], ln[:nnz.value]


def adjust_path(off, nbrs, lens):
    off = np.ascontiguousarray(off, dtype=np.int64)
    nbrs = np.ascontiguousarray(nbrs, dtype=np.int32)
    lens = np.ascontiguousarray(lens, dtype=np.float64)
    n = len(off) - 1
    nnz = C.c_int64(0)
    oo = np.empty(n + 1, dtype=np.int64)
    on = np.empty(max(1, len(nbrs)), dtype=np.int32)
    ol = np.empty(max(1, len(nbrs)), dtype=np.float64)
    rc = lib().or_adjust_path(off.ctypes.data, nbrs.ctypes.data, lens.ctypes.data, n,
                              oo.ctypes.data, on.ctypes.data, ol.ctypes.data, C.byref(nnz))
    assert rc == 0
    return oo, on[:nnz.value], ol[:nnz.value]


# ------------------------------------------------------ graph statistics --

def graph_stats(off, nbrs, lens, metric: int, frac: float = 0.05, keep: int = 10):
    """Table 4's graph statistics, from their definitions in Section 3.2:
    mean out-degree of the t nodes of largest out-degree, mean in-degree of
    the t nodes of smallest in-degree (t = max(1, floor(frac * n))), and the
    mean edge length of the transposed graph cut to each node's `keep`
    shortest incoming edges.  A squared-L2 length counts as its square root
    (the Euclidean distance the paper reports); a cosine length as is."""
    off = np.asarray(off, dtype=np.int64)
    nbrs = np.asarray(nbrs, dtype=np.int64)
    lens = np.asarray(lens, dtype=np.float64)
    n = len(off) - 1
    if n == 0:
        return 0.0, 0.0, 0.0
    t = max(1, int(math.floor(frac * n)))
    outdeg = np.diff(off)
    indeg = np.bincount(nbrs, minlength=n)
    top = float(np.sort(outdeg)[::-1][:t].sum()) / t
    bottom = float(np.sort(indeg)[:t].sum()) / t
    incoming = [[] for _ in range(n)]
    for v in range(n):
        for e in range(off[v], off[v + 1]):
            incoming[nbrs[e]].append(lens[e])
    kept = []
    for lst in incoming:
        kept.extend(sorted(lst)[:keep])
    kept = np.array(kept, dtype=np.float64)
    if metric == L2SQ:
        kept = np.sqrt(kept)
    return top, bottom, float(kept.mean()) if len(kept) else 0.0


# ----------------------------------------- degree-parameter optimisation --

def degree_loss(search, p_l=0.90, p_u=0.98, eps_max=1.0, iters=30, samples=10):
    """Equation 2 measured from searches (Section 2.6): search(eps) gives
    (mean precision, mean distance computations).  The upper range is the
    binary-search midpoint whose precision first falls in [p_u, p_u + 0.005),
    the lower one the first in (p_l - 0.005, p_l] searched below it (0 when
    the smallest range already exceeds p_l); ten evenly spaced ranges between
    them give (p, C); the trapezoidal rule integrates log10 C over their
    precision span, divided by that span.  Returns (L, [(eps, p, C)]), L = inf
    when p_u is not reached."""
    def bracket_search(target, up, lo, hi):
        if not up and search(lo)[0] > target:
            return lo
        if search(hi)[0] < target:
            return None
        for _ in range(iters):
            mid = (lo + hi) / 2
            p = search(mid)[0]
            inside = (target <= p < target + 0.005) if up else (target - 0.005 < p <= target)
            if inside:
                return mid
            too_low = p < target if up else p <= target - 0.005
            if too_low:
                lo = mid
            else:
                hi = mid
        return hi if up else lo

    eu = bracket_search(p_u, True, 0.0, eps_max)
    if eu is None:
        return math.inf, []
    el = bracket_search(p_l, False, 0.0, eu)
    eps = [el + (eu - el) * i / (samples - 1) for i in range(samples)]
    pts = [(e,) + tuple(search(e)) for e in eps]
    p = np.array([t[1] for t in pts])
    y = np.log10(np.array([t[2] for t in pts], dtype=np.float64))
    o = np.argsort(p, kind="stable")
    p, y = p[o], y[o]
    if p[-1] == p[0]:
        return float(y.mean()), pts
    area = float(np.sum((p[1:] - p[:-1]) * (y[1:] + y[:-1]) / 2))
    return area / float(p[-1] - p[0]), pts


# ------------------------------------------- ANNG construction (Alg 9) --

def anng(x: np.ndarray, metric: int, order, k_c: int, eps_c: float, n_seeds: int = 8,
         n_pivots: int = 1024, max_batch: int = 65536):
    """Algorithm 9 with batched insertion: the first object of `order` starts
    alone; each later batch (as large as everything inserted so far, at most
    max_batch) runs KnnSearch(G_a, o, k_c, eps_c, inf) on the graph of the
    earlier batches, seeded by each object's n_seeds nearest among the first
    n_pivots inserted objects, and adds o -> n and n -> o for every result n.
    Returns CSR lists sorted by (length, id)."""
    n = len(x)
    order = np.asarray(order, dtype=np.int64)
    B = Vectors.from_array(x, metric)
    adj = [[] for _ in range(n)]

    def csr():
        lists = [sorted(a) for a in adj]
        off = np.zeros(n + 1, np.int64)
        off[1:] = np.cumsum([len(a) for a in lists])
        nb = np.array([i for a in lists for _, i in a], dtype=np.int32)
        ln = np.array([l for a in lists for l, _ in a], dtype=np.float64)
        return off, nb, ln

    done = min(1, n)
    while done < n:
        b = min(done, max_batch, n - done)
        ids = order[done:done + b]
        off, nb, _ = csr()
        Q = Vectors.from_array(x[ids], metric)
        piv = order[:min(done, n_pivots)].astype(np.int32)
        seeds, _ = topk(Q, B, n_seeds, cand=piv)
        r = search(B, off, nb, Q, seeds, k_c, eps_c)
        for t, o in enumerate(ids):
            for nn, d in zip(r["ids"][t, :k_c], r["dists"][t, :k_c]):
                if nn >= 0:
                    adj[int(o)].append((float(d), int(nn)))
                    adj[int(nn)].append((float(d), int(o)))
        done += b
    return csr()


def aknng(off, nbrs, lens, k_c: int):
    """The first step of ConstructGraph (Algorithm 8, Section 2.6):
    G_k = ConstructAdjustedGraph(G_a, k_c, 0), i.e. Algorithm 2 with e_i = 0
    run on the graph G_a (an ANNG), each node's list being the S of
    Algorithm 2.  Returns G_k as the padded table it feeds the degree
    adjustments: ids [n][k_c] (-1 padding) and dists [n][k_c] (+inf)."""
    off = np.asarray(off, np.int64)
    n = len(off) - 1
    deg = np.diff(off)
    width = max(1, int(deg.max()) if n else 1)
    ids = np.full((n, width), -1, np.int32)
    dd = np.full((n, width), np.inf)
    for v in range(n):
        ids[v, :deg[v]] = nbrs[off[v]:off[v + 1]]
        dd[v, :deg[v]] = lens[off[v]:off[v + 1]]
    go, gn, gl = adjust_degree(ids, dd, k_c, 0)
    out_i = np.full((n, k_c), -1, np.int32)
    out_d = np.full((n, k_c), np.inf)
    for v in range(n):
        m = go[v + 1] - go[v]
        out_i[v, :m] = gn[go[v]:go[v + 1]]
        out_d[v, :m] = gl[go[v]:go[v + 1]]
    return out_i, out_d


# ------------------------------------------------- tree-based seeds ------

def vptree_build(B: Vectors, prio, leaf_size: int = 100, n_seeds: int = 10):
    """The 4-way vantage-point tree of the base rows (Section 3.2, Table 5);
    see or_vptree_build.  Returns a dict of numpy arrays."""
    n = B.n
    prio = np.ascontiguousarray(prio, dtype=np.uint32)
    vp = np.empty(n, np.int32)
    child = np.empty(n, np.int32)
    mu = np.zeros(3 * n, np.float64)
    seeds = np.empty(n * n_seeds, np.int32)
    nn, nl = C.c_int64(0), C.c_int64(0)
    rc = lib().or_vptree_build(B.ref, prio.ctypes.data, leaf_size, n_seeds, vp.ctypes.data,
                               child.ctypes.data, mu.ctypes.data, seeds.ctypes.data, C.byref(nn),
                               C.byref(nl))
    assert rc == 0
    m, l = nn.value, nl.value
    return dict(vp=vp[:m], child=child[:m], mu=mu[:3 * m].reshape(m, 3),
                seeds=seeds[:l * n_seeds].reshape(l, n_seeds), n_seeds=n_seeds)


def vptree_seeds(B: Vectors, Q: Vectors, tree):
    """Descent of every query: (seeds [nq][n_seeds], distance computations [nq])."""
    ns = tree["n_seeds"]
    out = np.empty((Q.n, ns), np.int32)
    dc = np.empty(Q.n, np.int32)
    vp = np.ascontiguousarray(tree["vp"])
    child = np.ascontiguousarray(tree["child"])
    mu = np.ascontiguousarray(tree["mu"], dtype=np.float64)
    sd = np.ascontiguousarray(tree["seeds"])
    rc = lib().or_vptree_seeds(B.ref, Q.ref, Q.n, vp.ctypes.data, child.ctypes.data,
                               mu.ctypes.data, sd.ctypes.data, ns, out.ctypes.data, dc.ctypes.data)
    assert rc == 0
    return out, dc


# ---------------------------------------------------------------- search --

def range_factor(eps: float, metric: int) -> np.float32:
    """Reading R5: fp32((1+eps)^2) on squared L2, fp32(1+eps) on cosine."""
    t = 1.0 + float(np.float32(eps))
    return np.float32(t * t if metric == L2SQ else t)


def dynamic_ep(eps: float, e0: float = 30.0, we: float = 20.0) -> int:
    """Equation 1, e_p = 10^(w_e eps) + e_0, floored to an edge count."""
    v = math.floor(10.0 ** (we * float(np.float32(eps))) + e0)
    return int(min(v, INF_EP))


def _per_query(v, nq, dtype):
    a = np.asarray(v, dtype=dtype)
    if a.ndim == 0:
        a = np.full(nq, a, dtype=dtype)
    return np.ascontiguousarray(a)


def search(base: Vectors, off, nbrs, queries: Vectors, seeds, k, eps, ep=INF_EP, eps1=None,
           ep1=None, k_stride=None, want_features=False, threads=None, probe_hops=1,
           max_dc=None, pool_k=0, probe_only=False):
    """Algorithm 1 for every query.  Returns dict with ids, dists, dc, hops,
    margin[, feat][, pool_ids, pool_d, pool_margin].  pool_k > 0: the pool_k
    smallest (d, id) over all distances computed (the candidates a rerank
    of low-precision rows takes).  probe_only (with eps1/ep1): stop at the
    switch after the probe expansions, like a pass that only predicts."""
    nq = queries.n
    seeds = np.ascontiguousarray(seeds, dtype=np.int32)
    kk = _per_query(k, nq, np.int32)
    ee = _per_query(eps, nq, np.float32)
    pp = _per_query(ep, nq, np.uint32)
    e1 = None if eps1 is None else _per_query(eps1, nq, np.float32)
    p1 = None if ep1 is None else _per_query(ep1, nq, np.uint32)
    md = None if max_dc is None else _per_query(max_dc, nq, np.int32)
    ks = int(kk.max()) if k_stride is None else k_stride
    off = np.ascontiguousarray(off, dtype=np.int64)
    nbrs = np.ascontiguousarray(nbrs, dtype=np.int32)
    ids = np.empty((nq, ks), dtype=np.int32)
    ds = np.empty((nq, ks), dtype=np.float64)
    dc = np.empty(nq, dtype=np.int64)
    hops = np.empty(nq, dtype=np.int64)
    margin = np.empty(nq, dtype=np.float64)
    feat = np.zeros((nq, NFEAT), dtype=np.float64) if want_features else None
    pid = np.empty((nq, max(pool_k, 1)), dtype=np.int32)
    pd = np.empty((nq, max(pool_k, 1)), dtype=np.float64)
    pm = np.empty(nq, dtype=np.float64)
    rc = lib().or_search(base.ref, off.ctypes.data, nbrs.ctypes.data, base.n, queries.ref, nq,
                         seeds.ctypes.data, seeds.shape[1], kk.ctypes.data, ee.ctypes.data,
                         pp.ctypes.data, _ptr(e1), _ptr(p1), probe_hops, _ptr(md), ks,
                         ids.ctypes.data,
                         ds.ctypes.data, dc.ctypes.data, hops.ctypes.data, margin.ctypes.data,
                         _ptr(feat), int(pool_k), pid.ctypes.data, pd.ctypes.data,
                         pm.ctypes.data, int(bool(probe_only)), threads or nthreads())
    assert rc == 0, rc
    out = dict(ids=ids, dists=ds, dc=dc, hops=hops, margin=margin)
    if want_features:
        out["feat"] = feat
    if pool_k > 0:
        out.update(pool_ids=pid, pool_d=pd, pool_margin=pm)
    return out


def hash_size(n: int, b: int = 11) -> int:
    return int(lib().or_hash_size(n, b))


def visited_replay(n: int, ops) -> np.ndarray:
    ops = np.ascontiguousarray(ops, dtype=np.int64)
    ans = np.empty(int((ops < 0).sum()), dtype=np.int32)
    rc = lib().or_visited_replay(n, ops.ctypes.data, len(ops), ans.ctypes.data)
    assert rc == 0
    return ans


def rerank(Q: Vectors, B: Vectors, pool, k: int):
    pool = np.ascontiguousarray(pool, dtype=np.int32)
    nq, psz = pool.shape
    ids = np.empty((nq, k), dtype=np.int32)
    ds = np.empty((nq, k), dtype=np.float64)
    rc = lib().or_rerank(Q.ref, B.ref, pool.ctypes.data, psz, nq, k, ids.ctypes.data,
                         ds.ctypes.data)
    assert rc == 0
    return ids, ds


# ---------------------------------------------------------------- recall --

def recall_at_k(res_ids, res_d, gt_d, k: int) -> np.ndarray:
    """Tie-tolerant recall@k: |{x in R : d(x,q) <= d_k^GT(q)}| / k, per query.

    The paper's precision is the fraction of returned objects that are true
    k nearest neighbours; with |R| = k that is recall@k.  Objects tied with
    the k-th true distance count as correct."""
    res_ids = np.asarray(res_ids)[:, :k]
    res_d = np.asarray(res_d, dtype=np.float64)[:, :k]
    kth = np.asarray(gt_d, dtype=np.float64)[:, k - 1:k]
    ok = (res_ids >= 0) & (res_d <= kth)
    return ok.sum(axis=1) / float(k)


# --------------------------------------------------- learned search range --

def feature_transform(feat: np.ndarray, metric: int) -> np.ndarray:
    """Raw first-expansion state -> predictor inputs (before z-scoring).

    Distances enter as log(d + c) with c = 1 for squared L2 on u8 data scale
    and c = 1e-3 on cosine; the 7 further seed distances as differences of
    those logs to the nearest seed; counts as log(1 + n)."""
    feat = np.asarray(feat, dtype=np.float64)
    c = 1e-3 if metric == COS else 1.0
    x = np.empty_like(feat)
    lg = np.log(np.maximum(feat[:, :8], 0.0) + c)
    x[:, 0] = lg[:, 0]
    x[:, 1:8] = lg[:, 1:8] - lg[:, :1]
    x[:, 8] = np.log1p(feat[:, 8])
    for j in (9, 10, 11, 12):
        x[:, j] = np.log(np.maximum(feat[:, j], 0.0) + c) - lg[:, 0]
    x[:, 13] = np.log1p(feat[:, 13])
    return x


_BF16_TABLE = None


def decode_bf16(bits) -> np.ndarray:
    """bfloat16 codes (uint16) -> exact fp64 values, through the oracle's codec."""
    global _BF16_TABLE
    if _BF16_TABLE is None:
        _BF16_TABLE = np.array([decode(BF16, c) for c in range(1 << 16)], dtype=np.float64)
    return _BF16_TABLE[np.asarray(bits, dtype=np.int64) & 0xFFFF]


def predict(feat, metric: int, w1_bits, b1, w2_bits, b2, mean, std, mode: str, *,
            head=0, head_per_query=None, shift=None, eps_cand=None, lam=0.0,
            lam_per_query=None, eps_min=0.0, eps_max=math.inf, e0=30.0, we=-1.0,
            ep_default=INF_EP):
    """The learned search range of every query (an extension, not in the
    paper), composed from its definition: raw state after the probe
    expansions -> feature_transform -> z-score with the stored statistics ->
    2-layer MLP in fp64 on the bf16-decoded weights -> choice.

    mode "curve": heads [0, G) estimate the recall and [G, 2G) log(1 + cost)
    at each candidate range eps_cand[g]; the query takes the first g of the
    largest recall_g - lambda * (exp(cost head) - 1) and that candidate's
    cost estimate.  mode "log_eps": head h (head_per_query[q] or `head`)
    gives log10(eps + 0.01) after adding shift[h]; cost = eps.  eps is
    clamped to [eps_min, eps_max]; e_p follows Equation 1 with (e0, we)
    when we >= 0, else ep_default.

    Returns dict eps (fp64), ep (int64), cost (fp64), margin: the relative
    gap of the decision (curve: best vs second score over max(1, |best|);
    log_eps: inf) and ep_margin: distance of 10^(we eps) + e0 to the next
    integer boundary, relative to its value (inf when we < 0)."""
    feat = np.asarray(feat, dtype=np.float64)
    nq = feat.shape[0]
    x = feature_transform(feat, metric)
    z = (x - np.asarray(mean, np.float32).astype(np.float64)) / \
        np.asarray(std, np.float32).astype(np.float64)
    b1 = np.asarray(b1, np.float32).astype(np.float64)
    b2 = np.asarray(b2, np.float32).astype(np.float64)
    H, T = len(b1), len(b2)
    W1 = decode_bf16(w1_bits).reshape(H, -1)
    W2 = decode_bf16(w2_bits).reshape(T, H)
    _, y = mlp_forward(z, W1, b1, W2, b2)
    margin = np.full(nq, np.inf)
    if mode == "curve":
        cand = np.asarray(eps_cand, np.float32).astype(np.float64)
        G = len(cand)
        lq = (np.full(nq, np.float32(lam), np.float64) if lam_per_query is None
              else np.asarray(lam_per_query, np.float32).astype(np.float64))
        score = y[:, :G] - lq[:, None] * (np.exp(y[:, G:2 * G]) - 1.0)
        best = np.argmax(score, axis=1)
        eps = cand[best]
        cost = np.exp(y[np.arange(nq), G + best]) - 1.0
        if G > 1:
            srt = np.sort(score, axis=1)
            margin = (srt[:, -1] - srt[:, -2]) / np.maximum(1.0, np.abs(srt[:, -1]))
    elif mode == "log_eps":
        h = (np.full(nq, int(head)) if head_per_query is None
             else np.asarray(head_per_query, np.int64))
        sh = np.zeros(T) if shift is None else np.asarray(shift, np.float32).astype(np.float64)
        yh = y[np.arange(nq), h] + sh[h]
        eps = 10.0 ** yh - 0.01
        cost = eps.copy()
    else:
        raise ValueError(mode)
    eps = np.clip(eps, float(np.float32(eps_min)), float(np.float32(eps_max)))
    if mode == "log_eps":
        cost = eps.copy()
    if we >= 0:
        v = 10.0 ** (float(np.float32(we)) * eps) + float(np.float32(e0))
        ep = np.minimum(np.floor(v), float(INF_EP)).astype(np.int64)
        frac = v - np.floor(v)
        ep_margin = np.minimum(frac, 1.0 - frac) / np.maximum(v, 1.0)
        ep_margin[eps == 0.0] = np.inf        # 10^0 + e0 is exact in any precision
    else:
        ep = np.full(nq, int(ep_default), np.int64)
        ep_margin = np.full(nq, np.inf)
    return dict(eps=eps, ep=ep, cost=cost, margin=margin, ep_margin=ep_margin, y=y)


def labels_from_sweep(recalls: np.ndarray, eps_grid, targets) -> np.ndarray:
    """label[q, t] = smallest grid eps whose per-query recall reaches targets[t]
    (the largest grid eps when none does).  recalls: (n_eps, nq)."""
    recalls = np.asarray(recalls)
    grid = np.asarray(eps_grid, dtype=np.float64)
    out = np.empty((recalls.shape[1], len(targets)), dtype=np.float64)
    for t, tgt in enumerate(targets):
        ok = recalls >= tgt - 1e-12
        first = np.where(ok.any(axis=0), ok.argmax(axis=0), len(grid) - 1)
        out[:, t] = grid[first]
    return out


# ------------------------------------------------------------------ MLP ---

def mlp_forward(X, W1, b1, W2, b2):
    X = np.ascontiguousarray(X, dtype=np.float64)
    B, F = X.shape
    H = W1.shape[0]
    T = W2.shape[0]
    hid = np.empty((B, H))
    Y = np.empty((B, T))
    args = [np.ascontiguousarray(a, dtype=np.float64) for a in (W1, b1, W2, b2)]
    rc = lib().or_mlp_forward(X.ctypes.data, B, F, args[0].ctypes.data, args[1].ctypes.data, H,
                              args[2].ctypes.data, args[3].ctypes.data, T, hid.ctypes.data,
                              Y.ctypes.data)
    assert rc == 0
    return hid, Y


def mlp_loss_grad(X, target, W1, b1, W2, b2, w=None):
    X = np.ascontiguousarray(X, dtype=np.float64)
    target = np.ascontiguousarray(target, dtype=np.float64)
    B, F = X.shape
    H = W1.shape[0]
    T = W2.shape[0]
    W1, b1, W2, b2 = [np.ascontiguousarray(a, dtype=np.float64) for a in (W1, b1, W2, b2)]
    wt = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
    g = [np.empty_like(a) for a in (W1, b1, W2, b2)]
    loss = lib().or_mlp_loss_grad(X.ctypes.data, target.ctypes.data, _ptr(wt), B, F,
                                  W1.ctypes.data, b1.ctypes.data, H, W2.ctypes.data,
                                  b2.ctypes.data, T, *[a.ctypes.data for a in g])
    return loss, g


def adam_step(p, g, m, v, lr, t, beta1=0.9, beta2=0.999, eps=1e-8):
    for a in (p, g, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    lib().or_adam_step(p.ctypes.data, g.ctypes.data, m.ctypes.data, v.ctypes.data, p.size, lr,
                       beta1, beta2, eps, t)
