"""ConstructANNG (Appendix, Algorithm 9) in batches on the GPU.

Algorithm 9 inserts objects one at a time: each new object o gets as edges
the k_c results of KnnSearch on the graph built so far (range eps_c, no
explored-edge limit), and every result n gets the reverse edge n -> o.  Here
objects are inserted in batches, in the order `order`:

* the first object starts the graph alone;
* each later batch, as large as everything inserted so far (at most
  `max_batch`), searches the graph of the earlier batches in parallel; its
  objects do not see each other.  With batches of one object this is the
  paper's sequential loop.

A new object never has an edge yet, so no edge is ever inserted twice, as in
the paper.  The seeds of a batch's objects are their n_seeds nearest among
the first n_pivots inserted objects (all of them while fewer are in).  Every step runs in the library's kernels (top-k, search, edge
insertion); this module only sequences the calls and gathers ids.
"""
from __future__ import annotations

import torch

from . import _lib as L
from . import api as A


def schedule(n: int, max_batch: int):
    """Batches as [start, end) positions of the insertion order."""
    out = [(0, min(1, n))]
    done = out[0][1]
    while done < n:
        b = min(done, max_batch, n - done)
        out.append((done, done + b))
        done += b
    return out


def build_anng(rows: torch.Tensor, metric: int, order: torch.Tensor, k_c: int, eps_c: float,
               n_seeds: int = 8, n_pivots: int = 1024, max_batch: int = 65536,
               base: A.Vectors | None = None) -> A.Graph:
    """rows: the base rows as a [n, dim] u8 or f32 device tensor (`base`, if
    given, is the same rows as library vectors, e.g. with a wider pitch)."""
    dev = rows.device
    n = rows.shape[0]
    base = base if base is not None else A.Vectors.from_tensor(rows, metric)
    dtype = base.dtype
    dist_t = base.dist_dtype
    order = order.to(torch.int32).contiguous()
    g = A.Graph(torch.zeros(n + 1, dtype=torch.int64, device=dev),
                torch.empty(0, dtype=torch.int32, device=dev),
                torch.empty(0, dtype=dist_t, device=dev))
    for a, b in schedule(n, max_batch)[1:]:
        ids = order[a:b].contiguous()
        qv = A.Vectors.from_tensor(A.gather_rows(rows, ids), metric)
        piv = order[:min(a, n_pivots)].contiguous()
        seeds, _ = A.topk(qv, base, n_seeds, cand=piv)
        req = A.search(base, g, qv, seeds, k=k_c, eps=eps_c)
        dst = req.ids[:, :k_c]
        src = ids[:, None].expand_as(dst)
        g = _link(g, src, dst, req.dists[:, :k_c].to(dist_t), dtype, metric)
    return g


def _link(g, src, dst, d, dtype, metric):
    """o -> n and n -> o for every (o, n) pair, both with length d."""
    s = torch.cat([src.reshape(-1), dst.reshape(-1)]).to(torch.int32).contiguous()
    t = torch.cat([dst.reshape(-1), src.reshape(-1)]).to(torch.int32).contiguous()
    ln = torch.cat([d.reshape(-1), d.reshape(-1)]).contiguous()
    # a padded result (-1) drops both directions: the library skips ids outside [0, n)
    return A.graph_add_edges(g, s, t, ln, dtype, metric)
