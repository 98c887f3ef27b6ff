"""Second, independent oracle for tiny inputs, written from what each step of
the method computes rather than from the printed listings: pure Python over
dicts and lists, no heaps, no shared code with the C oracle.

TEST INFRASTRUCTURE ONLY.  Distances come in as a callable, so the same code
serves exact integer and fp64 data.  Ties are broken by node id everywhere
(reading R4), and the readings R1, R2, R5, R11 and R12 apply as in the C
oracle.

* knn_search:  KnnSearch (Algorithm 1, Section 2) stated as: keep the set V
               of nodes whose distance has been computed; repeatedly expand
               the nearest node of V not expanded yet, as long as it lies
               within r(1 + eps), r being the k-th smallest distance in V;
               an expansion computes the distances of the first e_p entries
               of the node's list that are not in V yet.  R is the k nearest
               of V.  (The candidate set of the listing only ever holds
               nodes of V; a node it rejected lies beyond every later range,
               so "nearest unexpanded node of V" is the node it pops.)
* adjusted_graph: ConstructAdjustedGraph (Algorithm 2, Section 2.1) as the
               set identity N(G_e, o) = F(o) u Rv(o).
* adjusted_graph_with_constraint: Algorithm 3 (Section 2.2) as one pass
               over its edge decisions in their stated order.
* adjust_path: AdjustPath / HasPath (Algorithms 4 and 5, Section 2.3) as one
               pass over the edge decisions in their stated order, each edge
               tested for a shorter two-hop detour among the edges kept so far.
* PaperVisited: the visited-node table of Section 2.5 (Algorithms 6 and 7).
* construct_anng: Algorithm 9 (Appendix), one object at a time.
* vptree:      the 4-way vantage-point tree of the seeds (Section 3.2,
               Table 5), built depth first and renumbered breadth first.
"""
from __future__ import annotations

import math

import numpy as np


def knn_search(neigh, dist_to_q, seeds, k, thr_fn, ep=math.inf, max_dc=0, trace=None,
               visited=None):
    """neigh[s]: the edge list of s in stored order (ascending length);
    dist_to_q(n) = d(n, q); thr_fn(r) = r(1 + eps) in the reading's
    arithmetic (R5); ep: entries scanned per expansion (Equation 1's e_p,
    counting visited entries too).  max_dc > 0: a distance-computation
    budget checked before each expansion (not in the paper).  Returns
    (R as (d, id) ascending, distance computations, expansions).
    trace (a list) receives the count after the seeds and after each
    expansion; visited (a dict) receives id -> d for every node of V."""
    V = {} if visited is None else visited
    for s in seeds:                      # R2: distinct seeds, each one computation
        if s not in V:
            V[s] = dist_to_q(s)
    expanded = set()

    def nearest(m):
        return sorted((d, i) for i, d in V.items())[:m]

    def radius():
        best = nearest(k)
        return best[-1][0] if len(best) == k else math.inf

    if trace is not None:
        trace.append(len(V))
    scan = None if math.isinf(ep) else int(ep)
    while not (max_dc > 0 and len(V) >= max_dc):
        todo = [(d, i) for i, d in V.items() if i not in expanded]
        if not todo:
            break
        d, s = min(todo)
        if d > thr_fn(radius()):
            break
        expanded.add(s)
        for n in list(neigh[s])[:scan]:
            if n not in V:
                V[n] = dist_to_q(n)
        if trace is not None:
            trace.append(len(V))
    return nearest(k), len(V), len(expanded)


def adjusted_graph(knn, knn_d, e_o, e_i):
    """G_e of Algorithm 2: o keeps F(o), the first e_o entries of its own row,
    and receives Rv(o), the nodes m whose row holds o among its first e_i
    entries (reading R1: both bounds apply, the row ends the loop).  An edge
    takes the length stored in the row it comes from; a pair present both
    ways keeps the copy Algorithm 2's node order meets first (R17): the
    reverse one when m < o.  Returns per-node lists of (len, id), ascending."""
    n = len(knn)
    row = [[(knn_d[o][t], knn[o][t]) for t in range(len(knn[o])) if knn[o][t] >= 0]
           for o in range(n)]
    fwd = [{i: d for d, i in row[o][:e_o]} for o in range(n)]
    rev = [dict() for _ in range(n)]
    for m in range(n):
        for d, o in row[m][:e_i]:
            rev[o][m] = d
    out = []
    for o in range(n):
        edges = {}
        for m in set(fwd[o]) | set(rev[o]):
            if m in rev[o] and (m not in fwd[o] or m < o):
                edges[m] = rev[o][m]
            else:
                edges[m] = fwd[o][m]
        out.append(sorted((l, i) for i, l in edges.items()))
    return out


def adjusted_graph_with_constraint(knn, knn_d, e_o, e_i):
    """G_e of Algorithm 3.  Its first loop decides the edges o -> n of G_t
    (Algorithm 2 with (0, e_i): each node's reverse edges) one by one, nodes
    by ascending (|N(G_t, o)|, o) (R10) and within a node by (len, id): an
    edge is kept when n has no incoming edge yet, or when n's in-degree is
    below e_i and o's out-degree below e_o.  The second loop tops every node
    with fewer than e_o edges up from its own row, in row order.  Returns
    per-node lists of (len, id), ascending."""
    n = len(knn)
    Gt = adjusted_graph(knn, knn_d, 0, e_i)
    node_order = sorted(range(n), key=lambda x: (len(Gt[x]), x))
    decisions = [(o, l, t) for o in node_order for l, t in Gt[o]]
    out = [[] for _ in range(n)]
    indeg = [0] * n
    for o, l, t in decisions:
        if indeg[t] == 0 or (indeg[t] < e_i and len(out[o]) < e_o):
            out[o].append((l, t))
            indeg[t] += 1
    for o in range(n):
        have = {t for _, t in out[o]}
        for j in range(len(knn[o])):
            if len(out[o]) >= e_o:
                break
            t = knn[o][j]
            if t >= 0 and t not in have:
                out[o].append((knn_d[o][j], t))
                have.add(t)
    return [sorted(lst) for lst in out]


def construct_anng(order, dist, k_c, thr_fn, n_seeds, n_pivots):
    """Algorithm 9: objects join in `order`; a new object's edges are the
    k_c results of KnnSearch (range eps_c, unlimited e_p) on the graph of the
    objects before it, and each result gets the edge back.  Seeds: the
    n_seeds objects nearest the new one among the first n_pivots inserted,
    by (d, id).  Returns per-node lists of (len, id), ascending."""
    graph = {o: [] for o in order}
    for t, o in enumerate(order):
        before = order[:t]
        found = []
        if before:
            lists = {v: [i for _, i in sorted(graph[v])] for v in before}
            seeds = sorted(before[:n_pivots], key=lambda m: (dist(o, m), m))[:n_seeds]
            found, _, _ = knn_search(lists, lambda m: dist(o, m), seeds, k_c, thr_fn)
        for d, m in found:
            graph[o].append((d, m))
            graph[m].append((d, o))
    return {o: sorted(graph[o]) for o in order}


def vptree(ids, dist, prio, leaf_size, n_seeds):
    """Recursive build over the row ids `ids` with dist(a, b) and priorities
    prio[x].  Returns (vp, child, mu, seeds) lists in breadth-first numbering,
    child[v] = first of four children or -1 - leaf."""
    def build(members):
        v = min(members, key=lambda x: (prio[x], x))
        if len(members) <= leaf_size:
            near = sorted(members, key=lambda x: (dist(v, x), x))[:n_seeds]
            return {"vp": v, "seeds": near + [-1] * (n_seeds - len(near))}
        rest = sorted((x for x in members if x != v), key=lambda x: (dist(v, x), x))
        m1 = len(rest)
        cuts = [c * m1 // 4 for c in range(5)]
        return {"vp": v, "mu": [dist(v, rest[cuts[c]]) for c in (1, 2, 3)],
                "kids": [build(rest[cuts[c]:cuts[c + 1]]) for c in range(4)]}

    root = build(list(ids))
    order, q = [], [root]
    while q:                       # breadth-first numbering
        node = q.pop(0)
        order.append(node)
        q.extend(node.get("kids", []))
    index = {id(nd): i for i, nd in enumerate(order)}
    vp, child, mu, seeds = [], [], [], []
    for nd in order:
        vp.append(nd["vp"])
        if "kids" in nd:
            child.append(index[id(nd["kids"][0])])
            mu.append(nd["mu"])
        else:
            child.append(-1 - len(seeds))
            mu.append([0.0, 0.0, 0.0])
            seeds.append(nd["seeds"])
    return vp, child, mu, seeds


def adjust_path(G):
    """G_p of Algorithms 4 and 5.  G: per-node lists of (len, id).  The
    edges are decided in the order Algorithm 4 visits them: round j takes
    the j-th shortest edge of every node that has one, nodes in ascending id
    (R11: each decision sees every earlier one).  Edge n -> t of length l is
    dropped when the kept edges already hold n -> c and c -> t with
    len(c, t) < l (HasPath, strict, R12); otherwise it is kept.  Returns
    per-node lists of (id, len) in decision order."""
    n = len(G)
    ranked = [sorted(G[v]) for v in range(n)]
    decisions = sorted((j, v) for v in range(n) for j in range(len(ranked[v])))
    kept = [[] for _ in range(n)]
    for j, v in decisions:
        l, t = ranked[v][j]
        detour = any(m == t and lm < l for c, _ in kept[v] for m, lm in kept[c])
        if not detour:
            kept[v].append((t, l))
    return kept


class PaperVisited:
    """The visited-node set of Section 2.5: s = 2^floor((log2 n + b) / 2)
    slots addressed by the low bits of the id.  A slot holds the first id
    that hashed to it; any other id of that slot goes to the slot's overflow
    set.  Membership: the slot's id, else its overflow set."""

    def __init__(self, n, b=11):
        lg = int(n).bit_length() - 1
        self.s = 1 << ((lg + b) // 2)
        self.first = [None] * self.s
        self.more = [set() for _ in range(self.s)]

    def set(self, i):
        h = i % self.s
        if self.first[h] is None:
            self.first[h] = i
        elif self.first[h] != i:
            self.more[h].add(i)

    def isset(self, i):
        h = i % self.s
        return self.first[h] == i or i in self.more[h]


def brute_topk(D: np.ndarray, k: int, exclude_diag: bool = False):
    """k smallest (d, j) per row of a dense distance matrix via a stable sort."""
    D = np.array(D, dtype=np.float64, copy=True)
    if exclude_diag:
        np.fill_diagonal(D, np.inf)
    order = np.argsort(D, axis=1, kind="stable")[:, :k]
    return order.astype(np.int32), np.take_along_axis(D, order, axis=1)
