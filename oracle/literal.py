"""Second, independent oracle for tiny inputs: pure-Python loops that follow
the paper's algorithms in their printed order, with sets and lists only.

TEST INFRASTRUCTURE ONLY.  Distances come in as a callable dist(a, b), so the
same code serves exact integer and fp64 data.  Ties are broken by node id
(reading R4), and the readings R1, R2, R5, R11 and R12 apply as in the C oracle.

* knn_search:            Algorithm 1 (KnnSearch), C a plain Python set.
* adjusted_graph:        Algorithm 2 (ConstructAdjustedGraph).
* adjusted_graph_with_constraint: Algorithm 3, with M a set and the argmin
                         over (|N(G_t, x)|, x) taken afresh every step (R10).
* adjust_path/has_path:  Algorithms 4 and 5 (AdjustPath, HasPath).
* paper_visited:         Algorithms 6 and 7 (Set, IsSet) as a class.
* construct_anng:        Algorithm 9, one object at a time.
* vptree:                the 4-way vantage-point tree of the seeds (Section
                         3.2, Table 5), built depth first and renumbered
                         breadth first afterwards.
"""
from __future__ import annotations

import math

import numpy as np


def _key(d, i):
    return (d, i)


def knn_search(neigh, dist_to_q, seeds, k, thr_fn, ep=math.inf, max_dc=0, trace=None):
    """Algorithm 1.  neigh[s] is the edge list of s sorted by length;
    dist_to_q(n) is d(n, q); thr_fn(r) returns r(1+eps) in the reading's
    arithmetic.  max_dc > 0 adds a distance-computation budget checked before
    each pop (not in the paper).  Returns (R sorted by (d, id), distance
    computations, hops).  trace, if a list, receives the distance count after
    the seeds and after every expansion."""
    C = set()
    S = []                               # list of (d, id)
    R = []                               # list of (d, id)
    r = math.inf
    dc = 0
    for s in seeds:                      # R2: seeds de-duplicated, offered to R
        if s in C:
            continue
        C.add(s)
        d = dist_to_q(s)
        dc += 1
        S.append((d, s))
        if d <= r:
            R.append((d, s))
            if len(R) > k:
                R.remove(max(R))
            if len(R) == k:
                r = max(R)[0]
    hops = 0
    if trace is not None:
        trace.append(dc)
    while S:
        if max_dc > 0 and dc >= max_dc:
            break
        s = min(S)                       # argmin over S by (d, id)
        S.remove(s)
        if s[0] > thr_fn(r):
            return sorted(R), dc, hops
        hops += 1
        p = 1
        M = list(neigh[s[1]])            # already ascending by length
        while M and p <= ep:
            n = M.pop(0)
            if n not in C:
                C.add(n)
                d = dist_to_q(n)
                dc += 1
                if d <= thr_fn(r):
                    S.append((d, n))
                if d <= r:
                    R.append((d, n))
                    if len(R) > k:
                        R.remove(max(R))
                    if len(R) == k:
                        r = max(R)[0]
            p += 1
        if trace is not None:
            trace.append(dc)
    return sorted(R), dc, hops


def adjusted_graph(knn, knn_d, e_o, e_i):
    """Algorithm 2 with the loop guard read as "p <= e_o or p <= e_i" (R1).
    knn[o] lists o's neighbours, knn_d[o] their distances.  Returns per-node
    lists of (len, id) sorted ascending."""
    n = len(knn)
    Ge = [dict() for _ in range(n)]      # id -> length, per node
    for o in range(n):
        S = [(knn_d[o][t], knn[o][t]) for t in range(len(knn[o])) if knn[o][t] >= 0]
        p = 1
        while S and (p <= e_o or p <= e_i):
            dn = min(S)
            S.remove(dn)
            d, nn = dn
            if p <= e_o and nn not in Ge[o]:
                Ge[o][nn] = d
            if p <= e_i and o not in Ge[nn]:
                Ge[nn][o] = d
            p += 1
    return [sorted((l, i) for i, l in Ge[o].items()) for o in range(n)]


def adjusted_graph_with_constraint(knn, knn_d, e_o, e_i):
    """Algorithm 3.  Same input as adjusted_graph.  G_i is a list of sets;
    every argmin is taken over the remaining members.  Returns per-node lists
    of (len, id) sorted ascending."""
    n = len(knn)
    Gt = [dict((i, l) for l, i in lst) for lst in adjusted_graph(knn, knn_d, 0, e_i)]
    Ge = [dict() for _ in range(n)]
    Gi = [set() for _ in range(n)]
    M = set(range(n))
    while M:
        o = min(M, key=lambda x: (len(Gt[x]), x))
        M.remove(o)
        S = dict(Gt[o])
        while S:
            nn = min(S, key=lambda x: (S[x], x))
            d = S.pop(nn)
            if not Gi[nn] or (len(Gi[nn]) < e_i and len(Ge[o]) < e_o):
                Ge[o][nn] = d
                Gi[nn].add(o)
    for o in range(n):
        S = {knn[o][t]: knn_d[o][t] for t in range(len(knn[o])) if knn[o][t] >= 0}
        while S and len(Ge[o]) < e_o:
            nn = min(S, key=lambda x: (S[x], x))
            d = S.pop(nn)
            if nn not in Ge[o]:
                Ge[o][nn] = d
    return [sorted((l, i) for i, l in Ge[o].items()) for o in range(n)]


def construct_anng(order, dist, k_c, thr_fn, n_seeds, n_pivots):
    """Algorithm 9 as printed: objects in `order` one by one; each gets the
    KnnSearch results on the graph so far as edges, and each result gets the
    reverse edge.  Seeds: the n_seeds objects nearest the new one among the
    first n_pivots inserted, by (d, id).  Returns per-node lists of (len, id)
    sorted ascending."""
    adj = {o: [] for o in order}
    inserted = []
    for o in order:
        if inserted:
            neigh = {v: [i for _, i in sorted(adj[v])] for v in inserted}
            piv = sorted(inserted[:n_pivots], key=lambda m: (dist(o, m), m))[:n_seeds]
            R, _, _ = knn_search(neigh, lambda m: dist(o, m), piv, k_c, thr_fn)
            for d, m in R:
                adj[o].append((d, m))
                adj[m].append((d, o))
        inserted.append(o)
    return {o: sorted(adj[o]) for o in order}


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


def has_path(Gp, ns, nd, d_ns_nd):
    """Algorithm 5 with edge lengths as distances."""
    for c, _ in Gp[ns]:
        for m, lcm in Gp[c]:
            if m == nd and lcm < d_ns_nd:
                return True
    return False


def adjust_path(G):
    """Algorithm 4.  G: per-node lists of (len, id).  Returns G_p as per-node
    lists of (id, len) in insertion order."""
    n = len(G)
    Gt = [sorted(G[v]) for v in range(n)]
    Gp = [[] for _ in range(n)]
    Vt = [v for v in range(n) if Gt[v]]
    while Vt:
        for v in list(Vt):               # ascending id, immediate visibility (R11)
            ln, nd = min(Gt[v])
            if not has_path(Gp, v, nd, ln):
                Gp[v].append((nd, ln))
            Gt[v].remove((ln, nd))
            if not Gt[v]:
                Vt.remove(v)
    return Gp


class PaperVisited:
    """Algorithms 6 and 7: table b of size s plus collision lists L."""

    def __init__(self, n, b=11):
        lg = int(n).bit_length() - 1
        self.s = 1 << ((lg + b) // 2)
        self.b = [None] * self.s
        self.L = [set() for _ in range(self.s)]

    def set(self, i):
        h = i % self.s
        if self.b[h] is None:
            self.b[h] = i
        elif self.b[h] != i:
            self.L[h].add(i)

    def isset(self, i):
        h = i % self.s
        if self.b[h] == i:
            return True
        return i in self.L[h]


def brute_topk(D: np.ndarray, k: int, exclude_diag: bool = False):
    """k smallest (d, j) per row of a dense distance matrix via a stable sort."""
    D = np.array(D, dtype=np.float64, copy=True)
    if exclude_diag:
        np.fill_diagonal(D, np.inf)
    order = np.argsort(D, axis=1, kind="stable")[:, :k]
    return order.astype(np.int32), np.take_along_axis(D, order, axis=1)
