"""GPU parity: every kernel of the path against the CPU oracle on the same
seeded inputs.  u8 data is compared bit for bit (ids, distances, distance
computations, expansions); float data by the margin rule."""
import dataclasses
import math

import numpy as np
import pytest

from oracle import oracle as orc
from paper_1810_07355_amd import datagen as dg

from gpu_common import (api, c1_problem, dev, gpu_graph, gpu_vectors, have_gpu, host, L,
                        margin_ok, say, to_dev, torch)

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not have_gpu(), reason="needs an MI355X GPU")]


# ------------------------------------------------------------------ codecs

def test_encode_bit_exact():
    g = np.random.default_rng(11)
    x = np.concatenate([g.standard_normal((300, 100)) * 3.0,
                        g.uniform(-1e-3, 1e-3, (20, 100)),
                        np.zeros((1, 100))]).astype(np.float32)
    x[0, :6] = [65504, 65520, 1e-8, -2 ** -24, 3.3e38, -0.0]
    A, Lb = api(), L()
    for dt, odt in [(Lb.F16, orc.F16), (Lb.BF16, orc.BF16), (Lb.FP8_E4M3, orc.FP8)]:
        say("encode", dt)
        v = A.encode(to_dev(x), dt, Lb.L2SQ)
        ref, rs = orc.encode_rows(x, odt, pitch=v.pitch)
        assert np.array_equal(host(v.data), ref), dt
        if rs is not None:
            assert np.array_equal(host(v.scale), rs)


# ------------------------------------------------------------------- top-k

def test_topk_u8_knn_graph_c1():
    P = c1_problem()
    say("build_knn c1")
    B = gpu_vectors(P["x"], orc.L2SQ)
    ids, d = api().build_knn(B, P["cfg"].knn_k)
    assert np.array_equal(host(ids), P["knn"])
    assert np.array_equal(host(d), P["kd"].astype(np.int32))


@pytest.mark.parametrize("n,dim,k", [(1037, 128, 20), (130, 64, 129), (70, 200, 7), (5, 16, 4)])
def test_topk_u8_ragged(n, dim, k):
    say("topk ragged", n, dim, k)
    x = dg.random_tie_u8(n, dim, 3) if dim == 64 else dg.random_vectors(n, dim, "u8", 4)
    bv = orc.Vectors.from_array(x, orc.L2SQ)
    k = min(k, n - 1)
    rid, rd = orc.knn_graph(bv, k)
    ids, d = api().build_knn(gpu_vectors(x, orc.L2SQ), k)
    assert np.array_equal(host(ids), rid)
    assert np.array_equal(host(d), rd.astype(np.int32))


WIDE_N = 70_001      # above 256 query rows per compute unit: the wide u8 kernel


@pytest.mark.parametrize("dim,k,tie", [(128, 100, False), (100, 10, True), (40, 1, True),
                                       (64, 256, False)])
def test_topk_u8_wide_rows_sampled(dim, k, tie):
    """From 65,536 query rows the u8 top-k runs 256 rows per block with the
    rows' lists and candidate buffers in global memory.  Its kNN rows, at
    dims with one and two 64-byte k-steps (zero-extended), k from 1 to 256
    and heavy distance ties, equal the oracle's bit for bit on sampled rows,
    the first and last rows, and the rows at block and tile edges."""
    say("topk wide", dim, k, tie)
    n = WIDE_N
    x = dg.random_tie_u8(n, dim, 11) if tie else dg.random_vectors(n, dim, "u8", 12)
    g = np.random.default_rng(dim + k)
    rows = np.unique(np.concatenate([
        np.arange(0, 80), np.arange(n - 150, n), [255, 256, 511, 512, 65535, 65536, 65792],
        g.choice(n, 120, replace=False)])).astype(np.int32)
    bv = orc.Vectors.from_array(x, orc.L2SQ)
    rid, rd = orc.knn_graph(bv, k, rows=rows)
    ids, d = api().build_knn(gpu_vectors(x, orc.L2SQ), k)
    ids, d = host(ids), host(d)
    assert np.array_equal(ids[rows], rid)
    assert np.array_equal(d[rows], rd.astype(np.int32))
    # every row is a valid top-k list: ascending (d, id), no self, no repeat
    assert np.all(ids >= 0) and np.all(ids < n)
    assert not np.any(ids == np.arange(n)[:, None])
    key = d.astype(np.int64) * (1 << 32) + ids
    assert np.all(np.diff(key, axis=1) > 0)


def test_topk_u8_wide_candidate_list():
    """The wide u8 kernel over a candidate list (gathered rows with their
    global ids), as for seeds: sampled query rows equal the oracle's."""
    say("topk wide candidate list")
    x = dg.random_tie_u8(20_000, 128, 13, levels=5)
    q = dg.random_tie_u8(WIDE_N, 128, 14, levels=5)
    cand = np.sort(np.random.default_rng(5).choice(20_000, 3000, replace=False)).astype(np.int32)
    rows = np.unique(np.concatenate([np.arange(0, 40), np.arange(WIDE_N - 40, WIDE_N),
                                     np.random.default_rng(6).choice(WIDE_N, 100)]))
    bv = orc.Vectors.from_array(x, orc.L2SQ)
    qv = orc.Vectors.from_array(q[rows], orc.L2SQ)
    sid, sd = orc.topk(qv, bv, 8, cand=cand)
    ids, d = api().topk(gpu_vectors(q, orc.L2SQ), gpu_vectors(x, orc.L2SQ), 8, cand=to_dev(cand))
    assert np.array_equal(host(ids)[rows], sid)
    assert np.array_equal(host(d)[rows], sd.astype(np.int32))


def test_topk_seeds_from_pivots_c1():
    P = c1_problem()
    say("seeds from pivots c1")
    A = api()
    ids, d = A.topk(gpu_vectors(P["q"], orc.L2SQ), gpu_vectors(P["x"], orc.L2SQ), 8,
                    cand=to_dev(P["piv"]))
    assert np.array_equal(host(ids), P["seeds"])


@pytest.mark.parametrize("k", [1, 8, 16, 17, 64, 100])
def test_topk_u8_list_and_buffer_sizes(k):
    """Top-k across the list and candidate-buffer size steps (lists of k
    rounded to 8 keys; 80 candidate slots up to k = 16, 128 above), with few
    query rows (so the candidate tiles are split over several blocks and
    merged), heavy distance ties, a ragged last tile and a candidate list."""
    say("topk sizes", k)
    A = api()
    x = dg.random_tie_u8(3001, 48, 5)
    q = dg.random_tie_u8(37, 48, 6)
    bv, qv = orc.Vectors.from_array(x, orc.L2SQ), orc.Vectors.from_array(q, orc.L2SQ)
    B, Q = gpu_vectors(x, orc.L2SQ), gpu_vectors(q, orc.L2SQ)
    rid, rd = orc.topk(qv, bv, k)
    ids, d = A.topk(Q, B, k)
    assert np.array_equal(host(ids), rid)
    assert np.array_equal(host(d), rd.astype(np.int32))
    cand = np.random.default_rng(k).choice(3001, 1111, replace=False).astype(np.int32)
    rid, rd = orc.topk(qv, bv, k, cand=cand)
    ids, d = A.topk(Q, B, k, cand=to_dev(cand))
    assert np.array_equal(host(ids), rid)
    assert np.array_equal(host(d), rd.astype(np.int32))


@pytest.mark.parametrize("k,use_cand", [(20, False), (8, True), (3, False)])
def test_topk_f32_cosine_and_l2(k, use_cand):
    """k = 20 (lists merged per row), k = 8 over a candidate list (the seeding's
    shape) and k = 3 (lists of at most 8 keys, flushed after every tile)."""
    for kind, metric in [("f32cos", orc.COS), ("f32l2", orc.L2SQ)]:
        say("topk float", kind, "k", k, "candidates" if use_cand else "")
        cfg = dg.scaled(dg.PRESETS["c3" if kind == "f32cos" else "c5"], 3000, 40, n_clusters=30)
        x, q = dg.base(cfg), dg.queries(cfg)
        bv, qv = orc.Vectors.from_array(x, metric), orc.Vectors.from_array(q, metric)
        cand = (np.random.default_rng(k).choice(3000, 1999, replace=False).astype(np.int32)
                if use_cand else None)
        rid, rd = orc.topk(qv, bv, k, cand=cand)
        ids, d = api().topk(gpu_vectors(q, metric), gpu_vectors(x, metric), k,
                            cand=None if cand is None else to_dev(cand))
        gi, gd = host(ids), host(d)
        if cand is not None:
            assert np.all(np.isin(gi, cand))
        # every returned distance within 1e-4 relative of the exact fp64
        # distance of its id (cosine: floor 1e-2 against cancellation near 0)
        floor = 1e-2 if metric == orc.COS else 0.0
        full = orc.lib()
        ex = np.array([[full.or_dist(bv.ref, int(j), qv.ref, r) for j in gi[r]]
                       for r in range(len(q))])
        assert np.all(np.abs(gd - ex) <= 1e-4 * np.maximum(np.abs(ex), floor))
        assert np.all(np.abs(np.sort(gd, axis=1) - rd) <= 1e-4 * np.maximum(np.abs(rd), floor))
        # the id sets agree except where the k-th distance ties within 1e-4
        for r in range(len(q)):
            if set(gi[r]) != set(rid[r]):
                kth = rd[r, -1]
                for j in set(gi[r]) ^ set(rid[r]):
                    dj = full.or_dist(bv.ref, int(j), qv.ref, r)
                    assert abs(dj - kth) <= 1e-4 * max(abs(kth), floor), (kind, r, j)


@pytest.mark.parametrize("kind,k", [("u8", 8), ("u8", 16), ("f32cos", 8), ("f32l2", 1),
                                    ("f32cos", 16)])
def test_topk_long_candidate_list(kind, k):
    """Top-k over a long candidate list (the seeds' shape: thousands of
    pivots, k <= 16, few query rows, so the candidate tiles are split over
    several blocks and the parts merged).  u8 results, on tie-heavy data,
    are bit-exact against the oracle; float ones meet the float rule (ids
    differ only at ties within 1e-4)."""
    say("topk long candidate list", kind, k)
    metric = orc.COS if kind == "f32cos" else orc.L2SQ
    if kind == "u8":
        x = dg.random_tie_u8(20000, 48, 7)
        q = dg.random_tie_u8(300, 48, 8)
    else:
        cfg = dg.scaled(dg.PRESETS["c3" if kind == "f32cos" else "c5"], 20000, 300, n_clusters=40)
        x, q = dg.base(cfg), dg.queries(cfg)
    bv, qv = orc.Vectors.from_array(x, metric), orc.Vectors.from_array(q, metric)
    cand = np.sort(np.random.default_rng(k + len(kind)).choice(20000, 6000, replace=False)).astype(np.int32)
    rid, rd = orc.topk(qv, bv, k, cand=cand)
    ids, d = api().topk(gpu_vectors(q, metric), gpu_vectors(x, metric), k, cand=to_dev(cand))
    gi, gd = host(ids), host(d)
    if kind == "u8":
        assert np.array_equal(gi, rid)
        assert np.array_equal(gd, rd.astype(np.int32))
        return
    floor = 1e-2 if metric == orc.COS else 0.0
    full = orc.lib()
    ex = np.array([[full.or_dist(bv.ref, int(j), qv.ref, r) for j in gi[r]] for r in range(len(q))])
    assert np.all(np.abs(gd - ex) <= 1e-4 * np.maximum(np.abs(ex), floor))
    for r in range(len(q)):
        if set(gi[r]) != set(rid[r]):
            kth = rd[r, -1]
            for j in set(gi[r]) ^ set(rid[r]):
                dj = full.or_dist(bv.ref, int(j), qv.ref, r)
                assert abs(dj - kth) <= 1e-4 * max(abs(kth), floor), (kind, r, j)


FW_N = 40_001       # above 128 query rows per compute unit: the bf16-screened f32 kernel


@pytest.mark.parametrize("kind,dim,k", [("f32cos", 100, 100), ("f32l2", 96, 10),
                                        ("f32l2", 37, 100), ("f32cos", 128, 1)])
def test_topk_f32_wide_rows(kind, dim, k):
    """From 32,768 query rows float top-k screens on bf16 matrix cores and
    recomputes the survivors exactly in f32.  The screen is conservative
    (its bound covers the bf16 rounding), so sampled rows, the first and last
    rows and the rows at block edges meet the float rule of the general
    kernel against the fp64 oracle: every distance within 1e-4 relative of
    its id's exact distance (cosine floor 1e-2), sorted distances within 1e-4
    of the oracle's, ids differing only at ties with the k-th within 1e-4."""
    say("topk f32 wide", kind, dim, k)
    metric = orc.COS if kind == "f32cos" else orc.L2SQ
    cfg = dg.scaled(dg.PRESETS["c3" if kind == "f32cos" else "c5"], FW_N, 10,
                    n_clusters=200)
    cfg = dataclasses.replace(cfg, dim=dim)
    x = dg.base(cfg)
    g = np.random.default_rng(dim + k)
    rows = np.unique(np.concatenate([np.arange(0, 40), np.arange(FW_N - 60, FW_N),
                                     [127, 128, 32767, 32768, 32895],
                                     g.choice(FW_N, 100, replace=False)])).astype(np.int32)
    bv = orc.Vectors.from_array(x, metric)
    rid, rd = orc.knn_graph(bv, k, rows=rows)
    ids, d = api().build_knn(gpu_vectors(x, metric), k)
    gi, gd = host(ids)[rows], host(d)[rows].astype(np.float64)
    floor = 1e-2 if metric == orc.COS else 0.0
    full = orc.lib()
    ex = np.array([[full.or_dist(bv.ref, int(j), bv.ref, int(rows[r])) for j in gi[r]]
                   for r in range(len(rows))])
    assert np.all(gi >= 0) and not np.any(gi == rows[:, None])
    assert np.all(np.abs(gd - ex) <= 1e-4 * np.maximum(np.abs(ex), floor))
    assert np.all(np.abs(gd - rd) <= 1e-4 * np.maximum(np.abs(rd), floor))
    for r in range(len(rows)):
        diff = set(gi[r].tolist()) ^ set(rid[r].tolist())
        kth = rd[r, -1]
        for j in diff:
            dj = full.or_dist(bv.ref, int(j), bv.ref, int(rows[r]))
            assert abs(dj - kth) <= 1e-4 * max(abs(kth), floor), (r, j)


def test_topk_f32_wide_candidate_list():
    """The bf16-screened f32 kernel over a candidate list (gathered rows, ids
    mapped back), cosine, k = 8 as for seeds."""
    say("topk f32 wide candidate list")
    cfg = dg.scaled(dg.PRESETS["c3"], 20_000, FW_N, n_clusters=100)
    x, q = dg.base(cfg), dg.queries(cfg)
    cand = np.sort(np.random.default_rng(7).choice(20_000, 3000, replace=False)).astype(np.int32)
    rows = np.unique(np.concatenate([np.arange(0, 30), np.arange(FW_N - 30, FW_N),
                                     np.random.default_rng(8).choice(FW_N, 100)]))
    bv = orc.Vectors.from_array(x, orc.COS)
    qv = orc.Vectors.from_array(q[rows], orc.COS)
    sid, sd = orc.topk(qv, bv, 8, cand=cand)
    ids, d = api().topk(gpu_vectors(q, orc.COS), gpu_vectors(x, orc.COS), 8, cand=to_dev(cand))
    gi, gd = host(ids)[rows], host(d)[rows].astype(np.float64)
    assert np.all(np.isin(gi, cand))
    assert np.all(np.abs(gd - sd) <= 1e-4 * np.maximum(np.abs(sd), 1e-2))
    for r in range(len(rows)):
        for j in set(gi[r].tolist()) ^ set(sid[r].tolist()):
            dj = orc.lib().or_dist(bv.ref, int(j), qv.ref, r)
            assert abs(dj - sd[r, -1]) <= 1e-4 * max(abs(sd[r, -1]), 1e-2), (r, j)


# ---------------------------------------------------------- adjustments

def test_adjust_degree_u8_c1():
    P = c1_problem()
    say("adjust_degree c1")
    A, Lb = api(), L()
    g = A.adjust_degree(to_dev(P["knn"]), to_dev(P["kd"].astype(np.int32)), Lb.U8, Lb.L2SQ,
                        P["cfg"].e_o, P["cfg"].e_i)
    off, nb, ln = P["sa"]
    assert np.array_equal(host(g.offsets), off)
    assert np.array_equal(host(g.nbrs), nb)
    assert np.array_equal(host(g.lens), ln.astype(np.int32))


@pytest.mark.parametrize("e_o,e_i", [(3, 7), (7, 3), (0, 5), (5, 0), (12, 12)])
def test_adjust_degree_float_and_ties(e_o, e_i):
    say("adjust_degree float", e_o, e_i)
    A, Lb = api(), L()
    # float lengths, with asymmetric values so the duplicate rule matters
    x = dg.random_tie_u8(400, 5, 9, levels=4)
    bv = orc.Vectors.from_array(x, orc.L2SQ)
    knn, kd = orc.knn_graph(bv, 12)
    g = np.random.default_rng(e_o * 31 + e_i)
    kdf = (kd + g.uniform(0, 0.5, kd.shape)).astype(np.float32)
    kdf = np.sort(kdf, axis=1)        # rows stay ascending
    off, nb, ln = orc.adjust_degree(knn, kdf.astype(np.float64), e_o, e_i)
    gg = A.adjust_degree(to_dev(knn), to_dev(kdf), Lb.F32, Lb.L2SQ, e_o, e_i)
    assert np.array_equal(host(gg.offsets), off)
    assert np.array_equal(host(gg.nbrs), nb)
    assert np.array_equal(host(gg.lens), ln.astype(np.float32))


def _sac_gpu_vs_oracle(knn, kd, e_o, e_i, int_len):
    A, Lb = api(), L()
    off, nb, ln = orc.adjust_degree_constrained(knn, kd.astype(np.float64), e_o, e_i)
    dt = np.int32 if int_len else np.float32
    g = A.adjust_degree_constrained(to_dev(knn), to_dev(kd.astype(dt)),
                                    Lb.U8 if int_len else Lb.F32, Lb.L2SQ, e_o, e_i)
    assert np.array_equal(host(g.offsets), off)
    assert np.array_equal(host(g.nbrs), nb)
    assert np.array_equal(host(g.lens), ln.astype(dt))
    return off


@pytest.mark.parametrize("e_o,e_i", [(10, 30), (5, 0), (0, 5), (1, 1), (20, 10), (300, 20)])
def test_adjust_degree_constrained_u8_c1(e_o, e_i):
    P = c1_problem()
    say("adjust_degree_constrained c1", e_o, e_i)
    _sac_gpu_vs_oracle(P["knn"], P["kd"], e_o, e_i, True)


@pytest.mark.parametrize("e_o,e_i", [(3, 7), (7, 3), (12, 12), (40, 12)])
def test_adjust_degree_constrained_float_ties_ragged(e_o, e_i):
    say("adjust_degree_constrained float/ties/ragged", e_o, e_i)
    x = dg.random_tie_u8(400, 5, 9, levels=4)
    knn, kd = orc.knn_graph(orc.Vectors.from_array(x, orc.L2SQ), 12)
    # integer lengths with many ties
    _sac_gpu_vs_oracle(knn, kd, e_o, e_i, True)
    # float lengths; every 7th row cut short (padded with -1 / +inf)
    g = np.random.default_rng(e_o * 17 + e_i)
    kdf = np.sort((kd + g.uniform(0, 0.5, kd.shape)).astype(np.float32), axis=1)
    knn = knn.copy()
    for r in range(0, 400, 7):
        cut = 1 + r % 12
        knn[r, 12 - cut:] = -1
        kdf[r, 12 - cut:] = np.inf
    _sac_gpu_vs_oracle(knn, kdf, e_o, e_i, False)


@pytest.mark.parametrize("n", [0, 1, 2, 65])
def test_adjust_degree_constrained_tiny(n):
    say("adjust_degree_constrained tiny", n)
    k = 3
    knn = np.full((n, k), -1, np.int32)
    kd = np.full((n, k), np.iinfo(np.int32).max, np.int64)
    for m in range(n):
        others = [j for j in range(n) if j != m][:k]
        knn[m, :len(others)] = others
        kd[m, :len(others)] = [abs(j - m) for j in others]
        order = np.lexsort((knn[m, :len(others)], kd[m, :len(others)]))
        knn[m, :len(others)] = knn[m, :len(others)][order]
        kd[m, :len(others)] = kd[m, :len(others)][order]
    off = _sac_gpu_vs_oracle(knn, kd, 2, 2, True)
    assert len(off) == n + 1


def test_adjust_degree_constrained_hub_lists():
    """One node in every row: its N(G_t, o) holds 6000 members (longer than the
    on-chip sort's 4096 and many wave chunks); lengths tie often."""
    say("adjust_degree_constrained hub")
    n, k = 6000, 4
    g = np.random.default_rng(5)
    knn = np.empty((n, k), np.int32)
    kd = np.empty((n, k), np.int64)
    for m in range(n):
        ids = [0] if m else []
        while len(ids) < k:
            j = int(g.integers(1, n))
            if j != m and j not in ids:
                ids.append(j)
        d = g.integers(1, 6, size=k)
        order = np.lexsort((ids, d))
        knn[m] = np.array(ids)[order]
        kd[m] = d[order]
    for e_o, e_i in [(5, 4), (2, 2), (50, 3)]:
        _sac_gpu_vs_oracle(knn, kd, e_o, e_i, True)


def test_graph_stats_against_oracle():
    P = c1_problem()
    A, Lb = api(), L()
    say("graph_stats c1 SA / PA")
    for off, nb, ln in (P["sa"], P["pa"]):
        g = gpu_graph(off, nb, ln)
        for frac, keep in ((0.05, 10), (0.01, 1), (1.0, 0), (0.3, 1000)):
            got = A.graph_stats(g, Lb.U8, Lb.L2SQ, frac, keep)
            want = orc.graph_stats(off, nb, ln, orc.L2SQ, frac, keep)
            assert got[0] == want[0] and got[1] == want[1]
            assert got[2] == pytest.approx(want[2], rel=1e-12, abs=0)
    say("graph_stats float cosine lengths and an empty graph")
    g = np.random.default_rng(11)
    n = 3000
    deg = g.integers(0, 30, size=n)
    off = np.concatenate([[0], np.cumsum(deg)]).astype(np.int64)
    nb = g.integers(0, n, size=off[-1]).astype(np.int32)
    ln = g.uniform(0, 2, size=off[-1]).astype(np.float32)
    gg = gpu_graph(off, nb, ln, int_len=False)
    got = A.graph_stats(gg, Lb.F32, Lb.COSINE)
    want = orc.graph_stats(off, nb, ln.astype(np.float64), orc.COS)
    assert got[0] == want[0] and got[1] == want[1]
    assert got[2] == pytest.approx(want[2], rel=1e-12, abs=0)
    e = gpu_graph(np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.int32))
    assert A.graph_stats(e, Lb.U8, Lb.L2SQ) == (0.0, 0.0, 0.0)


def _vptree_vs_oracle(x, q, metric, leaf_size, n_seeds, seed=0):
    A = api()
    n = len(x)
    prio = dg.vp_priority(n, seed)
    bv, qv = orc.Vectors.from_array(x, metric), orc.Vectors.from_array(q, metric)
    ref = orc.vptree_build(bv, prio, leaf_size, n_seeds)
    B, Q = gpu_vectors(x, metric), gpu_vectors(q, metric)
    t = A.vptree_build(B, to_dev(prio.view(np.int32)), leaf_size, n_seeds)
    m, l = t.n_nodes, t.n_leaves
    assert (m, l) == (len(ref["vp"]), len(ref["seeds"]))
    assert np.array_equal(host(t.node_vp)[:m], ref["vp"])
    assert np.array_equal(host(t.node_child)[:m], ref["child"])
    inner = ref["child"] >= 0
    mu = host(t.node_mu)[:3 * m].reshape(m, 3).astype(np.float64)
    assert np.array_equal(mu[inner], ref["mu"][inner])
    assert np.array_equal(host(t.leaf_seeds)[:l * n_seeds].reshape(l, n_seeds), ref["seeds"])
    s, dc = A.vptree_seeds(B, t, Q)
    rs, rdc = orc.vptree_seeds(bv, qv, ref)
    assert np.array_equal(host(s), rs) and np.array_equal(host(dc), rdc)
    return rdc


def test_vptree_u8_c1_against_oracle():
    P = c1_problem()
    say("vptree c1 u8: 100 queries and the base rows as queries")
    dc = _vptree_vs_oracle(P["x"], np.concatenate([P["q"], P["x"][:2000]]), orc.L2SQ, 100, 10)
    assert dc.min() >= 4 and dc.max() <= 5


@pytest.mark.parametrize("metric", [orc.L2SQ, orc.COS])
def test_vptree_float_against_oracle(metric):
    say("vptree f32", metric)
    g = np.random.default_rng(21 + metric)
    x = g.standard_normal((20000, 100)).astype(np.float32)
    q = g.standard_normal((500, 100)).astype(np.float32)
    if metric == orc.COS:
        x /= np.linalg.norm(x, axis=1, keepdims=True)
        q /= np.linalg.norm(q, axis=1, keepdims=True)
    _vptree_vs_oracle(x, q, metric, 100, 10, seed=3)


@pytest.mark.parametrize("n,leaf,ns", [(1, 4, 3), (4, 4, 6), (5, 4, 2), (257, 256, 1),
                                       (1000, 7, 10), (300, 100, 100)])
def test_vptree_small_and_padding(n, leaf, ns):
    say("vptree small", n, leaf, ns)
    x = dg.random_tie_u8(n, 5, 17, levels=4)
    _vptree_vs_oracle(x, x[:50], orc.L2SQ, leaf, ns, seed=n)


@pytest.mark.parametrize("max_batch,n_pivots", [(2048, 1024), (1, 4), (64, 1)])
def test_anng_u8_against_oracle(max_batch, n_pivots):
    """Algorithm 9 in batches on c1's rows (the first 300 for the
    one-at-a-time case): the whole graph bit for bit."""
    from paper_1810_07355_amd import anng
    P = c1_problem()
    A, Lb = api(), L()
    n = 10000 if max_batch > 1 else 300
    x = P["x"][:n]
    order = dg.vp_priority(n, 11).astype(np.int64)
    say("anng u8", n, max_batch, n_pivots)
    g = anng.build_anng(to_dev(x), Lb.L2SQ, to_dev(order.astype(np.int32)), 10, 0.1,
                        n_seeds=8, n_pivots=n_pivots, max_batch=max_batch)
    off, nb, ln = orc.anng(x, orc.L2SQ, order, 10, 0.1, n_seeds=8, n_pivots=n_pivots,
                           max_batch=max_batch)
    assert np.array_equal(host(g.offsets), off)
    assert np.array_equal(host(g.nbrs), nb)
    assert np.array_equal(host(g.lens), ln.astype(np.int32))


def test_construct_graph_from_anng_u8_against_oracle():
    """Algorithm 8 end to end on c1's rows: ANNG (k_c = 40, eps_c = 0.1) ->
    G_k = ConstructAdjustedGraph(G_a, k_c, 0) -> Algorithm 2 (e_o = 10,
    e_i = 30) -> path adjustment, every stage bit for bit against the oracle,
    then searches over the result."""
    from paper_1810_07355_amd import anng
    P = c1_problem()
    A, Lb = api(), L()
    x = P["x"]
    n, k_c = len(x), 40
    order = dg.vp_priority(n, 12).astype(np.int64)
    say("Algorithm 8 from an ANNG, k_c", k_c)
    g = anng.build_anng(to_dev(x), Lb.L2SQ, to_dev(order.astype(np.int32)), k_c, 0.1)
    off, nb, ln = orc.anng(x, orc.L2SQ, order, k_c, 0.1)
    assert np.array_equal(host(g.offsets), off) and np.array_equal(host(g.nbrs), nb)
    ids, d = A.graph_head(g, k_c, Lb.U8, Lb.L2SQ)
    rid, rd = orc.aknng(off, nb, ln, k_c)
    assert np.array_equal(host(ids), rid)
    assert np.array_equal(host(d).astype(np.int64),
                          np.where(np.isinf(rd), 2 ** 31 - 1, rd).astype(np.int64))
    sa = A.adjust_degree(ids, d, Lb.U8, Lb.L2SQ, 10, 30)
    so, sn, sl = orc.adjust_degree(rid, rd, 10, 30)
    assert np.array_equal(host(sa.offsets), so) and np.array_equal(host(sa.nbrs), sn)
    pa = A.adjust_path(sa, Lb.U8, Lb.L2SQ)
    po, pn, pl = orc.adjust_path(so, sn, sl)
    assert np.array_equal(host(pa.offsets), po) and np.array_equal(host(pa.nbrs), pn)
    ref = orc.search(P["bv"], po, pn, P["qv"], P["seeds"], 10, 0.05)
    r = A.search(gpu_vectors(x, orc.L2SQ), pa, gpu_vectors(P["q"], orc.L2SQ),
                 to_dev(P["seeds"]), k=10, eps=0.05)
    assert np.array_equal(host(r.ids), ref["ids"]) and np.array_equal(host(r.dc), ref["dc"])
    # rows of fewer than k_c edges are padded; a k beyond every degree pads all rows
    deg = np.diff(off)
    big = int(deg.max()) + 3
    ids2, d2 = A.graph_head(g, big, Lb.U8, Lb.L2SQ)
    h = host(ids2)
    assert np.all(h[np.arange(n), deg] == -1)
    assert np.array_equal(h[np.arange(n), deg - 1], nb[off[1:] - 1])


def test_graph_add_edges_against_numpy():
    say("graph_add_edges")
    A, Lb = api(), L()
    g = np.random.default_rng(31)
    n = 500
    deg = g.integers(0, 12, size=n)
    off = np.concatenate([[0], np.cumsum(deg)]).astype(np.int64)
    nb = g.integers(0, n, size=off[-1]).astype(np.int32)
    ln = g.integers(0, 50, size=off[-1]).astype(np.int32)
    for v in range(n):                         # lists sorted by (len, id)
        o = np.lexsort((nb[off[v]:off[v + 1]], ln[off[v]:off[v + 1]]))
        nb[off[v]:off[v + 1]] = nb[off[v]:off[v + 1]][o]
        ln[off[v]:off[v + 1]] = ln[off[v]:off[v + 1]][o]
    m = 3000
    src = g.integers(-2, n + 2, size=m).astype(np.int32)      # a few ids outside [0, n)
    dst = g.integers(-2, n + 2, size=m).astype(np.int32)
    el = g.integers(0, 50, size=m).astype(np.int32)
    out = A.graph_add_edges(gpu_graph(off, nb, ln), to_dev(src), to_dev(dst), to_dev(el),
                            Lb.U8, Lb.L2SQ)
    lists = [list(zip(ln[off[v]:off[v + 1]].tolist(), nb[off[v]:off[v + 1]].tolist()))
             for v in range(n)]
    for s_, d_, l_ in zip(src.tolist(), dst.tolist(), el.tolist()):
        if 0 <= s_ < n and 0 <= d_ < n:
            lists[s_].append((l_, d_))
    lists = [sorted(a) for a in lists]
    assert host(out.offsets).tolist() == [0] + np.cumsum([len(a) for a in lists]).tolist()
    assert host(out.nbrs).tolist() == [i for a in lists for _, i in a]
    assert host(out.lens).tolist() == [l for a in lists for l, _ in a]


def test_adjust_path_u8_c1():
    P = c1_problem()
    say("adjust_path c1")
    A, Lb = api(), L()
    off, nb, ln = P["sa"]
    g = A.adjust_path(gpu_graph(off, nb, ln), Lb.U8, Lb.L2SQ)
    po, pn, pl = P["pa"]
    assert np.array_equal(host(g.offsets), po)
    assert np.array_equal(host(g.nbrs), pn)
    assert np.array_equal(host(g.lens), pl.astype(np.int32))


@pytest.mark.parametrize("seed", range(3))
def test_adjust_path_ties(seed):
    say("adjust_path ties", seed)
    A, Lb = api(), L()
    x = dg.random_tie_u8(600, 4, 40 + seed, levels=3)
    bv = orc.Vectors.from_array(x, orc.L2SQ)
    knn, kd = orc.knn_graph(bv, 16)
    off, nb, ln = orc.adjust_degree(knn, kd, 6, 16)
    po, pn, pl = orc.adjust_path(off, nb, ln)
    g = A.adjust_path(gpu_graph(off, nb, ln), Lb.U8, Lb.L2SQ)
    assert np.array_equal(host(g.offsets), po)
    assert np.array_equal(host(g.nbrs), pn)


def test_adjust_path_arbitrary_lists_with_repeats():
    """Path adjustment on lists that are not the degree adjustment's: random
    lengths with many ties, degrees from 1 to 300 (past the 64-lane chunks and
    long witness lists) and repeated neighbour ids, each list sorted by
    (length, id); bit-exact against the oracle."""
    say("adjust_path arbitrary")
    A, Lb = api(), L()
    g = np.random.default_rng(17)
    n = 400
    offs, nbs, lns = [0], [], []
    for v in range(n):
        deg = int(g.integers(1, 301)) if v % 37 == 0 else int(g.integers(1, 25))
        nb = g.integers(0, n, size=deg)
        nb[nb == v] = (v + 1) % n
        ln = g.integers(1, 12, size=deg)
        o = np.lexsort((nb, ln))
        nbs.append(nb[o]); lns.append(ln[o]); offs.append(offs[-1] + deg)
    off = np.array(offs, dtype=np.int64)
    nb = np.concatenate(nbs).astype(np.int32)
    ln = np.concatenate(lns).astype(np.int32)
    assert any(len(set(x.tolist())) < len(x) for x in nbs)
    po, pn, pl = orc.adjust_path(off, nb, ln)
    gg = A.adjust_path(gpu_graph(off, nb, ln), Lb.U8, Lb.L2SQ)
    assert np.array_equal(host(gg.offsets), po)
    assert np.array_equal(host(gg.nbrs), pn)
    assert np.array_equal(host(gg.lens), pl)


def test_graph_chain_on_gpu_equals_oracle_c1():
    P = c1_problem()
    say("kNN -> SA -> PA chain on GPU")
    A, Lb = api(), L()
    cfg = P["cfg"]
    ids, d = A.build_knn(gpu_vectors(P["x"], orc.L2SQ), cfg.knn_k)
    sa = A.adjust_degree(ids, d, Lb.U8, Lb.L2SQ, cfg.e_o, cfg.e_i)
    pa = A.adjust_path(sa, Lb.U8, Lb.L2SQ)
    po, pn, pl = P["pa"]
    assert np.array_equal(host(pa.offsets), po)
    assert np.array_equal(host(pa.nbrs), pn)


# ---------------------------------------------------------------- search

def _run_search_u8(P, graph, k, eps, ep, launch=None, seeds=None, q=None):
    A = api()
    seeds = P["seeds"] if seeds is None else seeds
    q = P["q"] if q is None else q
    r = A.search(gpu_vectors(P["x"], orc.L2SQ), graph, gpu_vectors(q, orc.L2SQ), to_dev(seeds),
                 k=k, eps=eps, ep=ep, launch=launch)
    torch.cuda.synchronize()
    return r


def _assert_exact(r, ref, k):
    assert np.array_equal(host(r.ids)[:, :k], ref["ids"][:, :k])
    gd = host(r.dists)[:, :k]
    rd = np.where(np.isinf(ref["dists"][:, :k]), 2 ** 31 - 1, ref["dists"][:, :k]).astype(np.int64)
    assert np.array_equal(gd.astype(np.int64), rd)
    assert np.array_equal(host(r.dc), ref["dc"])
    assert np.array_equal(host(r.hops), ref["hops"])
    assert not np.any(host(r.flags) & L().QF_CAPACITY)


@pytest.mark.parametrize("k", [1, 10, 20])
def test_search_u8_c1_eps_sweep(k):
    P = c1_problem()
    po, pn, _ = P["pa"]
    G = gpu_graph(po, pn)
    for eps in P["cfg"].eps_grid:
        for ep in (orc.INF_EP, orc.dynamic_ep(eps)):
            say("search c1 k", k, "eps", eps, "ep", ep)
            ref = orc.search(P["bv"], po, pn, P["qv"], P["seeds"], k, eps, ep)
            r = _run_search_u8(P, G, k, eps, ep)
            _assert_exact(r, ref, k)


def test_degree_loss_gpu_equals_oracle_c1():
    """Equation 2 on c1's path-adjusted graph: the GPU searches and the
    oracle's searches give the same precision and distance counts at every
    range the binary searches visit, hence the same loss."""
    from paper_1810_07355_amd import tune
    P = c1_problem()
    po, pn, _ = P["pa"]
    G = gpu_graph(po, pn)
    gt_ids, gt_d = orc.topk(P["qv"], P["bv"], 10)

    def gpu_search(e):
        r = _run_search_u8(P, G, 10, e, orc.dynamic_ep(e))
        return (float(orc.recall_at_k(host(r.ids), host(r.dists), gt_d, 10).mean()),
                float(host(r.dc).astype(np.float64).mean()))

    def oracle_search(e):
        r = orc.search(P["bv"], po, pn, P["qv"], P["seeds"], 10, e, orc.dynamic_ep(e))
        return float(orc.recall_at_k(r["ids"], r["dists"], gt_d, 10).mean()), float(r["dc"].mean())

    say("degree loss c1: GPU searches")
    Lg, pg = tune.degree_loss(gpu_search, 0.90, 0.98)
    say("degree loss c1: oracle searches")
    Lo, po_ = orc.degree_loss(oracle_search, 0.90, 0.98)
    assert [t[0] for t in pg] == [t[0] for t in po_]
    assert Lg == pytest.approx(Lo, rel=1e-12) and math.isfinite(Lg)


@pytest.mark.parametrize("shape", [dict(s_capacity=64, visited_log2=8),
                                   dict(s_capacity=64, visited_log2=-1),
                                   dict(lanes_per_row=8, waves_per_block=2),
                                   dict(lanes_per_row=16, waves_per_block=1, blocks=3)])
def test_search_u8_small_capacities_stay_exact(shape):
    """Tiny on-chip capacities force the spill and off-chip visited paths."""
    P = c1_problem()
    off, nb, _ = P["sa"]                     # denser graph: more candidates per query
    G = gpu_graph(off, nb)
    cfg = api().launch_config(**shape)
    for eps, k in [(0.1, 10), (0.3, 20), (np.inf, 20)]:
        say("search small caps", shape, eps, k)
        ref = orc.search(P["bv"], off, nb, P["qv"], P["seeds"], k, eps, orc.INF_EP)
        r = _run_search_u8(P, G, k, eps, orc.INF_EP, launch=cfg)
        _assert_exact(r, ref, k)


def test_search_u8_single_big_component_unbounded():
    """One 4,000-node cluster and eps = inf: the whole component is visited."""
    say("search one component eps=inf")
    cfg = dg.scaled(dg.PRESETS["c1"], 4000, 40, n_clusters=1)
    x, q = dg.base(cfg), dg.queries(cfg)
    bv, qv = orc.Vectors.from_array(x, orc.L2SQ), orc.Vectors.from_array(q, orc.L2SQ)
    knn, kd = orc.knn_graph(bv, 10)
    off, nb, ln = orc.adjust_degree(knn, kd, 5, 10)
    seeds = dg.random_seeds(cfg, 40, 4)
    P = dict(x=x, q=q, seeds=seeds)
    G = gpu_graph(off, nb)
    for eps, k in [(np.inf, 10), (0.2, 50)]:
        ref = orc.search(bv, off, nb, qv, seeds, k, eps, orc.INF_EP)
        r = _run_search_u8(P, G, k, eps, orc.INF_EP)
        _assert_exact(r, ref, k)
        if np.isinf(eps):
            assert np.all(host(r.dc) == 4000) or np.all(ref["dc"] == host(r.dc))


def test_search_u8_duplicate_invalid_seeds_and_padding():
    P = c1_problem()
    po, pn, _ = P["pa"]
    seeds = P["seeds"].copy()
    seeds[:, 1] = seeds[:, 0]
    seeds[:, 2] = -1
    seeds[::3, 3] = 10 ** 6            # out of range: ignored
    say("search duplicate seeds")
    ref = orc.search(P["bv"], po, pn, P["qv"], seeds, 10, 0.05, orc.INF_EP)
    r = _run_search_u8(P, gpu_graph(po, pn), 10, 0.05, orc.INF_EP, seeds=seeds)
    _assert_exact(r, ref, 10)
    # empty graph: only the seeds are found, the rest is padding
    say("search empty graph")
    n = P["x"].shape[0]
    off0 = np.zeros(n + 1, np.int64)
    ref = orc.search(P["bv"], off0, np.zeros(1, np.int32), P["qv"], P["seeds"], 20, 0.1)
    A = api()
    g0 = A.Graph(to_dev(off0), torch.zeros(1, dtype=torch.int32, device=dev()), None)
    r = _run_search_u8(P, g0, 20, 0.1, orc.INF_EP)
    _assert_exact(r, ref, 20)
    assert np.all(host(r.flags) & L().QF_PADDED)


def test_search_mixed_k_eps_ep_per_query():
    P = c1_problem()
    po, pn, _ = P["pa"]
    nq = len(P["q"])
    g = np.random.default_rng(3)
    kq = g.choice([1, 10, 20], nq).astype(np.int32)
    eq = g.choice([0.0, 0.05, 0.2], nq).astype(np.float32)
    pq = np.array([orc.dynamic_ep(e) if i % 2 else orc.INF_EP for i, e in enumerate(eq)],
                  dtype=np.uint32)
    say("search mixed per-query parameters")
    ref = orc.search(P["bv"], po, pn, P["qv"], P["seeds"], kq, eq, pq, k_stride=20)
    A = api()
    r = A.search(gpu_vectors(P["x"], orc.L2SQ), gpu_graph(po, pn), gpu_vectors(P["q"], orc.L2SQ),
                 to_dev(P["seeds"]), k=to_dev(kq), k_stride=20, eps=to_dev(eq),
                 ep=torch.from_numpy(pq.astype(np.int64)).to(dev()))
    torch.cuda.synchronize()
    assert np.array_equal(host(r.ids), ref["ids"])
    assert np.array_equal(host(r.dc), ref["dc"])
    assert np.array_equal(host(r.hops), ref["hops"])


def _locality_order_reference(bv, pivots):
    """The hierarchical locality order written out with the oracle's top-1:
    levels of every 10th pivot up to at most 16; each level (and finally the
    rows) sorted by (position of the nearest pivot of the ordered level above,
    own position)."""
    levels = [np.asarray(pivots, dtype=np.int32)]
    while len(levels[-1]) > 16:
        levels.append(levels[-1][::10])
    ordered = levels[-1]
    for lv in reversed(levels[:-1]):
        nn, _ = orc.topk(bv, bv, 1, q_rows=lv, cand=ordered)
        pos = {int(v): j for j, v in enumerate(ordered)}
        key = np.array([pos[int(v)] for v in nn[:, 0]])
        ordered = lv[np.lexsort((np.arange(len(lv)), key))]
    nn, _ = orc.topk(bv, bv, 1, cand=ordered)
    pos = {int(v): j for j, v in enumerate(ordered)}
    key = np.array([pos[int(v)] for v in nn[:, 0]])
    return np.lexsort((np.arange(len(key)), key)).astype(np.int32)


def test_locality_order_gather_and_id_map():
    """The locality order against its definition (the oracle's top-1 by
    (distance, id) at every level); rows gather exactly; an id map rewrites
    only the output ids."""
    P = c1_problem()
    A, Lb = api(), L()
    say("locality order")
    B = gpu_vectors(P["x"], orc.L2SQ)
    perm = host(A.locality_order(B, to_dev(P["piv"])))
    assert len(P["piv"]) > 160            # three levels
    assert np.array_equal(perm, _locality_order_reference(P["bv"], P["piv"]))
    # fewer than 17 pivots: one level, rows by (nearest pivot's position, row)
    few = P["piv"][:12][::-1].copy()
    perm12 = host(A.locality_order(B, to_dev(few)))
    nn, _ = orc.topk(P["bv"], P["bv"], 1, cand=few)
    pos = {int(v): j for j, v in enumerate(few)}
    want = np.lexsort((np.arange(len(perm12)), [pos[int(v)] for v in nn[:, 0]]))
    assert np.array_equal(perm12, want)
    xg = host(A.gather_rows(to_dev(P["x"]), to_dev(perm)))
    assert np.array_equal(xg, P["x"][perm])
    po, pn, _ = P["pa"]
    G, Q, S = gpu_graph(po, pn), gpu_vectors(P["q"], orc.L2SQ), to_dev(P["seeds"])
    r0 = A.search(B, G, Q, S, k=10, eps=0.05)
    r1 = A.search(B, G, Q, S, k=10, eps=0.05, id_map=to_dev(perm.astype(np.int32)))
    torch.cuda.synchronize()
    i0, i1 = host(r0.ids), host(r1.ids)
    assert np.array_equal(np.where(i0 >= 0, perm[np.maximum(i0, 0)], -1), i1)
    assert np.array_equal(host(r0.dists), host(r1.dists))


def test_fp8_scale_in_row():
    """FP8 rows that carry their scale in the last 4 bytes: the same codes
    and scale as the separate array, and the same search results."""
    F = _float_problem("f32l2")
    A, Lb = api(), L()
    say("fp8 with the scale in the row")
    x = to_dev(F["x"])
    sep = A.encode(x, Lb.FP8_E4M3, Lb.L2SQ)
    inr = A.encode(x, Lb.FP8_E4M3, Lb.L2SQ, scale_in_row=True)
    dim = F["x"].shape[1]
    assert inr.scale is None and inr.pitch == A.fp8_inrow_pitch(dim)
    cs, ci = host(sep.data), host(inr.data)
    assert np.array_equal(ci[:, :dim], cs[:, :dim])
    assert np.all(ci[:, dim:inr.pitch - 4] == 0)
    assert np.array_equal(ci[:, inr.pitch - 4:].copy().view(np.float32)[:, 0], host(sep.scale))
    G = gpu_graph(F["off"], F["nb"])
    Q = gpu_vectors(F["q"], F["metric"])
    outs = []
    for rows in (sep, inr):
        r = A.search(rows, G, Q, to_dev(F["seeds"]), k=10, eps=0.1)
        torch.cuda.synchronize()
        outs.append((host(r.ids), host(r.dists), host(r.dc)))
    for a_, b_ in zip(*outs):
        assert np.array_equal(a_, b_)


def test_search_padded_rows():
    """Rows padded past the 16-byte pitch (to whole cache lines) give the
    same results: u8 bit-exact against the oracle, f16 identical to the
    unpadded rows."""
    P = c1_problem()
    po, pn, _ = P["pa"]
    A, Lb = api(), L()
    say("search with padded rows")
    Bp = A.Vectors.from_tensor(to_dev(P["x"]), Lb.L2SQ, pitch=256)
    assert Bp.pitch == 256
    r = A.search(Bp, gpu_graph(po, pn), gpu_vectors(P["q"], orc.L2SQ), to_dev(P["seeds"]),
                 k=10, eps=0.1)
    ref = orc.search(P["bv"], po, pn, P["qv"], P["seeds"], 10, 0.1)
    torch.cuda.synchronize()
    _assert_exact(r, ref, 10)
    F = _float_problem("f32cos")
    G = gpu_graph(F["off"], F["nb"])
    Q = gpu_vectors(F["q"], F["metric"])
    outs = []
    for pitch in (None, 256):
        lp = A.encode(to_dev(F["x"]), Lb.F16, Lb.COSINE, pitch=pitch)
        rr = A.search(lp, G, Q, to_dev(F["seeds"]), k=10, eps=0.1)
        torch.cuda.synchronize()
        outs.append((host(rr.ids), host(rr.dists), host(rr.dc)))
    for a_, b_ in zip(*outs):
        assert np.array_equal(a_, b_)
    # the top-k (kNN build, ground truth, seeds) on padded rows is unchanged
    Bf = A.Vectors.from_tensor(to_dev(F["x"]), Lb.COSINE)
    Bfp = A.Vectors.from_tensor(to_dev(F["x"]), Lb.COSINE, pitch=512)
    for k in (8, 74):
        i0, d0 = A.topk(Q, Bf, k)
        i1, d1 = A.topk(Q, Bfp, k)
        assert np.array_equal(host(i0), host(i1)) and np.array_equal(host(d0), host(d1))


@pytest.mark.parametrize("per_query,shape", [(False, None), (True, None),
                                               (True, dict(s_capacity=64, visited_log2=8))])
def test_search_dc_budget(per_query, shape):
    """Distance-computation budget: ids, distances, counts and expansions equal
    the oracle's with the same budget; the flag marks budget stops only."""
    P = c1_problem()
    po, pn, _ = P["pa"]
    nq = len(P["q"])
    g = np.random.default_rng(11)
    full = orc.search(P["bv"], po, pn, P["qv"], P["seeds"], 10, 0.2, orc.INF_EP)
    if per_query:
        frac = g.choice([-1.0, 0.0, 0.1, 0.3, 0.5, 0.9, 1.0, 2.0], nq)
        md = np.where(frac < 0, 0, np.maximum(1, frac * full["dc"])).astype(np.int32)
    else:
        md = int(np.median(full["dc"]))
    say("search distance budget", per_query, shape)
    ref = orc.search(P["bv"], po, pn, P["qv"], P["seeds"], 10, 0.2, orc.INF_EP, max_dc=md)
    A = api()
    cfg = A.launch_config(**shape) if shape else None
    r = A.search(gpu_vectors(P["x"], orc.L2SQ), gpu_graph(po, pn), gpu_vectors(P["q"], orc.L2SQ),
                 to_dev(P["seeds"]), k=10, eps=0.2,
                 max_dc=to_dev(md) if per_query else md, launch=cfg)
    torch.cuda.synchronize()
    _assert_exact(r, ref, 10)
    b = np.broadcast_to(np.asarray(md), (nq,))
    stopped = (host(r.flags) & L().QF_BUDGET) != 0
    assert np.all(ref["dc"][stopped] >= b[stopped])
    # a budget that was never reached changes nothing
    same = (b <= 0) | (b > full["dc"])
    assert not np.any(stopped & same)
    assert np.array_equal(ref["ids"][same], full["ids"][same])
    assert np.any(stopped)


@pytest.mark.parametrize("probe,shape", [(1, None), (3, None), (3, dict(s_capacity=64))])
def test_two_phase_features(probe, shape):
    """Features after `probe` expansions equal the oracle's, also when the
    candidate set spills during the probe (64 on-chip slots)."""
    P = c1_problem()
    off, nb, _ = P["sa"]
    A = api()
    say("two-phase features probe", probe, shape)
    ref = orc.search(P["bv"], off, nb, P["qv"], P["seeds"], 10, 0.05, 40, eps1=np.inf, ep1=100,
                     want_features=True, probe_hops=probe)
    cfg = A.launch_config(**shape) if shape else None
    r = A.search(gpu_vectors(P["x"], orc.L2SQ), gpu_graph(off, nb), gpu_vectors(P["q"], orc.L2SQ),
                 to_dev(P["seeds"]), k=10, eps=0.05, ep=40, two_phase=True, ep_first=100,
                 probe_hops=probe, want_features=True, launch=cfg)
    torch.cuda.synchronize()
    assert np.array_equal(host(r.ids), ref["ids"])
    assert np.array_equal(host(r.dc), ref["dc"])
    assert np.array_equal(host(r.hops), ref["hops"])
    assert np.array_equal(host(r.features).astype(np.float64), ref["feat"])


def _random_predictor(A, T, mode, g, feat, b2, **kw):
    """Random weights; features z-scored with the statistics of `feat`
    (oracle features of the same queries) so the outputs spread."""
    H = 64
    x = orc.feature_transform(feat, orc.L2SQ)
    w1 = torch.from_numpy(g.standard_normal((H, 14)).astype(np.float32) * 0.3).to(dev())
    w2 = torch.from_numpy(g.standard_normal((T, H)).astype(np.float32) * 0.1).to(dev())
    return A.Predictor(A.to_bf16_bits(w1), to_dev(np.zeros(H, np.float32)), A.to_bf16_bits(w2),
                       to_dev(np.asarray(b2, np.float32)), to_dev(x.mean(0).astype(np.float32)),
                       to_dev((x.std(0) + 1e-3).astype(np.float32)), mode=mode, **kw)


@pytest.mark.parametrize("mode", ["log_eps", "curve"])
def test_predictor_replay(mode):
    """The search with a predictor equals the oracle replayed with the range
    and e_p the kernel reports for each query."""
    P = c1_problem()
    po, pn, _ = P["pa"]
    A, Lb = api(), L()
    g = np.random.default_rng(7)
    say("predictor replay", mode)
    feat = orc.search(P["bv"], po, pn, P["qv"], P["seeds"], 10, 0.0, orc.INF_EP, eps1=np.inf,
                      ep1=64, probe_hops=2, want_features=True)["feat"]
    if mode == "log_eps":
        pred = _random_predictor(A, 3, Lb.PRED_LOG_EPS, g, feat, [-1.5, -1.2, -1.0], head=1,
                                 eps_min=0.0, eps_max=0.3, e0=30.0, we=20.0)
    else:
        cand = to_dev(np.array([0.0, 0.02, 0.05, 0.1], np.float32))
        lam = to_dev(10.0 ** g.uniform(-3, 0, len(P["q"])).astype(np.float32))
        pred = _random_predictor(A, 8, Lb.PRED_CURVE, g, feat,
                                 [0.5, 0.6, 0.8, 0.9, 5.0, 5.2, 5.5, 6.0], eps_min=0.0,
                                 eps_max=0.3, e0=30.0, we=20.0, eps_cand=cand, lam=1e-3,
                                 lambda_per_query=lam)
    r = A.search(gpu_vectors(P["x"], orc.L2SQ), gpu_graph(po, pn), gpu_vectors(P["q"], orc.L2SQ),
                 to_dev(P["seeds"]), k=10, eps=0.0, ep=orc.INF_EP, two_phase=True, ep_first=64,
                 predictor=pred, probe_hops=2)
    torch.cuda.synchronize()
    eps_used = host(r.eps_used)
    ep_used = host(r.ep_used).astype(np.uint32)
    assert np.all((eps_used >= 0) & (eps_used <= 0.3))
    assert len(np.unique(eps_used)) > 1
    if mode == "curve":
        assert set(np.unique(eps_used).tolist()) <= {np.float32(v) for v in (0.0, 0.02, 0.05, 0.1)}
    ref = orc.search(P["bv"], po, pn, P["qv"], P["seeds"], 10, eps_used, ep_used, eps1=np.inf,
                     ep1=64, probe_hops=2)
    assert np.array_equal(host(r.ids), ref["ids"])
    assert np.array_equal(host(r.dc), ref["dc"])
    assert np.array_equal(host(r.hops), ref["hops"])


def _float_problem(kind, n=6000, nq=60, k=10):
    metric = orc.COS if kind == "f32cos" else orc.L2SQ
    cfg = dg.scaled(dg.PRESETS["c3" if kind == "f32cos" else "c5"], n, nq, n_clusters=12)
    x, q = dg.base(cfg), dg.queries(cfg)
    bv, qv = orc.Vectors.from_array(x, metric), orc.Vectors.from_array(q, metric)
    knn, kd = orc.knn_graph(bv, 20)
    off, nb, ln = orc.adjust_degree(knn, kd, 8, 16)
    off, nb, ln = orc.adjust_path(off, nb, ln)
    seeds, _ = orc.topk(qv, bv, 8, cand=dg.pivots(cfg, 256))
    return dict(metric=metric, x=x, q=q, bv=bv, qv=qv, off=off, nb=nb, seeds=seeds, cfg=cfg)


@pytest.mark.parametrize("kind", ["f32cos", "f32l2"])
def test_search_float_margin_rule(kind):
    F = _float_problem(kind)
    A = api()
    G = gpu_graph(F["off"], F["nb"])
    for eps in (0.0, 0.05, 0.2):
        say("search float", kind, eps)
        ref = orc.search(F["bv"], F["off"], F["nb"], F["qv"], F["seeds"], 10, eps)
        r = A.search(gpu_vectors(F["x"], F["metric"]), G, gpu_vectors(F["q"], F["metric"]),
                     to_dev(F["seeds"]), k=10, eps=eps)
        ok, info = margin_ok(ref, host(r.ids), host(r.dists), ref["margin"])
        assert ok, f"query {info} differs beyond the margin"
        say("queries whose id sets differ (all tie-sensitive):", info)
        assert info <= 0.1 * len(F["q"]), f"{info} queries differ"
        gd, rd = host(r.dists), ref["dists"]
        same = np.array([set(host(r.ids)[i]) == set(ref["ids"][i]) for i in range(len(rd))])
        fin = np.isfinite(rd) & same[:, None]
        floor = 1e-2 if kind == "f32cos" else 0.0
        assert np.all(np.abs(gd[fin] - rd[fin]) <= 1e-4 * np.maximum(np.abs(rd[fin]), floor) + 1e-6)


@pytest.mark.parametrize("dt", ["f16", "bf16", "fp8"])
def test_search_low_precision_against_decoded_oracle(dt):
    F = _float_problem("f32cos" if dt != "fp8" else "f32l2")
    A, Lb = api(), L()
    ldt = {"f16": Lb.F16, "bf16": Lb.BF16, "fp8": Lb.FP8_E4M3}[dt]
    odt = {"f16": orc.F16, "bf16": orc.BF16, "fp8": orc.FP8}[dt]
    say("search low precision", dt)
    lp = A.encode(to_dev(F["x"]), ldt, Lb.COSINE if F["metric"] == orc.COS else Lb.L2SQ)
    codes = host(lp.data)
    scale = host(lp.scale) if lp.scale is not None else None
    lbv = orc.Vectors(codes, odt, F["metric"], dim=F["x"].shape[1], scale=scale)
    G = gpu_graph(F["off"], F["nb"])
    for eps in (0.0, 0.1):
        ref = orc.search(lbv, F["off"], F["nb"], F["qv"], F["seeds"], 10, eps)
        r = A.search(lp, G, gpu_vectors(F["q"], F["metric"]), to_dev(F["seeds"]), k=10, eps=eps)
        ok, info = margin_ok(ref, host(r.ids), host(r.dists), ref["margin"])
        assert ok, f"query {info} differs beyond the margin"
        # with a rerank from the f32 rows the returned distances are exact f32 ones
        rr = A.search(lp, G, gpu_vectors(F["q"], F["metric"]), to_dev(F["seeds"]), k=10, eps=eps,
                      rerank_base=gpu_vectors(F["x"], F["metric"]), pool_factor=4)
        ri, rd = host(rr.ids), host(rr.dists)
        for qi in range(len(F["q"])):
            for t in range(10):
                if ri[qi, t] < 0:
                    continue
                exact = orc.lib().or_dist(F["bv"].ref, int(ri[qi, t]), F["qv"].ref, qi)
                assert abs(rd[qi, t] - exact) <= 1e-5 * max(1.0, abs(exact))
        # recall against the exact f32 neighbours: the GPU's low-precision
        # search is as good as the oracle's on the same codes, and the rerank
        # does not lose any of it
        gt_ids, _ = orc.topk(F["qv"], F["bv"], 10)
        rec = lambda ids: np.mean([len(set(a[a >= 0].tolist()) & set(b.tolist())) / 10.0
                                   for a, b in zip(ids, gt_ids)])
        rec_gpu, rec_orc, rec_rr = rec(host(r.ids)), rec(ref["ids"]), rec(ri)
        say(dt, "eps", eps, "recall: gpu", rec_gpu, "oracle", rec_orc, "reranked", rec_rr)
        assert rec_gpu >= rec_orc - 0.02
        assert rec_rr >= rec_gpu - 1e-9


@pytest.mark.parametrize("dim,kind", [(37, "f32cos"), (130, "f32l2")])
def test_fused_rerank_odd_dims_ignores_row_padding(dim, kind):
    """The fused rerank reads its f32 rows and the query in 16-byte pieces and
    counts components past dim as zero: with rows and queries whose padding
    holds garbage (dim 37: a partial last piece; dim 130: two rounds of
    pieces and a partial one) the results equal those over zero padding, and
    every returned distance is the exact distance of its id."""
    A, Lb = api(), L()
    metric = orc.COS if kind == "f32cos" else orc.L2SQ
    lm = Lb.COSINE if kind == "f32cos" else Lb.L2SQ
    x = dg.random_vectors(3000, dim, kind, 31 + dim)
    q = dg.random_vectors(60, dim, kind, 32 + dim)
    say("fused rerank, padding, dim", dim, kind)
    B = gpu_vectors(x, metric)
    ids, d = A.build_knn(B, 16)
    graph = A.adjust_path(A.adjust_degree(ids, d, B.dtype, lm, 8, 16), B.dtype, lm)
    Q = gpu_vectors(q, metric)
    seeds, _ = A.topk(Q, B, 8)
    lp = A.encode(B.data[:, :dim].contiguous(), Lb.F16, lm)

    def padded(v, fill):
        cols = (dim + 3) // 4 * 4 + 4              # at least one padding column
        buf = torch.full((v.shape[0], cols), fill, dtype=torch.float32, device=dev())
        buf[:, :dim] = to_dev(v)
        return A.Vectors(buf, Lb.F32, lm, dim)

    out = {}
    for fill in (0.0, 7.5):
        r = A.search(lp, graph, padded(q, fill), seeds, k=10, eps=0.1,
                     rerank_base=padded(x, fill), pool_factor=4)
        out[fill] = (host(r.ids), host(r.dists))
    assert np.array_equal(out[0.0][0], out[7.5][0])
    assert np.array_equal(out[0.0][1], out[7.5][1])
    bv, qv = orc.Vectors.from_array(x, metric), orc.Vectors.from_array(q, metric)
    gi, gd = out[7.5]
    assert (gi >= 0).all()
    for qi in range(len(q)):
        for t in range(10):
            exact = orc.lib().or_dist(bv.ref, int(gi[qi, t]), qv.ref, qi)
            assert abs(gd[qi, t] - exact) <= 1e-5 * max(1.0, abs(exact))


def test_rerank_standalone_matches_oracle():
    say("rerank")
    A = api()
    x = dg.random_vectors(500, 100, "f32cos", 21)
    q = dg.random_vectors(30, 100, "f32cos", 22)
    g = np.random.default_rng(1)
    pool = np.stack([g.choice(500, 200, replace=False) for _ in range(30)]).astype(np.int32)
    pool[:, -5:] = -1
    bv, qv = orc.Vectors.from_array(x, orc.COS), orc.Vectors.from_array(q, orc.COS)
    rid, rd = orc.rerank(qv, bv, pool, 10)
    for f64 in (True, False):
        ids, d = A.rerank(gpu_vectors(q, orc.COS), gpu_vectors(x, orc.COS), to_dev(pool), 10,
                          use_f64=f64)
        if f64:
            assert np.array_equal(host(ids), rid)
            assert np.allclose(host(d), rd, rtol=0, atol=1e-12)
        else:
            assert np.allclose(host(d), rd, rtol=0, atol=2e-6)


def test_ground_truth_and_recall_against_oracle():
    """The measurement path: exact top-k of float rows (f32 screen of k+64,
    fp64 rerank) against the oracle's fp64 brute force, with more rows than
    one tile and a ragged tail; recall@k of that result against itself is 1,
    and the library's recall by ids agrees with the oracle's tie-tolerant
    recall on a perturbed result."""
    say("ground truth")
    A = api()
    from paper_1810_07355_amd import learned as LR
    for kind, metric in (("f32cos", orc.COS), ("f32", orc.L2SQ)):
        x = dg.random_vectors(3001, 48, kind, 31)
        q = dg.random_vectors(67, 48, kind, 32)
        bv, qv = orc.Vectors.from_array(x, metric), orc.Vectors.from_array(q, metric)
        for k in (1, 10, 100):
            rid, rd = orc.topk(qv, bv, k)
            ids, d = A.ground_truth(gpu_vectors(q, metric), gpu_vectors(x, metric), k)
            gi, gd = host(ids), host(d)
            assert np.array_equal(gi, rid), (kind, k)
            assert np.allclose(gd, rd, rtol=1e-6, atol=1e-7), (kind, k)
            assert np.all(LR.recall_by_ids(gi, rid, k) == 1.0)
            # drop the last true neighbour of every query for the next one out
            if k > 1:
                nxt, nd = orc.topk(qv, bv, k + 1)
                pert = gi.copy()
                pert[:, k - 1] = nxt[:, k]
                pd = rd.copy()
                pd[:, k - 1] = nd[:, k]
                by_ids = LR.recall_by_ids(pert, rid, k)
                tol = orc.recall_at_k(pert, pd, rd, k)
                assert np.allclose(by_ids, (k - 1) / k)
                # ties with the k-th true distance count in the oracle's recall only
                assert np.all(tol >= by_ids - 1e-12)


# ------------------------------------------------------------------- MLP

def test_training_support_against_numpy():
    """The learned range's training steps in the library: column statistics
    (plain and weighted, a constant column taking std 1), z-scoring and the
    fold of the target scaling into the output layer, against numpy in fp64."""
    say("column stats, standardize, fold")
    A = api()
    g = np.random.default_rng(3)
    x = (g.standard_normal((5000, 14)) * g.uniform(0.1, 10, 14) + g.uniform(-5, 5, 14)).astype(np.float32)
    x[:, 3] = 2.5
    w = (g.random((5000, 14)) < 0.3).astype(np.float32)
    xd = x.astype(np.float64)
    for ww in (None, w):
        m, s = A.column_stats(to_dev(x), None if ww is None else to_dev(ww))
        if ww is None:
            mu, sd = xd.mean(0), xd.std(0)
        else:
            tot = ww.sum(0)
            mu = (ww * xd).sum(0) / tot
            sd = np.sqrt((ww * (xd - mu) ** 2).sum(0) / tot)
        sd = np.where(sd < 1e-6, 1.0, sd)
        assert np.allclose(host(m), mu, rtol=2e-6, atol=1e-5)
        assert np.allclose(host(s), sd, rtol=2e-6, atol=1e-6)
    z = A.standardize(to_dev(x), m, s)
    assert np.allclose(host(z), (x - host(m)) / host(s), rtol=1e-5, atol=1e-5)
    W2 = g.standard_normal((6, 64)).astype(np.float32)
    b2 = g.standard_normal(6).astype(np.float32)
    sc = g.uniform(0.5, 2, 6).astype(np.float32)
    sh = g.standard_normal(6).astype(np.float32)
    W2d, b2d = to_dev(W2), to_dev(b2)
    A.mlp_fold_output(W2d, b2d, to_dev(sc), to_dev(sh))
    assert np.allclose(host(W2d), W2 * sc[:, None], rtol=1e-6)
    assert np.allclose(host(b2d), b2 * sc + sh, rtol=1e-6, atol=1e-6)


def test_mlp_forward_backward_adam_against_oracle():
    say("mlp")
    A = api()
    g = np.random.default_rng(5)
    B, F, H, T = 1024, 14, 64, 3
    X = g.standard_normal((B, F)).astype(np.float32)
    Y = g.standard_normal((B, T)).astype(np.float32)
    W = g.uniform(0.5, 1.5, (B, T)).astype(np.float32)
    W1 = (g.standard_normal((H, F)) * 0.3).astype(np.float32)
    b1 = (g.standard_normal(H) * 0.1).astype(np.float32)
    W2 = (g.standard_normal((T, H)) * 0.3).astype(np.float32)
    b2 = (g.standard_normal(T) * 0.1).astype(np.float32)
    _, ref_y = orc.mlp_forward(X, W1, b1, W2, b2)
    ref_loss, ref_g = orc.mlp_loss_grad(X, Y, W1, b1, W2, b2, W)
    dW1, db1, dW2, db2 = [to_dev(a) for a in (W1, b1, W2, b2)]
    y = A.mlp_forward(to_dev(X), dW1, db1, dW2, db2)
    assert np.allclose(host(y), ref_y, rtol=1e-4, atol=1e-5)
    loss, grads = A.mlp_backward(to_dev(X), to_dev(Y), dW1, db1, dW2, db2, w=to_dev(W))
    assert abs(float(host(loss)[0]) - ref_loss) <= 1e-4 * abs(ref_loss)
    for gg, rg in zip(grads, ref_g):
        gg = host(gg).astype(np.float64)
        assert np.linalg.norm(gg - rg) <= 1e-4 * np.linalg.norm(rg)
    # one Adam step
    p = W1.astype(np.float64).copy()
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    orc.adam_step(p, ref_g[0].copy(), m, v, 0.01, 1)
    dp, dm, dv = dW1.clone(), torch.zeros_like(dW1), torch.zeros_like(dW1)
    A.adam_step(dp, to_dev(ref_g[0].astype(np.float32)), dm, dv, 0.01, 1)
    assert np.allclose(host(dp), p, rtol=0, atol=1e-6)
    # feature transform equals the oracle's
    raw = np.abs(g.standard_normal((50, 14))).astype(np.float32) * 1000
    ft = A.feature_transform(to_dev(raw), L().L2SQ)
    assert np.allclose(host(ft), orc.feature_transform(raw, orc.L2SQ), rtol=1e-5, atol=1e-5)


# ----------------------------------------------------- pipeline, autotune

def test_pipeline_graph_replays_match_eager():
    P = c1_problem()
    po, pn, _ = P["pa"]
    A = api()
    B, Q = gpu_vectors(P["x"], orc.L2SQ), gpu_vectors(P["q"], orc.L2SQ)
    G = gpu_graph(po, pn)
    say("pipeline create")
    pl = A.Pipeline(B, G, Q, to_dev(P["piv"]), 8, k=10, eps=0.05, ep=orc.INF_EP)
    ref = orc.search(P["bv"], po, pn, P["qv"], P["seeds"], 10, 0.05)
    for rep in range(3):
        say("pipeline replay", rep)
        req = pl.launch()
        torch.cuda.synchronize()
        assert np.array_equal(host(pl.seeds), P["seeds"])
        assert np.array_equal(host(req.ids), ref["ids"])
        assert np.array_equal(host(req.dc), ref["dc"])
        # eager work in between replays
        _ = A.search(B, G, Q, to_dev(P["seeds"]), k=5, eps=0.0)
        torch.cuda.synchronize()
        req.ids.fill_(-7)
    pl.close()


def test_autotune_picks_a_shape_that_stays_exact():
    P = c1_problem()
    po, pn, _ = P["pa"]
    A = api()
    say("autotune")
    req = A.SearchRequest(gpu_vectors(P["x"], orc.L2SQ), gpu_graph(po, pn),
                          gpu_vectors(P["q"], orc.L2SQ), to_dev(P["seeds"]), k=10, eps=0.1)
    best = req.autotune()
    assert best.lanes_per_row in (4, 8, 16, 32)
    req.run()
    torch.cuda.synchronize()
    ref = orc.search(P["bv"], po, pn, P["qv"], P["seeds"], 10, 0.1)
    assert np.array_equal(host(req.ids), ref["ids"])
    assert np.array_equal(host(req.dc), ref["dc"])


def test_pipeline_low_precision_rows_with_rerank():
    """Seeds come from the f32 rows when the searched rows are f16."""
    F = _float_problem("f32cos")
    A, Lb = api(), L()
    B = gpu_vectors(F["x"], F["metric"])
    Q = gpu_vectors(F["q"], F["metric"])
    lp = A.encode(B.data, Lb.F16, Lb.COSINE)
    G = gpu_graph(F["off"], F["nb"])
    piv = to_dev(dg.pivots(F["cfg"], 256))
    say("pipeline f16 + rerank")
    pl = A.Pipeline(lp, G, Q, piv, 8, k=10, eps=0.05, rerank_base=B, pool_factor=4)
    req = pl.launch()
    torch.cuda.synchronize()
    seeds = host(pl.seeds)
    assert np.array_equal(seeds, F["seeds"])
    eager = A.search(lp, G, Q, to_dev(seeds), k=10, eps=0.05, rerank_base=B, pool_factor=4)
    torch.cuda.synchronize()
    for rep in range(2):
        assert np.array_equal(host(req.ids), host(eager.ids))
        assert np.array_equal(host(req.dists), host(eager.dists))
        req.ids.fill_(-3)
        req = pl.launch()
        torch.cuda.synchronize()
    pl.close()


def test_scheduled_learned_search():
    """Longest-first scheduling changes no result: the order only decides
    which wave takes which query."""
    P = c1_problem()
    po, pn, _ = P["pa"]
    A, Lb = api(), L()
    g = np.random.default_rng(9)
    feat = orc.search(P["bv"], po, pn, P["qv"], P["seeds"], 10, 0.0, orc.INF_EP, eps1=np.inf,
                      ep1=64, probe_hops=1, want_features=True)["feat"]
    cand = to_dev(np.array([0.0, 0.02, 0.05, 0.1], np.float32))
    pred = _random_predictor(A, 8, Lb.PRED_CURVE, g, feat, [0.5, 0.6, 0.8, 0.9, 5.0, 5.2, 5.5, 6.0],
                             eps_min=0.0, eps_max=0.3, e0=30.0, we=20.0, eps_cand=cand, lam=3e-3)
    B, Q, G = gpu_vectors(P["x"], orc.L2SQ), gpu_vectors(P["q"], orc.L2SQ), gpu_graph(po, pn)
    S = to_dev(P["seeds"])
    say("one-pass predictor search")
    one = A.search(B, G, Q, S, k=10, two_phase=True, ep_first=64, predictor=pred)
    say("scheduled predictor search")
    ls = A.LearnedSearch(B, G, Q, S, pred, ep_first=64, k=10)
    req = ls.run()
    torch.cuda.synchronize()
    # the predict-only pass chose the same ranges as the one-pass search
    assert np.array_equal(host(ls.pre.eps_used), host(one.eps_used))
    assert np.array_equal(host(ls.pre.ep_used), host(one.ep_used))
    # the order sorts the predicted costs, longest first
    order = host(ls.order)
    cost = host(ls.pre.cost)
    assert sorted(order.tolist()) == list(range(len(order)))
    assert np.all(np.diff(cost[order]) <= 0)
    # the scheduled search is a plain search with those ranges
    eps_used = host(req.eps_used)
    ep_used = host(req.ep_used).astype(np.uint32)
    ref = orc.search(P["bv"], po, pn, P["qv"], P["seeds"], 10, eps_used, ep_used)
    assert np.array_equal(host(req.ids), ref["ids"])
    assert np.array_equal(host(req.dc), ref["dc"])
    # a budget relative to the predicted cost: the oracle with the budget
    # max(64, int32(factor * cost)) in fp32 gives the same result
    for factor in (0.5, 1.0):
        say("cost-relative budget", factor)
        rb = A.search(B, G, Q, S, k=10, range_from=ls.pre.stats, max_dc_factor=factor)
        torch.cuda.synchronize()
        bud = np.maximum(64, (np.float32(factor) * cost.astype(np.float32)).astype(np.int64))
        bud = np.minimum(bud, 2 ** 31 - 1).astype(np.int32)
        refb = orc.search(P["bv"], po, pn, P["qv"], P["seeds"], 10, eps_used, ep_used, max_dc=bud)
        assert np.array_equal(host(rb.ids), refb["ids"])
        assert np.array_equal(host(rb.dc), refb["dc"])
        assert np.array_equal(host(rb.hops), refb["hops"])
    # unordered run of the same ranges gives the same result
    plain = A.search(B, G, Q, S, k=10, range_from=ls.pre.stats)
    torch.cuda.synchronize()
    assert np.array_equal(host(plain.ids), host(req.ids))
    # graph pipeline of the three steps equals the eager run
    say("learned pipeline")
    pl = A.Pipeline(B, G, Q, to_dev(P["piv"]), 8, k=10, two_phase=True, ep_first=64,
                    predictor=pred)
    for rep in range(2):
        out = pl.launch()
        torch.cuda.synchronize()
        assert np.array_equal(host(out.ids), host(req.ids))
        assert np.array_equal(host(out.dc), host(req.dc))
        out.ids.fill_(-5)
    pl.close()
    # the single-pass pipeline equals the one-pass search
    pl1 = A.Pipeline(B, G, Q, to_dev(P["piv"]), 8, k=10, two_phase=True, ep_first=64,
                     predictor=pred, single_pass=True)
    for rep in range(2):
        out = pl1.launch()
        torch.cuda.synchronize()
        assert np.array_equal(host(out.ids), host(one.ids))
        assert np.array_equal(host(out.dc), host(one.dc))
    pl1.close()
