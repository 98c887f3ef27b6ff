"""onng_search_static (no device allocation, static scratch) against
onng_search (caller workspace): same ids, distances and per-query counters,
on two calls in a row, the second with a smaller input.  Collected last so a
failure here cannot hide the other GPU tests."""
import numpy as np
import pytest

from gpu_common import (api, c1_problem, dev, gpu_graph, gpu_vectors, have_gpu, host, say,
                        to_dev)
from oracle import oracle as orc
from paper_1810_07355_amd import datagen as dg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _same(a, b):
    torch.cuda.synchronize()
    assert np.array_equal(host(a.ids), host(b.ids))
    assert np.array_equal(host(a.dists), host(b.dists))
    # every counter but the per-query device time (column 7)
    assert np.array_equal(host(a.stats)[:, :7], host(b.stats)[:, :7])


def test_search_static_matches_workspace_search():
    if not have_gpu():
        pytest.skip("no GPU")
    A = api()
    P = c1_problem()
    po, pn, _ = P["pa"]
    B, G = gpu_vectors(P["x"], orc.L2SQ), gpu_graph(po, pn)
    # 3,000 queries of the c1 mixture: more queries than the static scratch
    # has wave slots at this base size, so the persistent waves loop
    q = dg.train_queries(P["cfg"], 3000)
    Q = gpu_vectors(q, orc.L2SQ)
    seeds, _ = A.topk(Q, B, 8, cand=to_dev(P["piv"]))
    say("static scratch: 3000 queries, k=10, eps=0.1, DA e_p")
    kw = dict(k=10, eps=0.1, ep=orc.dynamic_ep(0.1))
    ref = A.search(B, G, Q, seeds, **kw)
    got = A.search(B, G, Q, seeds, static_scratch=True, **kw)
    _same(ref, got)
    # second call, smaller: 37 queries, k=5, eps=0.02, unlimited e_p
    say("static scratch: 37 queries, k=5, eps=0.02")
    Q2 = gpu_vectors(q[:37], orc.L2SQ)
    s2 = seeds[:37].contiguous()
    ref2 = A.search(B, G, Q2, s2, k=5, eps=0.02)
    got2 = A.search(B, G, Q2, s2, k=5, eps=0.02, static_scratch=True)
    _same(ref2, got2)
    # and the oracle agrees with both (u8: bit-exact)
    oref = orc.search(P["bv"], po, pn, orc.Vectors.from_array(q[:37], orc.L2SQ),
                      host(s2), 5, 0.02)
    assert np.array_equal(host(got2.ids), oref["ids"])
    assert np.array_equal(host(got2.dc), oref["dc"])


def test_search_static_float_rerank():
    """Float rows with the fused f32 rerank, then a smaller call."""
    if not have_gpu():
        pytest.skip("no GPU")
    A, Lb = api(), __import__("paper_1810_07355_amd._lib", fromlist=["_lib"])
    cfg = dg.scaled(dg.PRESETS["c3"], 6000, 200, n_clusters=12)
    x, q = dg.base(cfg), dg.queries(cfg)
    bv, qv = orc.Vectors.from_array(x, orc.COS), orc.Vectors.from_array(q, orc.COS)
    knn, kd = orc.knn_graph(bv, 20)
    off, nb, ln = orc.adjust_path(*orc.adjust_degree(knn, kd, 8, 16))
    B, Q, G = gpu_vectors(x, orc.COS), gpu_vectors(q, orc.COS), gpu_graph(off, nb)
    lp = A.encode(B.data, Lb.FP8_E4M3, Lb.COSINE, scale_in_row=True,
                  pitch=A.row_pitch(A.fp8_inrow_pitch(x.shape[1]), Lb.U8, 128))
    seeds, _ = A.topk(Q, B, 8, cand=to_dev(dg.pivots(cfg, 256)))
    for n in (200, 11):
        say("static scratch: fp8 cosine + rerank,", n, "queries")
        Qn = gpu_vectors(q[:n], orc.COS)
        sn = seeds[:n].contiguous()
        kw = dict(k=10, eps=0.1, rerank_base=B, pool_factor=4)
        _same(A.search(lp, G, Qn, sn, **kw), A.search(lp, G, Qn, sn, static_scratch=True, **kw))
