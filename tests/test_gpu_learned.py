"""What the learned search range gains over the method without it.

On a 200,000-object cosine set of the benchmark's recipe, the curve
predictor is trained with the library's own kernels on sweep labels of
20,000 training queries.  On 2,000 held-out queries it must reach the
same mean recall@10 (0.98) as the best single search range with fewer distance
computations.  Both operating points are found by bisection (the range for
the plain method, lambda for the learned one).  The gain is measured, not
pinned: the paper has no learned range.
"""
import numpy as np
import pytest

from paper_1810_07355_amd import datagen as dg

from gpu_common import api, have_gpu, L, say, to_dev, torch

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not have_gpu(), reason="needs an MI355X GPU")]


def test_learned_range_gain():
    from paper_1810_07355_amd import learned as LR
    A, Lb = api(), L()
    K, NS, TARGET = 10, 8, 0.98
    cfg = dg.scaled(dg.PRESETS["c3"], 200_000, 2000, n_clusters=400, n_train=20_000)
    say("learned gain: building the index")
    B = A.Vectors.from_tensor(to_dev(dg.base(cfg)), Lb.COSINE)
    Q = A.Vectors.from_tensor(to_dev(dg.queries(cfg)), Lb.COSINE)
    T = A.Vectors.from_tensor(to_dev(dg.train_queries(cfg)), Lb.COSINE)
    ids, d = A.build_knn(B, cfg.knn_k)
    g = A.adjust_path(A.adjust_degree(ids, d, Lb.F32, Lb.COSINE, cfg.e_o, cfg.e_i), Lb.F32,
                      Lb.COSINE)
    piv = to_dev(dg.pivots(cfg))
    seeds, _ = A.topk(Q, B, NS, cand=piv)
    tseeds, _ = A.topk(T, B, NS, cand=piv)
    gt = A.ground_truth(Q, B, K)[0].cpu().numpy()
    tgt = A.ground_truth(T, B, K)[0].cpu().numpy()
    grid = [round(0.01 * i, 2) for i in range(0, 21)] + [0.25, 0.3, 0.4, 0.6]
    epf = LR.dynamic_ep(0.11)
    say("learned gain: label sweep")
    recs, dcs, feats = [], [], None
    for i, e in enumerate(grid):
        r = A.SearchRequest(B, g, T, tseeds, k=K, eps=e, ep=LR.dynamic_ep(e), two_phase=True,
                            ep_first=epf, want_features=(i == 0)).run()
        torch.cuda.synchronize()
        if i == 0:
            feats = r.features.clone()
        recs.append(LR.recall_by_ids(r.ids.cpu().numpy(), tgt, K))
        dcs.append(r.dc.cpu().numpy())
    recs, dcs = np.stack(recs), np.stack(dcs)
    cand = [0.08, 0.11, 0.14, 0.17, 0.20, 0.25, 0.40, 0.60]
    idx = [grid.index(c) if c in grid else int(np.argmin(np.abs(np.array(grid) - c)))
           for c in cand]
    say("learned gain: training")
    model = LR.train_targets(feats, LR.curve_targets(recs, dcs, idx), Lb.COSINE, steps=2000)

    def run_plain(e):
        r = A.SearchRequest(B, g, Q, seeds, k=K, eps=e, ep=LR.dynamic_ep(e)).run()
        torch.cuda.synchronize()
        return LR.recall_by_ids(r.ids.cpu().numpy(), gt, K).mean(), r.dc.float().mean().item()

    def run_learned(knob):
        pred = model.predictor(mode=Lb.PRED_CURVE, eps_cand=cand, lam=10.0 ** (-knob),
                               eps_min=0.0, eps_max=1.0, e0=30.0, we=20.0)
        r = A.LearnedSearch(B, g, Q, seeds, pred, ep_first=epf, k=K).run()
        torch.cuda.synchronize()
        return LR.recall_by_ids(r.ids.cpu().numpy(), gt, K).mean(), r.dc.float().mean().item()

    def bisect(fn, lo, hi, iters=12):
        rec, dc = fn(hi)
        assert rec >= TARGET, f"the top of the knob range only reaches recall {rec:.4f}"
        for _ in range(iters):
            mid = 0.5 * (lo + hi)
            r_, d_ = fn(mid)
            if r_ >= TARGET:
                hi, rec, dc = mid, r_, d_
            else:
                lo = mid
        return rec, dc

    rp, dp = bisect(run_plain, 0.0, 1.0)
    rl, dl = bisect(run_learned, 2.0, 9.0)
    say(f"recall {TARGET}: best single range {dp:.0f} distance computations (recall {rp:.4f}), "
        f"learned range {dl:.0f} (recall {rl:.4f}), ratio {dp / dl:.2f}")
    assert rl >= TARGET and rp >= TARGET
    assert dl < 0.9 * dp
