"""Shared helpers of the GPU parity tests: device transfer and oracle inputs."""
import functools
import sys

import numpy as np
import pytest

from oracle import oracle as orc
from paper_1810_07355_amd import datagen as dg

torch = pytest.importorskip("torch")


def have_gpu():
    return torch.cuda.is_available()


def api():
    from paper_1810_07355_amd import api as A
    return A


def L():
    from paper_1810_07355_amd import _lib
    return _lib


def dev():
    return torch.device("cuda:0")


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def say(*msg):
    print("[case]", *msg, flush=True)
    sys.stdout.flush()


@functools.lru_cache(maxsize=None)
def c1_problem():
    """C1 (10,000 x 128 u8) with the oracle's kNN, SA and PA graphs and seeds."""
    cfg = dg.PRESETS["c1"]
    x, q = dg.base(cfg), dg.queries(cfg)
    bv, qv = orc.Vectors.from_array(x, orc.L2SQ), orc.Vectors.from_array(q, orc.L2SQ)
    knn, kd = orc.knn_graph(bv, cfg.knn_k)
    sa = orc.adjust_degree(knn, kd, cfg.e_o, cfg.e_i)
    pa = orc.adjust_path(*sa)
    piv = dg.pivots(cfg)
    seeds, _ = orc.topk(qv, bv, 8, cand=piv)
    return dict(cfg=cfg, x=x, q=q, bv=bv, qv=qv, knn=knn, kd=kd, sa=sa, pa=pa, piv=piv,
                seeds=seeds)


def gpu_vectors(x, metric):
    A, Lb = api(), L()
    return A.Vectors.from_tensor(to_dev(x), Lb.L2SQ if metric == orc.L2SQ else Lb.COSINE)


def gpu_graph(off, nb, ln=None, int_len=True):
    A = api()
    lens = None
    if ln is not None:
        lens = to_dev(ln.astype(np.int32) if int_len else ln.astype(np.float32))
    return A.Graph(to_dev(off.astype(np.int64)), to_dev(nb.astype(np.int32)), lens)


def margin_ok(ref, gpu_ids, gpu_d, margin, tol=1e-4):
    """Float parity (margin rule): a query whose oracle decisions all had a
    relative margin >= tol must return the same id set.  Returns (ok, info):
    info is the failing query, or the number of queries whose sets differ
    (all of them tie-sensitive)."""
    differ = 0
    for qi in range(len(gpu_ids)):
        a = set(ref["ids"][qi][ref["ids"][qi] >= 0].tolist())
        b = set(gpu_ids[qi][gpu_ids[qi] >= 0].tolist())
        if a != b:
            if margin[qi] >= tol:
                return False, int(qi)
            differ += 1
    return True, differ


def random_predictor(T, mode, g, feat, b2, metric, H=64, **kw):
    """A predictor with random bf16 weights whose inputs are z-scored with the
    statistics of `feat` (oracle features of the same queries), so that its
    choices spread.  Returns (api.Predictor, dict of the host arrays the
    oracle's predict() takes)."""
    A = api()
    x = orc.feature_transform(feat, metric)
    w1 = torch.from_numpy(g.standard_normal((H, orc.NFEAT)).astype(np.float32) * 0.3).to(dev())
    w2 = torch.from_numpy(g.standard_normal((T, H)).astype(np.float32) * 0.1).to(dev())
    b1 = np.zeros(H, np.float32)
    b2 = np.asarray(b2, np.float32)
    mean = x.mean(0).astype(np.float32)
    std = (x.std(0) + 1e-3).astype(np.float32)
    w1b, w2b = A.to_bf16_bits(w1), A.to_bf16_bits(w2)
    pred = A.Predictor(w1b, to_dev(b1), w2b, to_dev(b2), to_dev(mean), to_dev(std), mode=mode,
                       **kw)
    host_w = dict(w1_bits=host(w1b).view(np.uint16), b1=b1, w2_bits=host(w2b).view(np.uint16),
                  b2=b2, mean=mean, std=std)
    return pred, host_w


def fp8_inrow(A, Lb, x_dev, metric, dim):
    """fp8-e4m3 rows with the scale in each row's last 4 bytes (128-byte
    pitch), as the benchmark stores them; and the oracle's view of the same
    codes (exact decode)."""
    lp = A.encode(x_dev, Lb.FP8_E4M3, Lb.COSINE if metric == orc.COS else Lb.L2SQ,
                  scale_in_row=True, pitch=A.row_pitch(A.fp8_inrow_pitch(dim), Lb.U8, 128))
    codes = host(lp.data)
    scale = np.ascontiguousarray(codes[:, -4:]).view(np.float32).reshape(-1)
    return lp, orc.Vectors(codes, orc.FP8, metric, dim=dim, scale=scale)
