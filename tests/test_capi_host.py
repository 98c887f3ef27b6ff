"""The C-ABI library loads, exports every function include/onng.h declares,
its ctypes mirror has the C layout, and argument errors come back as status
codes without touching a device.  CPU only."""
import ctypes as C
import os
import re
import subprocess

import numpy as np

import pytest

from paper_1810_07355_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "onng.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(onng_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    return L.load()


def test_every_declared_function_is_exported(lib):
    names = _declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(L.PROTOS), set(names) ^ set(L.PROTOS)


def test_struct_layout_matches_c(tmp_path):
    prog = tmp_path / "layout.c"
    prog.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "onng.h"
#define P(T) printf(#T " %zu\n", sizeof(T));
#define O(T, f) printf(#T "." #f " %zu\n", offsetof(T, f));
int main(void) {
  P(onng_vectors) P(onng_graph) P(onng_predictor) P(onng_launch_config) P(onng_search_params)
  P(onng_query_stats)
  O(onng_vectors, pitch_bytes) O(onng_vectors, metric)
  O(onng_predictor, head) O(onng_predictor, we) O(onng_predictor, mode)
  O(onng_predictor, eps_cand) O(onng_predictor, lambda_per_query)
  O(onng_search_params, eps_per_query) O(onng_search_params, ep_per_query)
  O(onng_search_params, two_phase) O(onng_search_params, predictor)
  O(onng_search_params, rerank_base) O(onng_search_params, pool_factor)
  O(onng_search_params, launch) O(onng_search_params, probe_hops)
  return 0;
}
''')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(prog), "-o",
                    str(exe)], check=True)
    out = dict(l.rsplit(" ", 1) for l in subprocess.run([str(exe)], capture_output=True,
                                                           text=True, check=True).stdout.split("\n") if l)
    ct = {"onng_vectors": L.Vectors_t, "onng_graph": L.Graph_t, "onng_predictor": L.Predictor_t,
          "onng_launch_config": L.LaunchConfig_t, "onng_search_params": L.SearchParams_t}
    for name, cls in ct.items():
        assert C.sizeof(cls) == int(out[name]), name
    assert int(out["onng_query_stats"]) == 32
    for key, val in out.items():
        if "." in key:
            sname, field = key.split(".")
            field = {"lambda": "lambda_"}.get(field, field)
            assert getattr(ct[sname], field).offset == int(val), key


def test_status_strings_and_version(lib):
    assert lib.onng_version() >= 10000
    assert lib.onng_status_string(0) == b"ok"
    assert lib.onng_status_string(-4) == b"workspace too small"


def _vec(n, dim, dtype=L.U8, metric=L.L2SQ, pitch=None, data=0x1000):
    pitch = pitch if pitch is not None else (dim + 15) // 16 * 16
    return L.Vectors_t(data, None, n, dim, dtype, pitch, metric, 0)


def test_argument_errors_without_device(lib):
    v = _vec(100, 128)
    ids = C.c_void_p(0x2000)
    # null base
    assert lib.onng_build_knn(None, 10, ids, ids, ids, 1 << 20, None) == L.ERR_INVALID_ARG
    assert b"base" in lib.onng_last_error()
    # k > n - 1
    assert lib.onng_build_knn(C.byref(v), 100, ids, ids, ids, 1 << 20, None) == L.ERR_INVALID_ARG
    # pitch not a multiple of 16
    bad = _vec(100, 100, pitch=100)
    assert lib.onng_build_knn(C.byref(bad), 5, ids, ids, ids, 1 << 20, None) == L.ERR_INVALID_ARG
    # cosine on u8 is not provided
    cu = _vec(100, 128, metric=L.COSINE)
    assert lib.onng_build_knn(C.byref(cu), 5, ids, ids, ids, 1 << 20, None) == L.ERR_UNSUPPORTED
    # misaligned data
    mis = _vec(100, 128, data=0x1004)
    assert lib.onng_build_knn(C.byref(mis), 5, ids, ids, ids, 1 << 20, None) == L.ERR_INVALID_ARG
    # FP8 without scale
    f8 = _vec(10, 96, dtype=L.FP8_E4M3)
    assert lib.onng_build_knn(C.byref(f8), 5, ids, ids, ids, 1 << 20, None) == L.ERR_INVALID_ARG


def test_search_argument_errors_without_device(lib):
    base = _vec(100, 128)
    q = _vec(5, 128)
    off = C.c_void_p(0x3000)
    g = L.Graph_t(0x3000, 0x4000, None, 100, 10)
    p = L.SearchParams_t()
    p.k, p.k_stride, p.epsilon, p.e_p = 10, 10, 0.0, L.EP_INF
    seeds = C.c_void_p(0x5000)
    out = C.c_void_p(0x6000)
    # too many seeds
    assert lib.onng_search(C.byref(base), C.byref(g), C.byref(q), seeds, 65, C.byref(p), out,
                           out, out, out, 1 << 30, None) == L.ERR_INVALID_ARG
    # k above k_stride
    p.k = 11
    assert lib.onng_search(C.byref(base), C.byref(g), C.byref(q), seeds, 8, C.byref(p), out,
                           out, out, out, 1 << 30, None) == L.ERR_INVALID_ARG
    p.k = 10
    # graph size differs from base
    g2 = L.Graph_t(0x3000, 0x4000, None, 99, 10)
    assert lib.onng_search(C.byref(base), C.byref(g2), C.byref(q), seeds, 8, C.byref(p), out,
                           out, out, out, 1 << 30, None) == L.ERR_INVALID_ARG
    # f32 queries against u8 rows
    qf = _vec(5, 128, dtype=L.F32, pitch=512)
    assert lib.onng_search(C.byref(base), C.byref(g), C.byref(qf), seeds, 8, C.byref(p), out,
                           out, out, out, 1 << 30, None) == L.ERR_INVALID_ARG
    # predictor without two_phase
    pred = L.Predictor_t()
    p.predictor = C.cast(C.byref(pred), C.c_void_p)
    assert lib.onng_search(C.byref(base), C.byref(g), C.byref(q), seeds, 8, C.byref(p), out,
                           out, out, out, 1 << 30, None) == L.ERR_INVALID_ARG
    assert b"two_phase" in lib.onng_last_error()


def test_other_entry_points_validate(lib):
    p = C.c_void_p(0x1000)
    assert lib.onng_encode(p, 10, 0, L.F16, p, 32, None, None) == L.ERR_INVALID_ARG
    assert lib.onng_encode(p, 10, 8, L.FP8_E4M3, p, 16, None, None) == L.ERR_INVALID_ARG
    assert lib.onng_mlp_forward(p, 4, 3, p, p, 65, p, p, 2, None, p, None) == L.ERR_INVALID_ARG
    assert lib.onng_adam_step(p, p, p, p, 10, 0.1, 0.9, 0.99, 1e-8, 0, None) == L.ERR_INVALID_ARG
    assert lib.onng_adjust_degree(None, None, 10, 4, L.U8, L.L2SQ, 2, 2, p, p, p, 80, None, p,
                                  1 << 20, None) == L.ERR_INVALID_ARG
    nnz = C.c_int64(0)
    assert lib.onng_adjust_degree(p, p, 10, 4, L.U8, L.L2SQ, 2, 2, p, p, p, 80, C.byref(nnz), p,
                                  16, None) == L.ERR_WORKSPACE
    assert lib.onng_pipeline_destroy(None) == L.OK
    assert lib.onng_column_stats(p, None, -1, 3, p, p, None) == L.ERR_INVALID_ARG
    assert lib.onng_column_stats(p, None, 10, 3, None, p, None) == L.ERR_INVALID_ARG
    assert lib.onng_standardize(p, 10, -2, p, p, p, None) == L.ERR_INVALID_ARG
    assert lib.onng_mlp_fold_output(p, None, 3, 4, p, p, None) == L.ERR_INVALID_ARG


def test_degree_loss_in_the_library(lib):
    """onng_degree_loss (Equation 2 from samples, host code in the library):
    log10 C linear in p integrates exactly by the trapezoid (L = the mean of
    the end values); unsorted samples give the same L; a zero precision span
    gives the mean of log10 C; bad inputs are rejected."""
    import ctypes as Cc
    out = Cc.c_double(0.0)
    p = np.linspace(0.90, 0.98, 10)
    c = 10.0 ** (2.0 + 10.0 * (p - 0.90))            # log10 C = 2 + 10 (p - 0.9)
    perm = np.random.default_rng(1).permutation(10)
    pa, ca = np.ascontiguousarray(p[perm]), np.ascontiguousarray(c[perm])
    assert lib.onng_degree_loss(pa.ctypes.data, ca.ctypes.data, 10,
                                    Cc.byref(out)) == L.OK
    assert abs(out.value - (2.0 + 2.8) / 2) < 1e-12
    flat = np.full(4, 0.95)
    cc = np.array([10.0, 100.0, 1000.0, 10000.0])
    assert lib.onng_degree_loss(flat.ctypes.data, cc.ctypes.data, 4,
                                    Cc.byref(out)) == L.OK
    assert abs(out.value - 2.5) < 1e-12
    bad = np.array([1.0, 0.0])
    assert lib.onng_degree_loss(flat.ctypes.data, bad.ctypes.data, 2,
                                    Cc.byref(out)) == L.ERR_INVALID_ARG
    assert lib.onng_degree_loss(flat.ctypes.data, cc.ctypes.data, 0,
                                    Cc.byref(out)) == L.ERR_INVALID_ARG


def test_recall_by_ids_definition():
    """recall@k by ids: the share of the k true neighbour ids among the first
    k returned ids; padding (-1) never counts, order does not matter."""
    from paper_1810_07355_amd import learned as LR
    gt = np.array([[3, 1, 4, 9], [2, 7, 1, 8]], dtype=np.int32)
    res = np.array([[4, 3, 5, 1], [-1, 8, 7, 2]], dtype=np.int32)
    assert np.allclose(LR.recall_by_ids(res, gt, 4), [3 / 4, 3 / 4])
    assert np.allclose(LR.recall_by_ids(res, gt, 2), [1 / 2, 0.0])
    assert np.allclose(LR.recall_by_ids(gt, gt, 4), [1.0, 1.0])
    g = np.random.default_rng(3)
    a = g.integers(0, 50, size=(20, 10)).astype(np.int32)
    b = np.stack([g.permutation(50)[:10] for _ in range(20)]).astype(np.int32)
    brute = [sum(1 for x in set(a[i].tolist()) if x in set(b[i].tolist())) for i in range(20)]
    # a result with repeated ids counts each repetition (the search never repeats one)
    rep = [sum(1 for x in a[i].tolist() if x in set(b[i].tolist())) for i in range(20)]
    assert np.allclose(LR.recall_by_ids(a, b, 10) * 10, rep)
    assert all(r >= u for r, u in zip(rep, brute))


def test_time_cost_and_curve_targets():
    """The curve heads' time cost: each query's time at each range, scaled so
    that the sweep's total equals its total distance computations (a
    per-query ratio of times is kept); curve targets put the recalls of the
    candidate ranges first, then log(1 + cost)."""
    from paper_1810_07355_amd import learned as LR
    us = np.array([[10.0, 30.0, 0.0], [20.0, 40.0, 100.0]])
    dcs = np.array([[100, 300, 50], [200, 350, 1000]])
    c = LR.time_cost(us, dcs)
    assert c.shape == us.shape
    assert np.isclose(c.sum(), dcs.sum())
    assert np.allclose(c / c.sum(), us / us.sum())
    assert c[0, 2] == 0.0
    rec = np.array([[0.5, 0.9, 1.0], [0.7, 1.0, 1.0]])
    t = LR.curve_targets(rec, c, [1, 0])
    assert t.shape == (3, 4)
    assert np.allclose(t[:, :2], rec[[1, 0]].T)
    assert np.allclose(t[:, 2:], np.log1p(c[[1, 0]].T))
