"""ctypes view of include/onng.h: structs, enums and prototypes of libonng.so.

The library is loaded from this package directory only; importing the
binding without a built library raises, there is no fallback."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libonng.so")

OK, ERR_INVALID_ARG, ERR_UNSUPPORTED, ERR_CAPACITY, ERR_WORKSPACE, ERR_DEVICE = 0, -1, -2, -3, -4, -5
U8, F32, F16, BF16, FP8_E4M3 = 0, 1, 2, 3, 4
L2SQ, COSINE = 0, 1
NFEAT = 14
QF_PADDED, QF_SPILLED, QF_CAPACITY, QF_BUDGET = 1, 2, 4, 8
PRED_LOG_EPS, PRED_CURVE = 0, 1
EP_INF = 0xFFFFFFFF

P = C.c_void_p


class Vectors_t(C.Structure):
    _fields_ = [("data", P), ("scale", P), ("n", C.c_int64), ("dim", C.c_int32),
                ("dtype", C.c_int32), ("pitch_bytes", C.c_int64), ("metric", C.c_int32),
                ("us", C.c_float)]


class Graph_t(C.Structure):
    _fields_ = [("offsets", P), ("nbrs", P), ("lens", P), ("n", C.c_int64), ("nnz", C.c_int64)]


class VPTree_t(C.Structure):
    _fields_ = [("node_vp", P), ("node_child", P), ("node_mu", P), ("leaf_seeds", P),
                ("node_capacity", C.c_int64), ("leaf_capacity", C.c_int64),
                ("leaf_size", C.c_int32), ("n_seeds", C.c_int32), ("n_nodes", C.c_int64),
                ("n_leaves", C.c_int64)]


class Predictor_t(C.Structure):
    _fields_ = [("w1_bf16", P), ("b1", P), ("w2_bf16", P), ("b2", P), ("feat_mean", P),
                ("feat_std", P), ("shift", P), ("head_per_query", P), ("head", C.c_int32),
                ("n_features", C.c_int32), ("hidden", C.c_int32), ("n_heads", C.c_int32),
                ("eps_min", C.c_float), ("eps_max", C.c_float), ("e0", C.c_float),
                ("we", C.c_float), ("mode", C.c_int32), ("n_cand", C.c_int32),
                ("eps_cand", P), ("lambda_", C.c_float), ("lambda_per_query", P)]


class LaunchConfig_t(C.Structure):
    _fields_ = [("waves_per_block", C.c_int32), ("lanes_per_row", C.c_int32),
                ("s_capacity", C.c_int32), ("visited_log2", C.c_int32),
                ("pool_capacity", C.c_int32), ("blocks", C.c_int32)]


class SearchParams_t(C.Structure):
    _fields_ = [("k", C.c_int32), ("k_stride", C.c_int32), ("k_per_query", P),
                ("epsilon", C.c_float), ("eps_per_query", P), ("e_p", C.c_uint32),
                ("ep_per_query", P), ("two_phase", C.c_int32), ("ep_first", C.c_uint32),
                ("predictor", P), ("features_out", P), ("rerank_base", P),
                ("pool_factor", C.c_int32), ("launch", P), ("probe_hops", C.c_uint32),
                ("predict_only", C.c_int32), ("range_from", P), ("order", P),
                ("max_dc", C.c_int32), ("max_dc_per_query", P), ("max_dc_factor", C.c_float),
                ("id_map", P), ("single_pass", C.c_int32), ("ws_reuse", C.c_int32)]


# exported symbols and their prototypes (must match include/onng.h)
PROTOS = {
    "onng_build_knn": (C.c_int, [P, C.c_int32, P, P, P, C.c_size_t, P]),
    "onng_topk": (C.c_int, [P, P, P, C.c_int64, C.c_int32, C.c_int32, P, P, P, C.c_size_t, P]),
    "onng_topk_workspace_size": (C.c_size_t, [P, P, C.c_int64, C.c_int32]),
    "onng_adjust_degree": (C.c_int, [P, P, C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                     C.c_int32, P, P, P, C.c_int64, P, P, C.c_size_t, P]),
    "onng_adjust_degree_workspace_size": (C.c_size_t, [C.c_int64, C.c_int32, C.c_int32,
                                                       C.c_int32]),
    "onng_adjust_degree_constrained": (C.c_int, [P, P, C.c_int64, C.c_int32, C.c_int32,
                                                 C.c_int32, C.c_int32, C.c_int32, P, P, P,
                                                 C.c_int64, P, P, C.c_size_t, P]),
    "onng_adjust_degree_constrained_workspace_size": (C.c_size_t, [C.c_int64, C.c_int32,
                                                                   C.c_int32, C.c_int32]),
    "onng_graph_stats": (C.c_int, [P, C.c_int32, C.c_int32, C.c_double, C.c_int32, P, P,
                                   C.c_size_t, P]),
    "onng_graph_stats_workspace_size": (C.c_size_t, [C.c_int64, C.c_int64]),
    "onng_graph_add_edges": (C.c_int, [P, P, P, P, C.c_int64, C.c_int32, C.c_int32, P, P, P,
                                       C.c_int64, P, P, C.c_size_t, P]),
    "onng_graph_add_edges_workspace_size": (C.c_size_t, [C.c_int64, C.c_int64, C.c_int64]),
    "onng_graph_head": (C.c_int, [P, C.c_int32, C.c_int32, C.c_int32, P, P, P]),
    "onng_vptree_build": (C.c_int, [P, P, P, P, C.c_size_t, P]),
    "onng_vptree_build_workspace_size": (C.c_size_t, [C.c_int64]),
    "onng_vptree_seeds": (C.c_int, [P, P, P, P, P, P]),
    "onng_adjust_path": (C.c_int, [P, C.c_int32, C.c_int32, P, P, P, P, P, C.c_size_t, P]),
    "onng_adjust_path_workspace_size": (C.c_size_t, [C.c_int64, C.c_int64]),
    "onng_search": (C.c_int, [P, P, P, P, C.c_int32, P, P, P, P, P, C.c_size_t, P]),
    "onng_search_workspace_size": (C.c_size_t, [P, C.c_int64, P]),
    "onng_search_static": (C.c_int, [P, P, P, P, C.c_int32, P, P, P, P, P]),
    "onng_order_by_cost": (C.c_int, [P, C.c_int64, P, P, C.c_size_t, P]),
    "onng_order_by_cost_workspace_size": (C.c_size_t, [C.c_int64]),
    "onng_locality_order": (C.c_int, [P, P, C.c_int64, P, P, C.c_size_t, P]),
    "onng_locality_order_workspace_size": (C.c_size_t, [P, C.c_int64]),
    "onng_gather_rows": (C.c_int, [P, C.c_int64, P, C.c_int64, P, P]),
    "onng_encode": (C.c_int, [P, C.c_int64, C.c_int32, C.c_int32, P, C.c_int64, P, P]),
    "onng_rerank": (C.c_int, [P, P, P, C.c_int32, C.c_int32, C.c_int32, P, P, P]),
    "onng_mlp_forward": (C.c_int, [P, C.c_int32, C.c_int32, P, P, C.c_int32, P, P, C.c_int32,
                                   P, P, P]),
    "onng_mlp_backward": (C.c_int, [P, P, P, C.c_int32, C.c_int32, P, P, C.c_int32, P, P,
                                    C.c_int32, P, P, P, P, P, P, C.c_size_t, P]),
    "onng_mlp_backward_workspace_size": (C.c_size_t, [C.c_int32, C.c_int32, C.c_int32]),
    "onng_adam_step": (C.c_int, [P, P, P, P, C.c_int64, C.c_float, C.c_float, C.c_float,
                                 C.c_float, C.c_int32, P]),
    "onng_feature_transform": (C.c_int, [P, C.c_int64, C.c_int32, P, P]),
    "onng_column_stats": (C.c_int, [P, P, C.c_int64, C.c_int32, P, P, P]),
    "onng_standardize": (C.c_int, [P, C.c_int64, C.c_int32, P, P, P, P]),
    "onng_mlp_fold_output": (C.c_int, [P, P, C.c_int32, C.c_int32, P, P, P]),
    "onng_degree_loss": (C.c_int, [P, P, C.c_int32, P]),
    "onng_autotune_search": (C.c_int, [P, P, P, P, C.c_int32, P, P, P, P, P, C.c_size_t, P, P]),
    "onng_pipeline_create": (C.c_int, [P, P, P, P, C.c_int64, C.c_int32, P, P, P, P, P, P,
                                       C.c_size_t, P, P]),
    "onng_pipeline_workspace_size": (C.c_size_t, [P, P, C.c_int64, C.c_int32, P]),
    "onng_pipeline_launch": (C.c_int, [P, P]),
    "onng_pipeline_destroy": (C.c_int, [P]),
    "onng_status_string": (C.c_char_p, [C.c_int]),
    "onng_last_error": (C.c_char_p, []),
    "onng_version": (C.c_int32, []),
}

_lib = None


class OnngError(RuntimeError):
    def __init__(self, fn: str, status: int, msg: str):
        super().__init__(f"{fn} failed with status {status}: {msg}")
        self.status = status


def load(path: str = LIB_PATH) -> C.CDLL:
    """Load libonng.so (built by __graft_entry__.build()); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build the HIP library first "
                          "(python -c 'import __graft_entry__ as g; g.build()')")
    lib = C.CDLL(path)
    for name, (res, args) in PROTOS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(name: str, status: int) -> None:
    if status != OK:
        lib = load()
        raise OnngError(name, status, lib.onng_last_error().decode())


def call(name: str, *args) -> None:
    check(name, getattr(load(), name)(*args))
