"""Seeded synthetic inputs shared by the HIP path, the oracle and the benchmark.

This module holds random draws only, none of the method's arithmetic.  The
paper evaluates on SIFT (1-byte, 128-d, Euclidean) and GloVe (100-d, angular),
with 1,000 queries and 100,000 training objects per dataset (Section 3,
opening paragraph).  Those datasets are not shipped here.  These generators
produce stand-ins with the same shapes, value ranges and cluster structure.

Every stream comes from numpy PCG64 seeded by
``SeedSequence(18100735, spawn_key=(config_id, stream))`` with
stream 0 = cluster centres, 1 = base vectors, 2 = queries,
3 = training queries, 4 = pivot ids, 5 = per-query mixed parameters,
6 + i = random seeds, 100 + b = further query batches b = 1, 2, ... (distinct
batches that keep several batches of fresh queries in flight), 200 + b their
mixed parameters, 300 the training queries' mixed parameters.

Workloads (sizes in ``PRESETS``):

* ``u8``: SIFT-like.  K equal-weight isotropic Gaussian clusters in 128-d,
  centres uniform in [32, 224], sigma 20, rounded half-to-even and clipped to
  [0, 255].
* ``f32cos``: GloVe-like.  Unit vectors from a von Mises-Fisher-like mixture.
  Directions mu_j are normalised standard normals.  Cluster weights follow
  Zipf(1.1), i.e. proportional to (j+1)^-1.1, which gives the word-frequency
  concentration the paper describes for GloVe (Section 3, dataset
  characteristics).  A point is normalise(mu_j + tau * z) with tau = 0.1.
* ``f32l2``: anisotropic Gaussian mixture with centres N(0, 2^2 I) and
  per-cluster, per-dimension sigma uniform in [0.5, 2].
"""
from __future__ import annotations

import dataclasses

import numpy as np

ROOT_SEED = 18100735


def rng(config_id: int, stream: int) -> np.random.Generator:
    return np.random.Generator(
        np.random.PCG64(np.random.SeedSequence(ROOT_SEED, spawn_key=(config_id, stream))))


@dataclasses.dataclass(frozen=True)
class Preset:
    name: str
    config_id: int
    kind: str              # "u8", "f32cos", "f32l2"
    n_base: int
    n_query: int
    dim: int
    n_clusters: int
    n_train: int = 0
    knn_k: int = 20
    e_o: int = 10
    e_i: int = 30
    search_k: tuple = (10,)
    eps_grid: tuple = (0.0, 0.02, 0.05, 0.1, 0.2)


PRESETS = {
    # 10,000 x 128 u8, 100 clusters: the size the oracle finishes in seconds.
    "c1": Preset("c1", 1, "u8", 10_000, 100, 128, 100, knn_k=20, e_o=10, e_i=30,
                 search_k=(10,), eps_grid=(0.0, 0.02, 0.05, 0.1, 0.2)),
    # 1,000,000 x 128 u8, 1,000 clusters.
    "c2": Preset("c2", 2, "u8", 1_000_000, 10_000, 128, 1000, knn_k=100, e_o=20, e_i=60,
                 search_k=(10, 100),
                 eps_grid=(0.0, 0.005, 0.01, 0.02, 0.03, 0.05, 0.07, 0.1, 0.15, 0.2, 0.3)),
    # 1,000,000 x 100 unit f32, cosine, 2,000 Zipf-weighted clusters.
    "c3": Preset("c3", 3, "f32cos", 1_000_000, 10_000, 100, 2000, n_train=100_000,
                 knn_k=100, e_o=20, e_i=60, search_k=(10,),
                 eps_grid=(0.0, 0.005, 0.01, 0.02, 0.03, 0.05, 0.07, 0.1, 0.15, 0.2, 0.3)),
    # c2's base and queries plus 100,000 training queries.
    "c4": Preset("c4", 2, "u8", 1_000_000, 10_000, 128, 1000, n_train=100_000, knn_k=100,
                 e_o=20, e_i=60, search_k=(10,),
                 eps_grid=(0.0, 0.005, 0.01, 0.02, 0.03, 0.05, 0.07, 0.1, 0.15, 0.2, 0.3)),
    # 10,000,000 x 96 f32 anisotropic mixture, L2.
    "c5": Preset("c5", 5, "f32l2", 10_000_000, 50_000, 96, 10_000, knn_k=64, e_o=20, e_i=60,
                 search_k=(1, 10, 100),
                 eps_grid=(0.0, 0.005, 0.01, 0.02, 0.03, 0.05, 0.07, 0.1, 0.15, 0.2, 0.3)),
}


def scaled(preset: Preset, n_base: int, n_query: int, n_clusters: int | None = None,
           n_train: int | None = None) -> Preset:
    """Same recipe at another size (used for small test cases)."""
    return dataclasses.replace(
        preset, n_base=n_base, n_query=n_query,
        n_clusters=preset.n_clusters if n_clusters is None else n_clusters,
        n_train=preset.n_train if n_train is None else n_train)


def _u8_mixture(cfg: Preset, n: int, stream: int, chunk: int = 1 << 18) -> np.ndarray:
    centres = rng(cfg.config_id, 0).uniform(32.0, 224.0, size=(cfg.n_clusters, cfg.dim))
    g = rng(cfg.config_id, stream)
    labels = g.integers(0, cfg.n_clusters, size=n)
    out = np.empty((n, cfg.dim), dtype=np.uint8)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        z = g.standard_normal(size=(e - s, cfg.dim))
        x = np.rint(centres[labels[s:e]] + 20.0 * z)
        out[s:e] = np.clip(x, 0, 255).astype(np.uint8)
    return out


def _zipf_weights(k: int, a: float = 1.1) -> np.ndarray:
    w = (np.arange(k, dtype=np.float64) + 1.0) ** (-a)
    return w / w.sum()


def _f32cos_mixture(cfg: Preset, n: int, stream: int, tau: float = 0.1,
                    chunk: int = 1 << 18) -> np.ndarray:
    mu = rng(cfg.config_id, 0).standard_normal(size=(cfg.n_clusters, cfg.dim))
    mu /= np.linalg.norm(mu, axis=1, keepdims=True)
    g = rng(cfg.config_id, stream)
    labels = g.choice(cfg.n_clusters, size=n, p=_zipf_weights(cfg.n_clusters))
    out = np.empty((n, cfg.dim), dtype=np.float32)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        x = mu[labels[s:e]] + tau * g.standard_normal(size=(e - s, cfg.dim))
        x /= np.linalg.norm(x, axis=1, keepdims=True)
        out[s:e] = x.astype(np.float32)
    return out


def _f32l2_mixture(cfg: Preset, n: int, stream: int, chunk: int = 1 << 18) -> np.ndarray:
    g0 = rng(cfg.config_id, 0)
    centres = 2.0 * g0.standard_normal(size=(cfg.n_clusters, cfg.dim))
    sigma = g0.uniform(0.5, 2.0, size=(cfg.n_clusters, cfg.dim))
    g = rng(cfg.config_id, stream)
    labels = g.integers(0, cfg.n_clusters, size=n)
    out = np.empty((n, cfg.dim), dtype=np.float32)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        lab = labels[s:e]
        x = centres[lab] + sigma[lab] * g.standard_normal(size=(e - s, cfg.dim))
        out[s:e] = x.astype(np.float32)
    return out


def _vectors(cfg: Preset, n: int, stream: int) -> np.ndarray:
    if cfg.kind == "u8":
        return _u8_mixture(cfg, n, stream)
    if cfg.kind == "f32cos":
        return _f32cos_mixture(cfg, n, stream)
    if cfg.kind == "f32l2":
        return _f32l2_mixture(cfg, n, stream)
    raise ValueError(cfg.kind)


def base(cfg: Preset) -> np.ndarray:
    return _vectors(cfg, cfg.n_base, 1)


def queries(cfg: Preset) -> np.ndarray:
    return _vectors(cfg, cfg.n_query, 2)


def query_batch(cfg: Preset, b: int) -> np.ndarray:
    """Batch b of n_query queries from the query distribution: batch 0 is
    queries(cfg), batch b >= 1 its own stream."""
    return queries(cfg) if b == 0 else _vectors(cfg, cfg.n_query, 100 + b)


def train_queries(cfg: Preset, n: int | None = None) -> np.ndarray:
    return _vectors(cfg, cfg.n_train if n is None else n, 3)


def pivot_count(n_base: int) -> int:
    """P = max(1024, N/100), capped at N (mirrors a tree leaf of <=100 objects)."""
    return int(min(n_base, max(1024, n_base // 100)))


def pivots(cfg: Preset, n_pivots: int | None = None) -> np.ndarray:
    """Seeded uniform sample of base ids, without replacement, ascending."""
    p = pivot_count(cfg.n_base) if n_pivots is None else n_pivots
    ids = rng(cfg.config_id, 4).choice(cfg.n_base, size=p, replace=False)
    return np.sort(ids).astype(np.int32)


def vp_priority(n: int, seed: int = 0) -> np.ndarray:
    """Seeded random ranks 0..n-1 (a permutation), one per base row: the
    vantage-point tree takes a node's lowest-ranked row as its vantage point,
    which makes that choice uniformly random."""
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence(ROOT_SEED, spawn_key=(97, seed))))
    return g.permutation(n).astype(np.uint32)


def random_seeds(cfg: Preset, n_query: int, n_seeds: int, stream_offset: int = 0) -> np.ndarray:
    """Uniformly random seed ids per query (the paper's "rand" seeding)."""
    g = rng(cfg.config_id, 6 + stream_offset)
    return g.integers(0, cfg.n_base, size=(n_query, n_seeds)).astype(np.int32)


def mixed_params(cfg: Preset, n_query: int, ks=(1, 10, 100), targets=(0.9, 0.95, 0.99),
                 stream: int = 5):
    """Per-query (k, target recall) drawn uniformly from the product set
    (stream 5 for the workload's queries, another stream for other batches
    or training queries)."""
    g = rng(cfg.config_id, stream)
    k = np.asarray(ks, dtype=np.int32)[g.integers(0, len(ks), size=n_query)]
    t = np.asarray(targets, dtype=np.float32)[g.integers(0, len(targets), size=n_query)]
    return k, t


def random_vectors(n: int, dim: int, kind: str, seed: int) -> np.ndarray:
    """Small unstructured inputs for edge-case tests."""
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence(ROOT_SEED, spawn_key=(99, seed))))
    if kind == "u8":
        return g.integers(0, 256, size=(n, dim)).astype(np.uint8)
    x = g.standard_normal(size=(n, dim))
    if kind == "f32cos":
        x /= np.linalg.norm(x, axis=1, keepdims=True)
    return x.astype(np.float32)


def random_tie_u8(n: int, dim: int, seed: int, levels: int = 3) -> np.ndarray:
    """u8 vectors with very few distinct values, so equal distances are common."""
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence(ROOT_SEED, spawn_key=(98, seed))))
    return (g.integers(0, levels, size=(n, dim)) * 7).astype(np.uint8)
