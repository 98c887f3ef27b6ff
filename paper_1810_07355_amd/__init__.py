"""MI355X (gfx950) implementation of the degree- and path-adjusted kNN-graph
search of Iwasaki & Miyazaki (arXiv 1810.07355).

The compute path lives in the HIP library libonng.so (C-ABI in
include/onng.h); `api` is its Python binding.  `datagen` holds the seeded
synthetic inputs.  Importing `api` requires the built library."""
import importlib

__all__ = ["api", "datagen"]


def __getattr__(name):
    if name in ("api", "datagen", "build"):
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
