"""Reverse-mode gradients of data-parallel scalar objectives on MI355X.

The work happens in libpgrad.so (hand-written HIP kernels for gfx950 behind
the C ABI of include/pgrad.h); this package is its thin Python binding.
Importing the package does not load the library; the first call does, and
fails loudly if it was not built.
"""
from __future__ import annotations

import importlib

__all__ = ["MeshObjective", "DenseObjective", "BatchedDense", "MeshBatch", "MeshFn", "DenseFn",
           "BatchedDenseFn", "MeshBatchFn", "Laplace1D", "Program", "ProgramFn", "PgError", "lib"]


def __getattr__(name):
    if name in __all__:
        return getattr(importlib.import_module(__name__ + ".pgrad"), name)
    if name in ("inputs", "pgrad", "build", "autotune"):
        return importlib.import_module(__name__ + "." + name)
    raise AttributeError(name)
