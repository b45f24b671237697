"""Smolyak sparse-grid quadrature on MI355X (gfx950) by a coordinate sweep.

The compute path is libsgmdi.so (HIP kernels behind the C ABI of
include/sgmdi.h); ``native`` is its ctypes binding.  ``workloads`` draws
seeded synthetic integrand batches.  Nothing here falls back to a CPU
implementation.
"""
from __future__ import annotations

from . import workloads  # noqa: F401

__all__ = ["workloads", "native", "integrate", "SGIntegral"]


def __getattr__(name):
    import importlib
    if name in ("native", "api", "build"):
        return importlib.import_module(f"{__name__}.{name}")
    if name in ("integrate", "SGIntegral", "params_tensor"):
        return getattr(importlib.import_module(f"{__name__}.api"), name)
    raise AttributeError(name)
