"""Incremental betweenness centrality on AMD Instinct MI355X (gfx950).

The GPU library (``libbcinc.so``, HIP kernels behind a C ABI) is loaded lazily
on first use of the binding, so that ``workloads`` can be imported on hosts
without a built library.
"""
import importlib

__all__ = ["workloads", "bcinc"]


def __getattr__(name):
    if name in ("bcinc", "workloads", "serve", "build"):
        return importlib.import_module(f".{name}", __name__)
    raise AttributeError(name)
