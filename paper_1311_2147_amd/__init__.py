"""Incremental betweenness centrality on AMD Instinct MI355X (gfx950).

The GPU library (``libbcinc.so``, HIP kernels behind a C ABI) is loaded lazily
on first use of the binding, so that ``workloads`` can be imported on hosts
without a built library.
"""

__all__ = ["workloads", "bcinc"]


def __getattr__(name):
    if name == "bcinc":
        from . import bcinc as _b

        return _b
    raise AttributeError(name)
