"""CPU oracle for incremental betweenness centrality.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg import this package.  It shares no code with the
GPU library and never imports it; inputs arrive as plain arrays (any object
with ``n``, ``directed``, ``src``, ``dst``, ``w`` attributes works).

The oracle is a from-scratch static computation on the current graph:
Dijkstra from every source with shortest-path counting and predecessor sets
(Alg 7, Eq.1), then Brandes' dependency accumulation (Alg 1, Eq.4), which
gives BC by Eq.3 over ordered pairs.  Since the incremental update of the
paper is exact (Theorem 1 with Lemmas 2-5), these values are what the GPU path
must hold after every update.

Readings of points the paper leaves open (identical on both sides):
  * unreachable t: distance INT64_MAX, sigma 0, contributes nothing to BC;
  * undirected graphs are their directed double G_D, so BC counts ordered
    pairs (twice the unordered convention);
  * path counts are exact uint64; overflow is reported, never wrapped.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .build import LIB_PATH, build as _build

INF = np.iinfo(np.int64).max

_ERRORS = {
    -1: "bad input",
    -2: "self-loop",
    -3: "non-positive weight",
    -4: "duplicate edge",
    -5: "sigma overflow",
    -6: "out of memory",
}


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle error {code}: {_ERRORS.get(code, '?')}")
        self.code = code


class SigmaOverflow(OracleError):
    pass


_lib = None


def _bind(lib):
    p = ctypes.c_void_p
    i32, i64 = ctypes.c_int32, ctypes.c_int64
    lib.oracle_brandes.argtypes = [i32, i64, p, p, p, i32, p, p, p, p, i32]
    lib.oracle_brandes.restype = ctypes.c_int
    lib.oracle_source.argtypes = [i32, i64, p, p, p, i32, i32, p, p, p, p, p, p]
    lib.oracle_source.restype = ctypes.c_int
    lib.oracle_rows.argtypes = [i32, i64, p, p, p, i32, i32, p, p, p, p, i32]
    lib.oracle_rows.restype = ctypes.c_int
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            _build()
        _lib = _bind(ctypes.CDLL(LIB_PATH))
    return _lib


def use_library(path: str):
    """Swap in another build of the oracle's C code (the mutation tests plant
    mistakes in a copy and check that the pins catch them).  Returns the
    previous handle; pass it to restore_library."""
    global _lib
    prev = _load()
    _lib = _bind(ctypes.CDLL(path))
    return prev


def restore_library(handle):
    global _lib
    _lib = handle


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _edges(g):
    src = np.ascontiguousarray(g.src, dtype=np.int32)
    dst = np.ascontiguousarray(g.dst, dtype=np.int32)
    w = np.ascontiguousarray(g.w, dtype=np.int64)
    return int(g.n), int(src.shape[0]), src, dst, w, 1 if g.directed else 0


def _check(rc):
    if rc == -5:
        raise SigmaOverflow(rc)
    if rc != 0:
        raise OracleError(rc)


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:
        return os.cpu_count() or 1


def brandes(g, rows: bool = True, estar: bool = False, threads: int | None = None):
    """All-pairs state and BC of graph g (Alg 7 + Alg 1).

    Returns dict with 'D' (int64 n x n, INF unreachable), 'sigma' (uint64 n x n),
    'bc' (float64 n) and, if asked, 'estar' (uint8 per arc id; undirected
    graphs use 2i for src->dst and 2i+1 for dst->src).
    """
    n, m, src, dst, w, directed = _edges(g)
    D = np.empty((n, n), dtype=np.int64) if rows else None
    S = np.empty((n, n), dtype=np.uint64) if rows else None
    bc = np.empty(n, dtype=np.float64)
    es = np.empty(m * (1 if directed else 2), dtype=np.uint8) if estar else None
    rc = _load().oracle_brandes(n, m, _ptr(src), _ptr(dst), _ptr(w), directed, _ptr(D), _ptr(S), _ptr(bc),
                                _ptr(es), threads or default_threads())
    _check(rc)
    out = {"bc": bc}
    if rows:
        out["D"], out["sigma"] = D, S
    if estar:
        out["estar"] = es
    return out


def source(g, s: int):
    """Single source s: d(s,.), sigma_s., delta_s.(.) and the arcs of DAG(s) (Eq.1)."""
    n, m, src, dst, w, directed = _edges(g)
    cap = max(1, m * (1 if directed else 2))
    d = np.empty(n, dtype=np.int64)
    sg = np.empty(n, dtype=np.uint64)
    de = np.empty(n, dtype=np.float64)
    da = np.empty(cap, dtype=np.int32)
    db = np.empty(cap, dtype=np.int32)
    cnt = np.zeros(1, dtype=np.int64)
    rc = _load().oracle_source(n, m, _ptr(src), _ptr(dst), _ptr(w), directed, int(s), _ptr(d), _ptr(sg), _ptr(de),
                               _ptr(da), _ptr(db), _ptr(cnt))
    _check(rc)
    k = int(cnt[0])
    return {"D": d, "sigma": sg, "delta": de, "dag_a": da[:k].copy(), "dag_b": db[:k].copy()}


def rows(g, sources, threads: int | None = None):
    """Rows d(s,.), sigma_s. and delta_s.(.) for each s in sources (k x n each)."""
    n, m, src, dst, w, directed = _edges(g)
    ss = np.ascontiguousarray(np.asarray(sources, dtype=np.int32))
    k = int(ss.shape[0])
    d = np.empty((k, n), dtype=np.int64)
    sg = np.empty((k, n), dtype=np.uint64)
    de = np.empty((k, n), dtype=np.float64)
    rc = _load().oracle_rows(n, m, _ptr(src), _ptr(dst), _ptr(w), directed, k, _ptr(ss), _ptr(d), _ptr(sg),
                             _ptr(de), threads or default_threads())
    _check(rc)
    return {"D": d, "sigma": sg, "delta": de}


def estar_arcs(g, threads: int | None = None):
    """E* as a set of directed arcs (a, b, w): arcs on some shortest path."""
    res = brandes(g, rows=False, estar=True, threads=threads)
    es = res["estar"]
    out = set()
    for i in range(int(g.src.shape[0])):
        a, b, w = int(g.src[i]), int(g.dst[i]), int(g.w[i])
        if g.directed:
            if es[i]:
                out.add((a, b, w))
        else:
            if es[2 * i]:
                out.add((a, b, w))
            if es[2 * i + 1]:
                out.add((b, a, w))
    return out
