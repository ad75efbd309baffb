"""Multi-core CPU comparator for the incremental BC update (C / OpenMP).

The paper's arc update (Lemma 2) and vertex update (Section 4: Alg 4 over the
new in-arcs, row v'' over the new out-arcs, Lemma 4 per pair), with the
partial dependency over the ancestors of the changed pairs, run over the
sources on CPU threads.  It starts from a computed state (the
rows and scores of a graph, for instance read back from the GPU library) and
is a comparator only: the GPU library never calls it.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcpu_incremental.so")
INF = np.iinfo(np.int64).max

_ERR = {-1: "bad argument", -2: "not a decrease", -3: "path-count overflow", -4: "distance overflow",
        -5: "out of memory"}
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        lib = ctypes.CDLL(LIB_PATH)
        P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        lib.icpu_create.argtypes = [I32, I64, P, P, P, ctypes.c_int, ctypes.c_int, ctypes.POINTER(P)]
        lib.icpu_set_rows.argtypes = [P, I32, I32, P, P]
        lib.icpu_get_rows.argtypes = [P, I32, I32, P, P]
        lib.icpu_set_scores.argtypes = [P, P]
        lib.icpu_get_scores.argtypes = [P, P]
        lib.icpu_update_edge.argtypes = [P, I32, I32, I64]
        lib.icpu_update_vertex.argtypes = [P, I32, I32, P, P, P]
        lib.icpu_destroy.argtypes = [P]
        lib.icpu_destroy.restype = None
        _lib = lib
    return _lib


class CpuError(RuntimeError):
    def __init__(self, rc, what):
        super().__init__(f"{what}: {_ERR.get(rc, rc)}")
        self.rc = rc


def _check(rc, what):
    if rc != 0:
        raise CpuError(rc, what)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class CpuIncremental:
    """One graph's incremental state on the host, updated on `threads` threads."""

    def __init__(self, g, threads: int = 0):
        lib = _load()
        self.n = g.n
        self.directed = bool(g.directed)
        src = np.ascontiguousarray(g.src, dtype=np.int32)
        dst = np.ascontiguousarray(g.dst, dtype=np.int32)
        w = np.ascontiguousarray(g.w, dtype=np.int64)
        h = ctypes.c_void_p()
        _check(lib.icpu_create(g.n, g.m, _p(src), _p(dst), _p(w), int(self.directed), int(threads), ctypes.byref(h)),
               "icpu_create")
        self.h = h

    def set_rows(self, s0: int, D: np.ndarray, S: np.ndarray):
        D = np.ascontiguousarray(D, dtype=np.int64)
        S = np.ascontiguousarray(S, dtype=np.uint64)
        cnt = D.shape[0]
        assert D.shape == (cnt, self.n) and S.shape == (cnt, self.n)
        _check(_load().icpu_set_rows(self.h, s0, cnt, _p(D), _p(S)), "icpu_set_rows")

    def set_scores(self, bc: np.ndarray):
        bc = np.ascontiguousarray(bc, dtype=np.float64)
        assert bc.shape == (self.n,)
        _check(_load().icpu_set_scores(self.h, _p(bc)), "icpu_set_scores")

    def rows(self, s0: int = 0, cnt: int | None = None):
        cnt = self.n - s0 if cnt is None else cnt
        D = np.empty((cnt, self.n), dtype=np.int64)
        S = np.empty((cnt, self.n), dtype=np.uint64)
        _check(_load().icpu_get_rows(self.h, s0, cnt, _p(D), _p(S)), "icpu_get_rows")
        return D, S

    def scores(self) -> np.ndarray:
        bc = np.empty(self.n, dtype=np.float64)
        _check(_load().icpu_get_scores(self.h, _p(bc)), "icpu_get_scores")
        return bc

    def update(self, up):
        """One update request (the workloads' Update: an edge or a vertex update)."""
        lib = _load()
        if up.kind == "edge":
            _check(lib.icpu_update_edge(self.h, up.u, up.v, up.w), "icpu_update_edge")
        else:
            e = up.edge_list()
            a = np.array([x[0] for x in e], dtype=np.int32)
            b = np.array([x[1] for x in e], dtype=np.int32)
            w = np.array([x[2] for x in e], dtype=np.int64)
            _check(lib.icpu_update_vertex(self.h, up.v, len(e), _p(a), _p(b), _p(w)), "icpu_update_vertex")

    def close(self):
        if self.h:
            _load().icpu_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
