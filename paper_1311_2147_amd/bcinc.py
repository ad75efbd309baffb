"""Python binding of libbcinc (argument marshalling only).

Every function here forwards to the C ABI of include/bcinc.h with the same
name; all computation runs in the library's HIP kernels.  PyTorch supplies the
device memory (graph arenas, the context scratch) and the stream.  There is no
CPU fallback: if the library is not built, importing this module raises.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbcinc.so")

# PyTorch ships its own HIP runtime under the same soname as the system one.
# Importing torch first makes the loader bind libbcinc.so to that runtime, so
# the process holds one HIP runtime and torch-owned buffers and streams are
# valid inside the library.
import torch  # noqa: E402,F401

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libbcinc.so is not built ({LIB_PATH}); run __graft_entry__.build() or "
                      "python -m paper_1311_2147_amd.build")

_lib = ctypes.CDLL(LIB_PATH)

BC_OK = 0
STATUS_NAMES = {
    0: "BC_OK", -1: "BC_ERR_INVALID_ARG", -2: "BC_ERR_SELF_LOOP", -3: "BC_ERR_BAD_WEIGHT",
    -4: "BC_ERR_DUPLICATE_EDGE", -5: "BC_ERR_NOT_INCIDENT", -6: "BC_ERR_NOT_INCREMENTAL",
    -7: "BC_ERR_ADMISSION", -8: "BC_ERR_CAPACITY", -9: "BC_ERR_SIGMA_OVERFLOW", -10: "BC_ERR_DIST_OVERFLOW",
    -11: "BC_ERR_HIP", -12: "BC_ERR_NO_DEVICE", -13: "BC_ERR_ESTAR_CAPACITY", -14: "BC_ERR_CHECK_FAILED",
}
INF = np.iinfo(np.int64).max


class BcError(RuntimeError):
    def __init__(self, code: int, msg: str = ""):
        super().__init__(f"{STATUS_NAMES.get(code, code)} ({code}): {msg}")
        self.code = code
        self.name = STATUS_NAMES.get(code, str(code))


class bc_config(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("flags", ctypes.c_int32), ("stream", ctypes.c_void_p),
                ("scratch", ctypes.c_void_p), ("scratch_bytes", ctypes.c_uint64),
                ("memory_budget", ctypes.c_uint64), ("slots", ctypes.c_int32), ("block", ctypes.c_int32),
                ("tune_cache", ctypes.c_char_p)]


class bc_edge(ctypes.Structure):
    _fields_ = [("a", ctypes.c_int32), ("b", ctypes.c_int32), ("w", ctypes.c_int64)]


class bc_request(ctypes.Structure):
    _fields_ = [("graph", ctypes.c_int32), ("kind", ctypes.c_int32), ("u", ctypes.c_int32), ("v", ctypes.c_int32),
                ("w", ctypes.c_int64), ("k", ctypes.c_int32), ("edges", ctypes.POINTER(bc_edge))]


class bc_update_stats(ctypes.Structure):
    _fields_ = [("affected_sources", ctypes.c_int64), ("changed_pairs", ctypes.c_int64),
                ("estar_arcs", ctypes.c_int64), ("max_levels", ctypes.c_int64), ("updates_applied", ctypes.c_int64),
                ("total_affected", ctypes.c_int64), ("total_changed", ctypes.c_int64),
                ("deferred_sources", ctypes.c_int64), ("scan_bytes", ctypes.c_int64),
                ("total_scan_bytes", ctypes.c_int64), ("search_arcs", ctypes.c_int64),
                ("search_rounds", ctypes.c_int64), ("check_rows", ctypes.c_int64),
                ("check_failures", ctypes.c_int64), ("check_source", ctypes.c_int64),
                ("check_target", ctypes.c_int64), ("check_kind", ctypes.c_int64)]


class bc_result(ctypes.Structure):
    _fields_ = [("done", ctypes.c_int32), ("status", ctypes.c_int32), ("t_enqueue_ns", ctypes.c_int64),
                ("t_start_ns", ctypes.c_int64), ("t_finish_ns", ctypes.c_int64)]


class bc_timing(ctypes.Structure):
    _fields_ = [("step_ms", ctypes.c_double), ("source_ms", ctypes.c_double), ("steps", ctypes.c_int64),
                ("rows_ms", ctypes.c_double)]


class bc_schedule(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("slots", ctypes.c_int32), ("big_b", ctypes.c_int32),
                ("wide_block", ctypes.c_int32), ("wide_stage", ctypes.c_int32), ("wide_slots", ctypes.c_int32),
                ("table", ctypes.c_int32)]


SCHEDULE_FIELDS = tuple(f for f, _ in bc_schedule._fields_)

BC_FLAG_TIMING = 1
BC_FLAG_FULL_SEARCH = 2
BC_FLAG_CHECK = 4

# kinds of a failed state check (bc_update_stats.check_kind)
CHECK_KINDS = {1: "source", 2: "relax", 3: "no_path", 4: "sigma", 5: "pred", 6: "unreached", 7: "symmetry",
               8: "estar"}


_P = ctypes.c_void_p
_i32, _i64, _u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
_SIGS = {
    "bc_graph_bytes": (_u64, [_i32, _i64, _i64]),
    "bc_scratch_bytes": (_u64, [_i32, _i32]),
    "bc_create": (_i32, [ctypes.POINTER(_P), ctypes.POINTER(bc_config)]),
    "bc_destroy": (_i32, [_P]),
    "bc_load_graph": (_i32, [_P, _i32, _i64, _P, _P, _P, _i32, _i64, _i64, _P, _u64, ctypes.POINTER(_i32)]),
    "bc_free_graph": (_i32, [_P, _i32]),
    "bc_clone_graph": (_i32, [_P, _i32, _P, _u64, ctypes.POINTER(_i32)]),
    "bc_update_edge": (_i32, [_P, _i32, _i32, _i32, _i64]),
    "bc_update_vertex": (_i32, [_P, _i32, _i32, _i32, ctypes.POINTER(bc_edge)]),
    "bc_submit": (_i32, [_P, _i32, ctypes.POINTER(bc_request), ctypes.POINTER(_u64), ctypes.POINTER(_i32)]),
    "bc_enqueue": (_i32, [_P, _i32, ctypes.POINTER(bc_request), ctypes.POINTER(_u64), ctypes.POINTER(_i32)]),
    "bc_step": (_i32, [_P, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_u64)]),
    "bc_poll": (_i32, [_P, _u64, ctypes.POINTER(bc_result)]),
    "bc_wait": (_i32, [_P, _u64]),
    "bc_sync": (_i32, [_P]),
    "bc_scores": (_i32, [_P, _i32, _P]),
    "bc_recompute": (_i32, [_P, _i32]),
    "bc_recompute_estar": (_i32, [_P, _i32]),
    "bc_get_rows": (_i32, [_P, _i32, _i32, _i32, _P, _P]),
    "bc_get_dag": (_i32, [_P, _i32, _i32, _P, _P, _i64, ctypes.POINTER(_i64)]),
    "bc_get_estar": (_i32, [_P, _i32, _P, _P, _P, _i64, ctypes.POINTER(_i64)]),
    "bc_get_arcs": (_i32, [_P, _i32, _P, _P, _P, _i64, ctypes.POINTER(_i64)]),
    "bc_get_delta": (_i32, [_P, _i32, _i32, _P]),
    "bc_get_delta_noalloc": (_i32, [_P, _i32, _i32, _P]),
    "bc_get_preds": (_i32, [_P, _i32, _i32, _P]),
    "bc_get_affected": (_i32, [_P, _i32, _P, _i64, ctypes.POINTER(_i64)]),
    "bc_state_hash": (_i32, [_P, _i32, _P]),
    "bc_check": (_i32, [_P, _i32]),
    "bc_get_stats": (_i32, [_P, _i32, ctypes.POINTER(bc_update_stats)]),
    "bc_get_timing": (_i32, [_P, ctypes.POINTER(bc_timing)]),
    "bc_reset_timing": (_i32, [_P]),
    "bc_set_schedule": (_i32, [_P, ctypes.POINTER(bc_schedule)]),
    "bc_get_schedule": (_i32, [_P, ctypes.POINTER(bc_schedule)]),
    "bc_autotune": (_i32, [_P, _i32, ctypes.POINTER(bc_request), _P, _u64, ctypes.POINTER(bc_schedule)]),
    "bc_status_string": (ctypes.c_char_p, [_i32]),
    "bc_last_error": (ctypes.c_char_p, [_P]),
}
for _name, (_res, _args) in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args

EXPORTED = tuple(_SIGS)


def _np_ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def bc_graph_bytes(n: int, arc_capacity: int, estar_capacity: int = 0) -> int:
    return int(_lib.bc_graph_bytes(n, arc_capacity, estar_capacity))


def bc_scratch_bytes(n_max: int, slots: int = 0) -> int:
    return int(_lib.bc_scratch_bytes(n_max, slots))


def _device_buffer(nbytes: int, device: int):
    """256-byte aligned device buffer owned by torch; returns (tensor, address)."""
    import torch

    t = torch.empty(nbytes + 256, dtype=torch.uint8, device=f"cuda:{device}")
    addr = t.data_ptr()
    return t, (addr + 255) & ~255


def default_estar_capacity(n: int, arc_capacity: int, m_arcs: int) -> int:
    """E* is every arc on some shortest path: close to all arcs of a sparse graph,
    about n ln n of a dense graph with random weights (Section 1 of the paper).
    Dense graphs get a bound with ample slack; the library reports
    BC_ERR_ESTAR_CAPACITY if a graph outgrows it."""
    if m_arcs <= 64 * n:
        return arc_capacity
    return int(min(arc_capacity, 8 * n * max(1.0, math.log(n)) + 4 * n + 4096))


class Context:
    """A bcinc context on one GPU (bc_create / bc_destroy)."""

    def __init__(self, device: int = 0, n_max: int = 4096, slots: int = 0, block: int = 0, memory_budget: int = 0,
                 stream=None, timing: bool = False, full_search: bool = False, tune_cache: str | None = None,
                 check: bool = False):
        import torch

        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self.scratch_bytes = bc_scratch_bytes(n_max, slots)
        self._scratch, addr = _device_buffer(self.scratch_bytes, device)
        flags = ((BC_FLAG_TIMING if timing else 0) | (BC_FLAG_FULL_SEARCH if full_search else 0)
                 | (BC_FLAG_CHECK if check else 0))
        self._tune_cache = tune_cache.encode() if tune_cache else None
        cfg = bc_config(device, flags, self.stream.cuda_stream, addr, self.scratch_bytes, memory_budget, slots, block,
                        self._tune_cache)
        h = ctypes.c_void_p()
        rc = _lib.bc_create(ctypes.byref(h), ctypes.byref(cfg))
        if rc != BC_OK:
            raise BcError(rc, "bc_create")
        self.h = h
        self.graphs: list[Graph] = []

    def _check(self, rc: int, what: str):
        if rc != BC_OK:
            raise BcError(rc, f"{what}: {_lib.bc_last_error(self.h).decode()}")

    def close(self):
        if self.h:
            _lib.bc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load_graph(self, g, arc_capacity: int | None = None, estar_capacity: int | None = None) -> "Graph":
        """bc_load_graph from any object with n, directed, src, dst, w."""
        src = np.ascontiguousarray(g.src, dtype=np.int32)
        dst = np.ascontiguousarray(g.dst, dtype=np.int32)
        w = np.ascontiguousarray(g.w, dtype=np.int64)
        m = int(src.shape[0])
        arcs = m if g.directed else 2 * m
        if arc_capacity is None:
            arc_capacity = arcs + max(1024, arcs // 8)
        if estar_capacity is None:
            estar_capacity = default_estar_capacity(int(g.n), arc_capacity, arcs)
        nbytes = bc_graph_bytes(int(g.n), arc_capacity, estar_capacity)
        arena, addr = _device_buffer(nbytes, self.device)
        gid = ctypes.c_int32()
        rc = _lib.bc_load_graph(self.h, int(g.n), m, _np_ptr(src), _np_ptr(dst), _np_ptr(w), 1 if g.directed else 0,
                                arc_capacity, estar_capacity, addr, nbytes, ctypes.byref(gid))
        self._check(rc, "bc_load_graph")
        gr = Graph(self, gid.value, int(g.n), bool(g.directed), arena, nbytes)
        self.graphs.append(gr)
        return gr

    @staticmethod
    def _requests(requests):
        """bc_request array of [(graph, update)]; the edge arrays it points to
        are returned alongside and must outlive the call.  A Batch is passed
        through as it was marshalled."""
        if isinstance(requests, Batch):
            return requests.reqs, requests.keep
        reqs = (bc_request * len(requests))()
        keep = []
        for i, (gr, up) in enumerate(requests):
            r = reqs[i]
            r.graph = gr.gid
            if up.kind == "edge":
                r.kind, r.u, r.v, r.w = 0, up.u, up.v, up.w
            else:
                arr = (bc_edge * len(up.edges))(*[bc_edge(a, b, w) for a, b, w in up.edges])
                keep.append(arr)
                r.kind, r.v, r.k, r.edges = 1, up.v, len(up.edges), arr
        return reqs, keep

    def autotune(self, requests) -> dict:
        """bc_autotune on a sample [(graph, update)]: sets and returns the
        fastest launch schedule.  The sampled graphs are not modified."""
        reqs, keep = self._requests(requests)
        graphs = {gr.gid: gr for gr, _ in requests}
        nbytes = sum((gr.nbytes + 255) // 256 * 256 for gr in graphs.values())
        ws, addr = _device_buffer(nbytes, self.device)
        out = bc_schedule()
        self._check(_lib.bc_autotune(self.h, len(requests), reqs, addr, nbytes, ctypes.byref(out)), "bc_autotune")
        del ws, keep
        return {f: getattr(out, f) for f in SCHEDULE_FIELDS}

    def batch(self, requests) -> "Batch":
        """[(graph, update)] marshalled once into the request array that
        submit and enqueue take (reusable; the graphs must stay resident)."""
        reqs, keep = self._requests(requests)
        return Batch(reqs, keep, len(requests))

    def submit(self, requests) -> int:
        """bc_submit of [(graph, update)] where update has kind/u/v/w/edges,
        or of a Batch."""
        reqs, keep = self._requests(requests)
        ticket = ctypes.c_uint64()
        bad = ctypes.c_int32(-1)
        rc = _lib.bc_submit(self.h, len(requests), reqs, ctypes.byref(ticket), ctypes.byref(bad))
        if rc != BC_OK:
            raise BcError(rc, f"bc_submit (request {bad.value}): {_lib.bc_last_error(self.h).decode()}")
        return ticket.value

    def enqueue(self, requests) -> list[int]:
        """bc_enqueue of [(graph, update)]: one ticket per request; nothing
        runs until a step launches it."""
        reqs, keep = self._requests(requests)
        tickets = (ctypes.c_uint64 * max(len(requests), 1))()
        bad = ctypes.c_int32(-1)
        rc = _lib.bc_enqueue(self.h, len(requests), reqs, tickets, ctypes.byref(bad))
        if rc != BC_OK:
            raise BcError(rc, f"bc_enqueue (request {bad.value}): {_lib.bc_last_error(self.h).decode()}")
        del keep
        return [int(tickets[i]) for i in range(len(requests))]

    def step(self, max_jobs: int = 0, want_ticket: bool = False):
        """bc_step: launches the head request of every queued graph; returns
        the number launched (and the step's ticket when asked)."""
        launched = ctypes.c_int32()
        st = ctypes.c_uint64()
        self._check(_lib.bc_step(self.h, max_jobs, ctypes.byref(launched), ctypes.byref(st) if want_ticket else None),
                    "bc_step")
        return (launched.value, int(st.value)) if want_ticket else launched.value

    def poll(self, ticket: int):
        """bc_poll: None while the ticket runs, then its result (status and
        CLOCK_MONOTONIC nanoseconds: enqueue on the host, start and finish
        stamped on the device)."""
        r = bc_result()
        self._check(_lib.bc_poll(self.h, ticket, ctypes.byref(r)), "bc_poll")
        if not r.done:
            return None
        return {"status": STATUS_NAMES.get(r.status, r.status), "t_enqueue_ns": r.t_enqueue_ns,
                "t_start_ns": r.t_start_ns, "t_finish_ns": r.t_finish_ns}

    def wait(self, ticket: int):
        self._check(_lib.bc_wait(self.h, ticket), "bc_wait")

    def sync(self):
        self._check(_lib.bc_sync(self.h), "bc_sync")

    def timing(self) -> dict:
        t = bc_timing()
        self._check(_lib.bc_get_timing(self.h, ctypes.byref(t)), "bc_get_timing")
        return {"step_ms": t.step_ms, "source_ms": t.source_ms, "steps": t.steps, "rows_ms": t.rows_ms}

    def reset_timing(self):
        self._check(_lib.bc_reset_timing(self.h), "bc_reset_timing")

    def schedule(self) -> dict:
        s = bc_schedule()
        self._check(_lib.bc_get_schedule(self.h, ctypes.byref(s)), "bc_get_schedule")
        return {f: getattr(s, f) for f in SCHEDULE_FIELDS}

    def set_schedule(self, **fields):
        """Changes the per-source launch schedule (bc_set_schedule); fields not
        given keep their value."""
        bad = set(fields) - set(SCHEDULE_FIELDS)
        if bad:
            raise TypeError(f"unknown schedule fields {sorted(bad)}")
        s = bc_schedule(**{f: int(fields.get(f, 0)) for f in SCHEDULE_FIELDS})
        self._check(_lib.bc_set_schedule(self.h, ctypes.byref(s)), "bc_set_schedule")


class Batch:
    """Requests already marshalled for bc_submit / bc_enqueue (Context.batch)."""

    def __init__(self, reqs, keep, count: int):
        self.reqs, self.keep, self.count = reqs, keep, count

    def __len__(self) -> int:
        return self.count


class Arcs:
    """A graph's arcs as load_graph takes them (n, directed, src, dst, w)."""

    def __init__(self, n: int, directed: bool, src, dst, w):
        self.n, self.directed = int(n), bool(directed)
        self.src, self.dst, self.w = src, dst, w

    @property
    def m(self) -> int:
        return int(len(self.src))


def save_checkpoint(gr: "Graph", path: str):
    """Writes the graph's current arcs (bc_get_arcs) to an .npz file."""
    a = gr.arcs()
    np.savez(path, n=np.int64(a.n), directed=np.int64(a.directed), src=a.src, dst=a.dst, w=a.w)


def load_checkpoint(ctx: "Context", path: str, **kw) -> "Graph":
    """Loads a checkpoint written by save_checkpoint (plain arrays only, no
    pickles): the static pass re-derives the state."""
    with np.load(path, allow_pickle=False) as z:
        a = Arcs(int(z["n"]), bool(z["directed"]), z["src"], z["dst"], z["w"])
    return ctx.load_graph(a, **kw)


class Graph:
    """A graph resident on the device (bc_graph_id)."""

    def __init__(self, ctx: Context, gid: int, n: int, directed: bool, arena, nbytes: int):
        self.ctx, self.gid, self.n, self.directed = ctx, gid, n, directed
        self._arena, self.nbytes = arena, nbytes

    def update_edge(self, u: int, v: int, w: int):
        self.ctx._check(_lib.bc_update_edge(self.ctx.h, self.gid, u, v, w), "bc_update_edge")

    def update_vertex(self, v: int, edges):
        arr = (bc_edge * len(edges))(*[bc_edge(a, b, w) for a, b, w in edges])
        self.ctx._check(_lib.bc_update_vertex(self.ctx.h, self.gid, v, len(edges), arr), "bc_update_vertex")

    def update(self, up):
        if up.kind == "edge":
            self.update_edge(up.u, up.v, up.w)
        else:
            self.update_vertex(up.v, up.edges)

    def prepare(self, up):
        """The update's bc_update_edge / bc_update_vertex call with its
        arguments marshalled once: returns a function of no arguments."""
        h, gid, chk = self.ctx.h, self.gid, self.ctx._check
        if up.kind == "edge":
            u, v, w = up.u, up.v, up.w
            return lambda: chk(_lib.bc_update_edge(h, gid, u, v, w), "bc_update_edge")
        arr = (bc_edge * len(up.edges))(*[bc_edge(a, b, w) for a, b, w in up.edges])
        v, k = up.v, len(up.edges)
        return lambda: chk(_lib.bc_update_vertex(h, gid, v, k, arr), "bc_update_vertex")

    def scores(self) -> np.ndarray:
        out = np.empty(self.n, dtype=np.float64)
        self.ctx._check(_lib.bc_scores(self.ctx.h, self.gid, _np_ptr(out)), "bc_scores")
        return out

    def recompute(self):
        self.ctx._check(_lib.bc_recompute(self.ctx.h, self.gid), "bc_recompute")

    def recompute_estar(self):
        self.ctx._check(_lib.bc_recompute_estar(self.ctx.h, self.gid), "bc_recompute_estar")

    def rows(self, s0: int = 0, cnt: int | None = None):
        cnt = self.n - s0 if cnt is None else cnt
        D = np.empty((cnt, self.n), dtype=np.int64)
        S = np.empty((cnt, self.n), dtype=np.uint64)
        self.ctx._check(_lib.bc_get_rows(self.ctx.h, self.gid, s0, cnt, _np_ptr(D), _np_ptr(S)), "bc_get_rows")
        return D, S

    def dag(self, s: int):
        cnt = ctypes.c_int64()
        self.ctx._check(_lib.bc_get_dag(self.ctx.h, self.gid, s, None, None, 0, ctypes.byref(cnt)), "bc_get_dag")
        k = cnt.value
        a = np.empty(max(k, 1), dtype=np.int32)
        b = np.empty(max(k, 1), dtype=np.int32)
        self.ctx._check(_lib.bc_get_dag(self.ctx.h, self.gid, s, _np_ptr(a), _np_ptr(b), k, ctypes.byref(cnt)),
                        "bc_get_dag")
        return a[:k], b[:k]

    def estar(self):
        cnt = ctypes.c_int64()
        self.ctx._check(_lib.bc_get_estar(self.ctx.h, self.gid, None, None, None, 0, ctypes.byref(cnt)), "bc_get_estar")
        k = cnt.value
        a = np.empty(max(k, 1), dtype=np.int32)
        b = np.empty(max(k, 1), dtype=np.int32)
        w = np.empty(max(k, 1), dtype=np.int64)
        self.ctx._check(_lib.bc_get_estar(self.ctx.h, self.gid, _np_ptr(a), _np_ptr(b), _np_ptr(w), k,
                                          ctypes.byref(cnt)), "bc_get_estar")
        return a[:k], b[:k], w[:k]

    def arcs(self) -> "Arcs":
        """bc_get_arcs: the current arcs, in the form load_graph takes."""
        cnt = ctypes.c_int64()
        self.ctx._check(_lib.bc_get_arcs(self.ctx.h, self.gid, None, None, None, 0, ctypes.byref(cnt)), "bc_get_arcs")
        k = cnt.value
        src = np.empty(max(k, 1), dtype=np.int32)
        dst = np.empty(max(k, 1), dtype=np.int32)
        w = np.empty(max(k, 1), dtype=np.int64)
        self.ctx._check(_lib.bc_get_arcs(self.ctx.h, self.gid, _np_ptr(src), _np_ptr(dst), _np_ptr(w), k,
                                         ctypes.byref(cnt)), "bc_get_arcs")
        return Arcs(self.n, self.directed, src[:k], dst[:k], w[:k])

    def delta(self, s: int) -> np.ndarray:
        out = np.empty(self.n, dtype=np.float64)
        self.ctx._check(_lib.bc_get_delta(self.ctx.h, self.gid, s, _np_ptr(out)), "bc_get_delta")
        return out

    def delta_noalloc(self, s: int, out_dev) -> None:
        """bc_get_delta_noalloc: enqueues the dependency row of s into out_dev
        (a float64 device tensor of n entries); no synchronisation."""
        if out_dev.dtype != torch.float64 or not out_dev.is_cuda or out_dev.numel() < self.n:
            raise ValueError("out_dev must be a float64 device tensor of n entries")
        self.ctx._check(_lib.bc_get_delta_noalloc(self.ctx.h, self.gid, s, ctypes.c_void_p(out_dev.data_ptr())),
                        "bc_get_delta_noalloc")

    def preds(self, s: int) -> np.ndarray:
        """bc_get_preds: stored DAG(s) predecessor per vertex (-1 none, -2 several)."""
        out = np.empty(self.n, dtype=np.int32)
        self.ctx._check(_lib.bc_get_preds(self.ctx.h, self.gid, s, _np_ptr(out)), "bc_get_preds")
        return out

    def affected(self) -> np.ndarray:
        """bc_get_affected: the affected sources of the last update, sorted."""
        cnt = ctypes.c_int64()
        self.ctx._check(_lib.bc_get_affected(self.ctx.h, self.gid, None, 0, ctypes.byref(cnt)), "bc_get_affected")
        k = cnt.value
        out = np.empty(max(k, 1), dtype=np.int32)
        self.ctx._check(_lib.bc_get_affected(self.ctx.h, self.gid, _np_ptr(out), k, ctypes.byref(cnt)),
                        "bc_get_affected")
        return np.sort(out[:k])

    def check(self):
        """bc_check: the whole state against its definitions on the device
        (raises BcError BC_ERR_CHECK_FAILED, naming the first failure)."""
        self.ctx._check(_lib.bc_check(self.ctx.h, self.gid), "bc_check")

    def state_hash(self) -> tuple[int, int]:
        out = np.zeros(2, dtype=np.uint64)
        self.ctx._check(_lib.bc_state_hash(self.ctx.h, self.gid, _np_ptr(out)), "bc_state_hash")
        return int(out[0]), int(out[1])

    def stats(self) -> dict:
        st = bc_update_stats()
        self.ctx._check(_lib.bc_get_stats(self.ctx.h, self.gid, ctypes.byref(st)), "bc_get_stats")
        return {f: getattr(st, f) for f, _ in bc_update_stats._fields_}

    def clone(self) -> "Graph":
        """bc_clone_graph: an independent resident copy of this graph's state."""
        arena, addr = _device_buffer(self.nbytes, self.ctx.device)
        gid = ctypes.c_int32()
        self.ctx._check(_lib.bc_clone_graph(self.ctx.h, self.gid, addr, self.nbytes, ctypes.byref(gid)),
                        "bc_clone_graph")
        gr = Graph(self.ctx, gid.value, self.n, self.directed, arena, self.nbytes)
        self.ctx.graphs.append(gr)
        return gr

    def free(self):
        self.ctx._check(_lib.bc_free_graph(self.ctx.h, self.gid), "bc_free_graph")
        self._arena = None
