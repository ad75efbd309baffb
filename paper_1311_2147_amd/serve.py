"""Serving loop: incremental updates for several resident graphs, continuously batched.

Requests (graph, update) arrive over time.  Each one is handed to the
library's queue as it arrives (bc_enqueue: validated at once, one ticket per
request); whenever fewer than `max_in_flight` steps are on the device, one
more step is launched (bc_step: the head request of every graph that has one,
as one batched launch sequence replayed from captured HIP graphs).  Requests
on one graph stay in order because the library's queue is a FIFO per graph
and a step takes at most one request per graph.  Requests that arrive while
steps run join the next step, so work from many graphs overlaps on the device
while no request waits for a fixed batch to fill.

Latency is completion minus arrival, both on CLOCK_MONOTONIC: the arrival is
the scheduled arrival time, the completion the device timestamp at which the
step holding the request finished (bc_poll's t_finish_ns).

Admission (Resident): graphs may be admitted to the device under a byte
budget (their arenas, about 16 n^2 bytes each).  A request for a graph with no
state on the device waits until the graph fits; graphs with no request queued
or in flight, and not much larger than it, are evicted for it (the smallest
one that frees enough, else least recently used first until enough is
free), their current
arcs kept on the host (bc_get_arcs) and loaded again by the static pass when
they are needed.  Requests are queued in arrival order, so a waiting request
holds back later ones until its graph is in (no graph starves).
"""
from __future__ import annotations

import collections
import time

import numpy as np


class Resident:
    """Graphs admitted to one context under a byte budget."""

    def __init__(self, ctx, arcs_list, budget_bytes: int, graph_bytes, victim_ratio: float = 2.0):
        self.ctx = ctx
        self.arcs = list(arcs_list)      # current arcs of every graph (host)
        self.budget = int(budget_bytes)
        self.graph_bytes = graph_bytes   # idx -> arena bytes the graph takes
        # a graph is evicted for another only if its arena is at most this
        # many times the other's: a small graph waits for a graph of its size
        # to go idle rather than push out a large one (whose reload costs far
        # more)
        self.victim_ratio = victim_ratio
        self.live = {}                   # idx -> library graph
        self.last_use = {}
        self.loads = 0
        self.evictions = 0
        self.load_s = 0.0

    def used(self) -> int:
        return sum(self.graph_bytes(i) for i in self.live)

    def get(self, idx):
        return self.live.get(idx)

    def admit(self, idx, busy, now):
        """Loads graph idx if it is not resident, evicting idle graphs (not in
        `busy`) as needed.  Returns the library graph, or None when it cannot
        fit until a busy graph goes idle."""
        if idx in self.live:
            self.last_use[idx] = now
            return self.live[idx]
        need = self.graph_bytes(idx)
        if need > self.budget:
            raise ValueError(f"graph {idx} needs {need} bytes, above the whole budget {self.budget}")
        free = self.budget - self.used()
        idle = [i for i in self.live if i not in busy and self.graph_bytes(i) <= self.victim_ratio * need]
        victims = []
        if free < need:
            # the smallest idle graph that frees enough by itself, else idle
            # graphs least recently used first until enough is free
            one = sorted((i for i in idle if free + self.graph_bytes(i) >= need), key=self.graph_bytes)
            if one:
                victims = one[:1]
                free += self.graph_bytes(one[0])
            else:
                for i in sorted(idle, key=lambda i: self.last_use.get(i, 0)):
                    victims.append(i)
                    free += self.graph_bytes(i)
                    if free >= need:
                        break
        if free < need:
            return None
        for i in victims:
            gr = self.live.pop(i)
            self.arcs[i] = gr.arcs()
            gr.free()
            self.evictions += 1
        t = time.perf_counter()
        gr = self.ctx.load_graph(self.arcs[idx])
        self.load_s += time.perf_counter() - t
        self.loads += 1
        self.live[idx] = gr
        self.last_use[idx] = now
        return gr


class Server:
    """Open-loop continuous batching over the library's request queue.

    graphs: library graphs, all resident, indexed by the requests' graph
    numbers; or resident: a Resident that admits graphs on demand."""

    def __init__(self, ctx, graphs=None, max_in_flight: int = 2, max_jobs: int = 0, resident: Resident | None = None):
        if (graphs is None) == (resident is None):
            raise ValueError("give either graphs or resident")
        self.ctx = ctx
        self.graphs = list(graphs) if graphs is not None else None
        self.resident = resident
        self.max_in_flight = max_in_flight
        self.max_jobs = max_jobs
        self.steps = 0
        self.stepped_requests = 0

    def _graph(self, idx, busy, now):
        if self.resident is None:
            return self.graphs[idx]
        return self.resident.admit(idx, busy, now)

    def run(self, arrivals, requests, clock=time.monotonic_ns, idle_sleep: float = 0.0002):
        """arrivals[i] (seconds from the start) is when requests[i] = (graph
        index, update) arrives.  Returns per-request latency (s), completion
        times (s from the start) and the wall time of the run (s)."""
        arrivals = np.asarray(arrivals, dtype=np.float64)
        R = len(requests)
        order = np.argsort(arrivals, kind="stable")
        t0 = clock()
        arr_ns = t0 + np.round(arrivals * 1e9).astype(np.int64)
        done_ns = np.zeros(R, dtype=np.int64)
        done = np.zeros(R, dtype=bool)
        open_tickets = {}                        # request ticket -> request id
        open_per_graph = collections.Counter()   # graph -> open tickets
        pending = collections.deque()            # arrived, not queued yet (arrival order)
        steps = collections.deque()              # step tickets on the device
        nxt = 0
        finished = 0
        while finished < R:
            now = clock()
            while nxt < R and arr_ns[order[nxt]] <= now:
                pending.append(int(order[nxt]))
                nxt += 1
            # requests go to the library's queue in arrival order; one whose
            # graph cannot be admitted yet holds back the ones behind it, so
            # resident graphs drain and the oldest waiting graph gets in
            ready = []
            while pending:
                rid = pending[0]
                gi = requests[rid][0]
                busy = set(g for g, c in open_per_graph.items() if c) | set(requests[r][0] for r, _ in ready)
                gr = self._graph(gi, busy, now)
                if gr is None:
                    break
                ready.append((rid, gr))
                pending.popleft()
            if ready:
                ts = self.ctx.enqueue([(gr, requests[rid][1]) for rid, gr in ready])
                for (rid, _), t in zip(ready, ts):
                    open_tickets[t] = rid
                    open_per_graph[requests[rid][0]] += 1
            # steps that finished free their place; launch the next one
            while steps and self.ctx.poll(steps[0]) is not None:
                steps.popleft()
            if len(steps) < self.max_in_flight:
                launched, st = self.ctx.step(self.max_jobs, want_ticket=True)
                if launched:
                    steps.append(st)
                    self.steps += 1
                    self.stepped_requests += launched
            # requests whose step finished
            for t in list(open_tickets):
                r = self.ctx.poll(t)
                if r is None:
                    continue
                if r["status"] != "BC_OK":
                    raise RuntimeError(f"request {open_tickets[t]} failed on the device: {r['status']}")
                rid = open_tickets.pop(t)
                open_per_graph[requests[rid][0]] -= 1
                done_ns[rid] = r["t_finish_ns"]
                done[rid] = True
                finished += 1
            if not open_tickets and not pending and nxt < R:
                wait = (arr_ns[order[nxt]] - clock()) / 1e9
                if wait > 0:
                    time.sleep(min(wait, 0.001))
            elif idle_sleep:
                time.sleep(idle_sleep)
        while steps:
            if self.ctx.poll(steps[0]) is not None:
                steps.popleft()
        wall = (clock() - t0) / 1e9
        lat = (done_ns - arr_ns) / 1e9
        return lat, (done_ns - t0) / 1e9, wall


def percentiles(lat_s):
    lat_ms = np.asarray(lat_s) * 1e3
    return {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99)),
            "mean": float(lat_ms.mean()), "max": float(lat_ms.max())}
