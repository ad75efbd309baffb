"""Serving loop: incremental updates for several resident graphs, continuously batched.

Requests (graph, update) arrive over time.  Each graph keeps a FIFO; a step
takes the head-of-line request of every graph that has one and is submitted
as one batched launch sequence (bc_submit: one job per graph, replayed from a
captured HIP graph).  Requests on one graph stay in order because a graph
contributes at most one request per step and steps execute in stream order.
Requests that arrive while steps are in flight join the next step, so work
from many graphs overlaps on the device while no request waits for a fixed
batch to fill.  Completion is observed by polling the step's ticket; latency
is completion minus arrival.
"""
from __future__ import annotations

import collections
import time

import numpy as np


class Server:
    def __init__(self, ctx, graphs, max_in_flight: int = 2):
        self.ctx = ctx
        self.graphs = list(graphs)
        self.max_in_flight = max_in_flight

    def run(self, arrivals, requests, clock=time.perf_counter, poll_sleep: float = 0.0):
        """Open-loop run.  arrivals[i] (seconds from start) is when requests[i]
        = (graph index, update) arrives.  Returns per-request latency (s),
        completion times and the wall time of the run."""
        order = np.argsort(np.asarray(arrivals), kind="stable")
        fifos = [collections.deque() for _ in self.graphs]
        inflight = collections.deque()  # (ticket, [request ids])
        done_at = np.full(len(requests), np.nan)
        t0 = clock()
        nxt = 0
        finished = 0
        while finished < len(requests):
            now = clock() - t0
            while nxt < len(order) and arrivals[order[nxt]] <= now:
                rid = int(order[nxt])
                fifos[requests[rid][0]].append(rid)
                nxt += 1
            while inflight and self.ctx.poll(inflight[0][0]):
                _, rids = inflight.popleft()
                t = clock() - t0
                for rid in rids:
                    done_at[rid] = t
                finished += len(rids)
            if len(inflight) < self.max_in_flight and any(fifos):
                step = [f.popleft() for f in fifos if f]
                ticket = self.ctx.submit([(self.graphs[requests[r][0]], requests[r][1]) for r in step])
                inflight.append((ticket, step))
                continue
            if nxt < len(order) and not inflight and not any(fifos):
                wait = arrivals[order[nxt]] - (clock() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.001))
            elif poll_sleep:
                time.sleep(poll_sleep)
        wall = clock() - t0
        lat = done_at - np.asarray(arrivals)
        return lat, done_at, wall


def percentiles(lat_s):
    lat_ms = np.asarray(lat_s) * 1e3
    return {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99)),
            "mean": float(lat_ms.mean()), "max": float(lat_ms.max())}
