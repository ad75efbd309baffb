"""The serving loop on the GPU: several graphs' streams served together
(steps batch whichever graphs have a request waiting) end in the same D and
sigma as each stream applied alone on the plain path, and equal the oracle."""
from __future__ import annotations

import numpy as np
import pytest

from gpu_util import BC_TOL, bc_err, check_full, make_ctx, say
from paper_1311_2147_amd import serve
from paper_1311_2147_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_served_mixed_run_equals_streams_alone():
    G, K = 3, 8
    graphs = [W.random_small(100, 0.05, 30, seed=70 + i, directed=i != 1) for i in range(G)]
    streams = [W.mixed_stream(g, K, 30, 80 + i, 0.35, 0.35, 6) for i, g in enumerate(graphs)]
    ctx = make_ctx(max(g.n for g in graphs), slots=16)
    served = [ctx.load_graph(g) for g in graphs]
    alone = [gr.clone() for gr in served]
    requests = [(i, streams[i][k]) for k in range(K) for i in range(G)]
    arrivals = np.sort(W.poisson_arrivals(len(requests), 4000.0, 90))
    lat, _, _ = serve.Server(ctx, served, max_in_flight=2).run(arrivals, requests)
    ctx.sync()
    say(f"served {len(requests)} requests, p50 {serve.percentiles(lat)['p50']:.2f} ms")
    for i in range(G):
        for up in streams[i]:
            alone[i].update(up)
        ctx.sync()
        assert served[i].state_hash() == alone[i].state_hash(), f"graph {i}: served state differs"
        assert bc_err(served[i].scores(), alone[i].scores()) <= BC_TOL
        cur = graphs[i]
        for up in streams[i]:
            cur = W.apply_update(cur, up)
        check_full(served[i], cur, f"served graph {i}")
    ctx.close()


def test_queue_tickets_and_device_times():
    """bc_enqueue queues without running; bc_step runs the head of every
    graph; results carry CLOCK_MONOTONIC times with enqueue <= start <=
    finish <= the host's reading after completion; bc_wait and bc_sync launch
    what is still queued; a direct update runs after everything queued before
    it.  The end state equals the plain path's."""
    import time

    G = 3
    graphs = [W.random_small(120, 0.05, 30, seed=140 + i, directed=True) for i in range(G)]
    streams = [W.mixed_stream(g, 6, 30, 150 + i, 0.35, 0.35, 5) for i, g in enumerate(graphs)]
    ctx = make_ctx(max(g.n for g in graphs), slots=16)
    grs = [ctx.load_graph(g) for g in graphs]
    plain = [gr.clone() for gr in grs]
    ctx.sync()
    h0 = [gr.state_hash() for gr in grs]
    # two requests per graph queued: nothing runs yet
    tickets = ctx.enqueue([(grs[i], streams[i][k]) for k in range(2) for i in range(G)])
    assert [gr.state_hash() for gr in grs] == h0, "queued requests changed state before a step"
    assert all(ctx.poll(t) is None for t in tickets)
    launched, st = ctx.step(want_ticket=True)
    assert launched == G, "a step takes the head of every graph"
    while ctx.poll(st) is None:
        pass
    done_first = []
    for t in tickets[:G]:
        r = None
        while r is None:
            r = ctx.poll(t)
        done_first.append(r)
    after = time.monotonic_ns()
    for r in done_first:
        assert r["status"] == "BC_OK"
        assert r["t_enqueue_ns"] <= r["t_start_ns"] + 200_000  # mapping error well below 0.2 ms
        assert r["t_start_ns"] <= r["t_finish_ns"] <= after + 200_000
    assert all(ctx.poll(t) is None for t in tickets[G:]), "second requests ran without a step"
    ctx.wait(tickets[G])      # launches the remaining heads
    more = ctx.enqueue([(grs[0], streams[0][2])])
    grs[0].update(streams[0][3])  # runs after the queued request before it
    ctx.sync()
    assert ctx.poll(more[0]) is not None
    for k in range(4):
        plain[0].update(streams[0][k])
    for i in range(1, G):
        for k in range(2):
            plain[i].update(streams[i][k])
    ctx.sync()
    for i in range(G):
        assert grs[i].state_hash() == plain[i].state_hash(), f"graph {i} differs from the plain path"
    ctx.close()


def test_admission_under_a_budget_reloads_evicted_graphs_exactly():
    """Four graphs under a budget that holds only some of them: requests for
    a graph that is not resident wait until idle graphs are evicted (their
    arcs kept on the host) and it is loaded again; every graph ends in the
    oracle's state."""
    from paper_1311_2147_amd import bcinc

    graphs = [W.random_small(n, 0.03, 40, seed=170 + i, directed=i % 2 == 0) for i, n in enumerate((300, 420, 360, 480))]
    streams = [W.mixed_stream(g, 10, 40, 180 + i, 0.35, 0.35, 5) for i, g in enumerate(graphs)]
    sizes = []
    for g in graphs:
        arcs = g.m if g.directed else 2 * g.m
        cap = arcs + max(1024, arcs // 8)
        sizes.append(bcinc.bc_graph_bytes(g.n, cap, bcinc.default_estar_capacity(g.n, cap, arcs)) + 256)
    budget = sizes[1] + sizes[3] + sizes[0] // 2  # the two largest fit, not three graphs
    ctx = make_ctx(max(g.n for g in graphs), slots=16)
    res = serve.Resident(ctx, graphs, budget, lambda i: sizes[i])
    requests = [(i, streams[i][k]) for k in range(10) for i in range(len(graphs))]
    arrivals = np.sort(W.poisson_arrivals(len(requests), 3000.0, 190))
    srv = serve.Server(ctx, resident=res, max_in_flight=2)
    lat, _, _ = srv.run(arrivals, requests)
    ctx.sync()
    say(f"[admission] {res.loads} loads, {res.evictions} evictions, p99 {serve.percentiles(lat)['p99']:.1f} ms")
    assert res.evictions >= 1 and res.used() <= budget
    for i, g in enumerate(graphs):
        cur = g
        for up in streams[i]:
            cur = W.apply_update(cur, up)
        gr = res.get(i)
        if gr is None:
            gr = ctx.load_graph(res.arcs[i])  # evicted at the end: its kept arcs must be the final graph
        check_full(gr, cur, f"admitted graph {i}")
    ctx.close()
