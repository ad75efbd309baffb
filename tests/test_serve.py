"""The serving loop's scheduling, on the CPU with a stand-in context that
keeps the library's queue rules (a FIFO per graph; a step takes the head of
every non-empty FIFO, oldest first): every request completes once, none is
queued before it arrives, a graph's requests run in arrival order and at
most one per step, no more steps are in flight than allowed, and graphs are
admitted under a byte budget by evicting idle ones."""
from __future__ import annotations

import collections

import numpy as np

from paper_1311_2147_amd import serve


class FakeClock:
    def __init__(self):
        self.t = 0

    def __call__(self):
        self.t += 100_000  # every look at the clock advances it by 0.1 ms
        return self.t


class FakeGraph:
    def __init__(self, idx):
        self.idx = idx
        self.freed = False

    def arcs(self):
        return f"arcs-{self.idx}"

    def free(self):
        self.freed = True


class FakeCtx:
    def __init__(self, clock, polls_to_finish=3):
        self.clock = clock
        self.polls = polls_to_finish
        self.queues = collections.defaultdict(collections.deque)
        self.next = 1
        self.req = {}        # request ticket -> [step id or None, update id, enqueue time]
        self.step_of = {}    # step ticket -> step id
        self.left = {}       # step id -> polls left
        self.steps = []      # (time, update ids, graphs)
        self.in_flight_max = 0
        self.seq = 0
        self.loaded = []

    def load_graph(self, arcs):
        idx = int(arcs.split("-")[1])
        self.loaded.append(idx)
        return FakeGraph(idx)

    def enqueue(self, reqs):
        out = []
        for gr, up in reqs:
            t = self.next
            self.next += 1
            self.queues[gr].append((self.seq, t))
            self.seq += 1
            self.req[t] = [None, id(up), self.clock.t]
            out.append(t)
        return out

    def step(self, max_jobs, want_ticket=False):
        heads = sorted((q[0][0], g) for g, q in self.queues.items() if q)
        if not heads:
            return (0, 0) if want_ticket else 0
        sid = len(self.steps)
        ups, gs = [], []
        for _, g in heads:
            _, t = self.queues[g].popleft()
            self.req[t][0] = sid
            ups.append(self.req[t][1])
            gs.append(g)
        self.steps.append((self.clock.t, ups, gs))
        self.left[sid] = self.polls
        self.in_flight_max = max(self.in_flight_max, sum(1 for v in self.left.values() if v > 0))
        st = self.next
        self.next += 1
        self.step_of[st] = sid
        return (len(ups), st) if want_ticket else len(ups)

    def poll(self, ticket):
        if ticket in self.step_of:
            sid = self.step_of[ticket]
            self.left[sid] -= 1
            return {"status": "BC_OK", "t_finish_ns": self.clock.t} if self.left[sid] <= 0 else None
        sid = self.req[ticket][0]
        if sid is None or self.left[sid] > 0:
            return None
        return {"status": "BC_OK", "t_finish_ns": self.clock.t}


def _check_schedule(ctx, arrivals, requests, done_at, lat):
    assert (done_at > 0).all() and (lat >= 0).all()
    pos = {id(up): i for i, (_, up) in enumerate(requests)}
    ran = []
    for t, ups, gs in ctx.steps:
        assert len(set(id(g) for g in gs)) == len(gs), "a graph got two requests in one step"
        for u in ups:
            assert arrivals[pos[u]] * 1e9 <= t, "request launched before it arrived"
        ran += ups
    assert sorted(pos[u] for u in ran) == list(range(len(requests))), "every request exactly once"
    for gi in set(g for g, _ in requests):
        order = [pos[u] for u in ran if requests[pos[u]][0] == gi]
        assert order == sorted(order), f"graph {gi} requests out of order"
    for t, (_, uid, when) in ctx.req.items():
        assert arrivals[pos[uid]] * 1e9 <= when, "request queued before it arrived"


def test_served_steps_keep_order_and_limits():
    rng = np.random.default_rng(5)
    G, R = 3, 60
    graphs = [f"g{i}" for i in range(G)]
    arrivals = np.sort(rng.uniform(0.0, 0.003, R))
    requests = [(int(rng.integers(0, G)), object()) for _ in range(R)]
    clock = FakeClock()
    ctx = FakeCtx(clock)
    srv = serve.Server(ctx, graphs, max_in_flight=2)
    lat, done_at, wall = srv.run(arrivals, requests, clock=clock, idle_sleep=0)
    assert wall > 0
    _check_schedule(ctx, arrivals, requests, done_at, lat)
    assert ctx.in_flight_max <= 2
    assert srv.stepped_requests == R


def test_admission_under_a_budget_evicts_idle_graphs_only():
    rng = np.random.default_rng(7)
    G, R = 4, 80
    sizes = [10, 10, 30, 30]  # bytes per graph
    arrivals = np.sort(rng.uniform(0.0, 0.01, R))
    requests = [(int(rng.integers(0, G)), object()) for _ in range(R)]
    clock = FakeClock()
    ctx = FakeCtx(clock)
    res = serve.Resident(ctx, [f"arcs-{i}" for i in range(G)], 50, lambda i: sizes[i])
    srv = serve.Server(ctx, resident=res, max_in_flight=2)
    lat, done_at, _ = srv.run(arrivals, requests, clock=clock, idle_sleep=0)
    _check_schedule(ctx, arrivals, requests, done_at, lat)
    assert res.used() <= 50
    assert res.loads == len(ctx.loaded) and res.evictions >= 1  # 30 + 30 never fit together
    # at no point were both large graphs resident: every step holds at most one of them
    for _, _, gs in ctx.steps:
        assert sum(1 for g in gs if g.idx >= 2) <= 1
