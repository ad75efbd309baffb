"""The serving loop's scheduling, on the CPU with a stand-in context: every
request completes once, a graph's requests are submitted in arrival order and
at most one per step, no step is submitted before its requests arrive, and
no more steps are in flight than allowed."""
from __future__ import annotations

import numpy as np

from paper_1311_2147_amd import serve


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1e-4  # every look at the clock advances it
        return self.t


class FakeCtx:
    """submit() records the step; a step completes after a few polls."""

    def __init__(self, clock, polls_to_finish=3):
        self.clock = clock
        self.steps = []
        self.left = {}
        self.in_flight_max = 0
        self.polls = polls_to_finish

    def submit(self, reqs):
        ticket = len(self.steps)
        self.steps.append((self.clock.t, [id(up) for _, up in reqs], [g for g, _ in reqs]))
        self.left[ticket] = self.polls
        self.in_flight_max = max(self.in_flight_max, sum(1 for v in self.left.values() if v > 0))
        return ticket

    def poll(self, ticket):
        self.left[ticket] -= 1
        return self.left[ticket] <= 0


def test_served_steps_keep_order_and_limits():
    rng = np.random.default_rng(5)
    G, R = 3, 60
    graphs = [f"g{i}" for i in range(G)]
    arrivals = np.sort(rng.uniform(0.0, 0.003, R))
    requests = [(int(rng.integers(0, G)), object()) for _ in range(R)]
    clock = FakeClock()
    ctx = FakeCtx(clock)
    lat, done_at, wall = serve.Server(ctx, graphs, max_in_flight=2).run(arrivals, requests, clock=clock)
    assert not np.isnan(done_at).any() and (lat >= 0).all() and wall > 0
    pos = {id(up): i for i, (_, up) in enumerate(requests)}
    submitted = []
    for t, ups, gs in ctx.steps:
        assert len(set(gs)) == len(gs), "a graph got two requests in one step"
        for u in ups:
            assert arrivals[pos[u]] <= t, "request submitted before it arrived"
        submitted += ups
    assert sorted(pos[u] for u in submitted) == list(range(R)), "every request exactly once"
    for gi in range(G):
        order = [pos[u] for u in submitted if requests[pos[u]][0] == gi]
        assert order == sorted(order), f"graph {gi} requests out of order"
    assert ctx.in_flight_max <= 2
