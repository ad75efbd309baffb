"""The served workload at full shape: 8 resident directed Chung-Lu graphs
(n = 4096, 8192, 16384, 32768, two of each) and a Poisson stream of 10,000
updates over them (35% insertions, 35% decreases, 30% vertex updates of 16
arcs), served by continuous batching.  Parity comes from a deterministic
replay of the same per-graph sequences on fresh loads, one update at a time:
sampled rows against the oracle every 1,000 updates (four sources from the
update's affected set, four uniform, and the updated vertex), BC against the
oracle for the graphs up to n = 8192 at those points, the replay's state
equal to the served state, and BC of every graph against the oracle at the
end."""
from __future__ import annotations

import time

import numpy as np
import pytest

import oracle
from gpu_util import BC_TOL, bc_err, check_sampled, make_ctx, say
from paper_1311_2147_amd import serve
from paper_1311_2147_amd import workloads as W

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def test_config5_served_full_shape_then_replayed_against_the_oracle():
    graphs = [W.config5_graph(W.C5_SIZES[i % 4], i) for i in range(8)]
    stream = W.config5_stream(graphs, 10000)
    ctx = make_ctx(32768)
    t0 = time.perf_counter()
    grs = [ctx.load_graph(g) for g in graphs]
    ctx.sync()
    say(f"[c5] loaded 8 graphs in {time.perf_counter() - t0:.1f}s")
    arrivals = W.poisson_arrivals(len(stream), 600.0, W.derive_seed(5, 5000))
    srv = serve.Server(ctx, grs, max_in_flight=2)
    lat, _, wall = srv.run(arrivals, stream)
    ctx.sync()
    p = serve.percentiles(lat)
    say(f"[c5] served 10000 updates in {wall:.1f}s ({10000 / wall:.0f}/s offered 600/s), {srv.steps} steps, "
        f"p50 {p['p50']:.2f} ms p99 {p['p99']:.2f} ms")
    served_hash = [gr.state_hash() for gr in grs]
    served_bc = [gr.scores() for gr in grs]
    for gr in grs:
        gr.free()
    del grs
    reps = [ctx.load_graph(g) for g in graphs]
    stores = [W.ArcStore(g) for g in graphs]
    rng = np.random.default_rng(55)
    t0 = time.perf_counter()
    for k, (gi, up) in enumerate(stream):
        reps[gi].update(up)
        for a, b, w in up.edge_list():
            stores[gi].set(a, b, w)
        if k % 1000 == 999:
            cur = stores[gi].to_graph()
            A = reps[gi].affected()
            srcs = set(int(x) for x in rng.choice(A, size=min(4, A.size), replace=False)) if A.size else set()
            srcs |= set(int(x) for x in rng.integers(0, cur.n, 4))
            srcs.add(int(up.v))
            check_sampled(reps[gi], cur, sorted(srcs), f"c5 replay #{k} graph {gi}")
            if cur.n <= 8192:
                e = bc_err(reps[gi].scores(), oracle.brandes(cur, rows=False)["bc"])
                assert e <= BC_TOL, f"c5 replay #{k} graph {gi}: BC error {e}"
            say(f"[c5] replay {k + 1}/10000 ({time.perf_counter() - t0:.0f}s): graph {gi} n={cur.n} "
                f"|A|={A.size} sampled rows match")
    ctx.sync()
    for i, g in enumerate(graphs):
        assert reps[i].state_hash() == served_hash[i], f"graph {i}: served and replayed states differ"
        assert bc_err(reps[i].scores(), served_bc[i]) <= BC_TOL
        ref = oracle.brandes(stores[i].to_graph(), rows=False)
        e = bc_err(served_bc[i], ref["bc"])
        say(f"[c5] graph {i} (n={g.n}): served BC against the oracle {e:.2e}")
        assert e <= BC_TOL, f"graph {i}: served BC differs from the oracle by {e}"
    ctx.close()
