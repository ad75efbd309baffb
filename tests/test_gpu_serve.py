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
