"""Checkpoint and restore: a graph's current arcs (bc_get_arcs, saved as plain
arrays) loaded again give the same D and sigma (state hash), the same E* and
BC within tolerance, all equal to the oracle's on the updated graph, and the
restored graph then follows further updates exactly as the original."""
from __future__ import annotations

import numpy as np
import pytest

from gpu_util import BC_TOL, bc_err, check_full, make_ctx, say
from paper_1311_2147_amd import bcinc
from paper_1311_2147_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("directed", [True, False], ids=["directed", "undirected"])
def test_checkpoint_round_trip(tmp_path, directed):
    g = W.random_small(120, 0.05, 50, seed=61 if directed else 62, directed=directed)
    ups = W.mixed_stream(g, 12, 50, 63 if directed else 64, 0.35, 0.35, 6)
    ctx = make_ctx(g.n, slots=16)
    gr = ctx.load_graph(g)
    cur = g
    for up in ups[:6]:
        gr.update(up)
        cur = W.apply_update(cur, up)
    ctx.sync()
    path = str(tmp_path / "graph.npz")
    bcinc.save_checkpoint(gr, path)
    a = gr.arcs()
    assert a.m == cur.m, "checkpoint arc count"
    def key(s, d):
        s, d = s.astype(np.int64), d.astype(np.int64)
        if not directed:
            s, d = np.minimum(s, d), np.maximum(s, d)
        return np.sort(s * g.n + d)

    assert np.array_equal(key(a.src, a.dst), key(cur.src, cur.dst)), "checkpoint arcs differ from the updated graph"
    r = bcinc.load_checkpoint(ctx, path)
    say(f"restored {'directed' if directed else 'undirected'} graph: {a.m} arcs")
    assert r.state_hash() == gr.state_hash()
    assert bc_err(r.scores(), gr.scores()) <= BC_TOL
    ea, eb = gr.estar()[:2], r.estar()[:2]
    ek = lambda a, b: np.sort(a.astype(np.int64) * g.n + b)  # E* holds arcs of G_D
    assert np.array_equal(ek(*ea), ek(*eb)), "E* differs after restore"
    check_full(r, cur, "restored", dags=(0, 5))
    for up in ups[6:]:
        gr.update(up)
        r.update(up)
        cur = W.apply_update(cur, up)
    assert r.state_hash() == gr.state_hash()
    check_full(r, cur, "restored then updated", dags=(0, 5))
    ctx.close()
