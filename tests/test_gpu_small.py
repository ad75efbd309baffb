"""GPU parity on small graphs: full oracle comparison after every update.

Covers the plain path (one update at a time through bc_update_edge /
bc_update_vertex) on the first workload (undirected G(64, 4/63)), the
hand-derived golden sequence, and tie-heavy directed and undirected graphs
with edge and vertex updates (weights in {1..3}, so Lemma 2 / Lemma 4 ties
and NUM-changed pairs are frequent).
"""
from __future__ import annotations

import json
import os

import numpy as np
import pytest

from gpu_util import check_full, make_ctx, say
from paper_1311_2147_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_load_state_matches_oracle_config1():
    g, _ = W.config1()
    say(f"[c1-load] n={g.n} m={g.m}")
    ctx = make_ctx(g.n, slots=16)
    gr = ctx.load_graph(g)
    check_full(gr, g, "c1-load", dags=range(0, 64, 7), deltas=range(0, 64, 9))
    ctx.close()


def test_config1_every_update():
    g, ups = W.config1()
    ctx = make_ctx(g.n, slots=16)
    gr = ctx.load_graph(g)
    cur = g
    for i, up in enumerate(ups):
        say(f"[c1] update {i}: {up.kind} {up.u}->{up.v} w={up.w} insert={up.insert}")
        gr.update(up)
        cur = W.apply_update(cur, up)
        check_full(gr, cur, f"c1 update {i}", dags=(up.u, up.v, (up.u + 31) % 64), deltas=(up.u, up.v))
    st = gr.stats()
    assert st["updates_applied"] == len(ups)
    ctx.close()


def test_golden_sequence_on_gpu():
    with open(os.path.join(GOLDEN, "diamond_updates.json")) as f:
        gold = json.load(f)
    e = np.asarray(gold["edges"], dtype=np.int64)
    g = W.Graph(gold["n"], gold["directed"], e[:, 0].astype(np.int32), e[:, 1].astype(np.int32), e[:, 2])
    ctx = make_ctx(g.n, slots=4)
    gr = ctx.load_graph(g)
    for i, step in enumerate(gold["steps"]):
        say(f"[golden] step {i}")
        u = step["update"]
        if u is not None:
            up = (W.Update("edge", u=u["u"], v=u["v"], w=u["w"]) if u["kind"] == "edge"
                  else W.Update("vertex", v=u["v"], edges=[tuple(x) for x in u["edges"]]))
            gr.update(up)
            g = W.apply_update(g, up)
        from fractions import Fraction
        want = np.array([float(Fraction(x)) if isinstance(x, str) else float(x) for x in step["bc"]])
        got = gr.scores()
        assert np.abs(got - want).max() <= 1e-12, (i, got, want)
        check_full(gr, g, f"golden {i}", dags=range(g.n), deltas=range(g.n))
    ctx.close()


@pytest.mark.parametrize("directed", [True, False])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_ties_mixed_stream(directed, seed):
    n = 48
    g = W.random_small(n, 0.08, 3, seed=seed, directed=directed)
    ups = W.mixed_stream(g, 24, 3, seed, 0.35, 0.35, 5)
    ctx = make_ctx(n, slots=8)
    gr = ctx.load_graph(g)
    cur = g
    for i, up in enumerate(ups):
        say(f"[ties d={directed} seed={seed}] update {i}: {up.kind} v={up.v} k={len(up.edge_list())}")
        gr.update(up)
        cur = W.apply_update(cur, up)
        check_full(gr, cur, f"ties {directed} {seed} #{i}", dags=(up.v, (up.v + 7) % n), deltas=(up.v,))
    ctx.close()
