"""Stored DAG predecessors (one tail per pair, or 'none' / 'several') after
loading and after every update, for every source, against the oracle's DAGs;
on graphs with many ties (unit weights) and with few (spread weights)."""
from __future__ import annotations

import pytest

from gpu_util import check_preds, make_ctx, say
from paper_1311_2147_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("case", ["config1", "ties", "spread", "complete"])
def test_stored_predecessors_of_every_source(case):
    if case == "config1":
        g, ups = W.config1()
    elif case == "ties":
        g = W.random_small(120, 0.05, 2, seed=5, directed=True)
        ups = W.mixed_stream(g, 12, 2, 6, 0.35, 0.35, 6)
    elif case == "spread":
        g = W.random_small(150, 0.04, 1000, seed=7, directed=True)
        ups = W.mixed_stream(g, 12, 1000, 8, 0.35, 0.35, 6)
    else:
        g, ups = W.config3(n=96, n_updates=6, k=12)
    ctx = make_ctx(g.n, slots=16)
    gr = ctx.load_graph(g)
    check_preds(gr, g, range(g.n), f"{case} load")
    cur = g
    for i, up in enumerate(ups):
        gr.update(up)
        cur = W.apply_update(cur, up)
        check_preds(gr, cur, range(g.n), f"{case} #{i}")
    say(f"[{case}] {len(ups)} updates, predecessors of all {g.n} sources checked after each")
    ctx.close()
