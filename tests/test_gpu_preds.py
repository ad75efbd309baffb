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


@pytest.mark.parametrize("sch", [{"big_b": 1, "wide_stage": 1, "wide_block": 1024, "block": 128, "table": 128},
                                 {"big_b": 4, "wide_stage": 2, "wide_block": 256, "block": 64, "table": 256}])
@pytest.mark.parametrize("case", ["ties", "spread"])
def test_stored_predecessors_through_the_wide_kernel(case, sch):
    """Arc updates only (Alg 2 gives the changed targets' new predecessors),
    with deferral thresholds that send most affected sources through the wide
    kernel: the first 16 as paired old and new passes on two workgroups, the
    rest as one workgroup each.  Ties (weights 1 and 2) make many changed
    targets keep their distance and gain paths, whose new in-arcs are the old
    ones and row v's."""
    if case == "ties":
        g = W.random_small(140, 0.05, 2, seed=11, directed=True)
        ups = W.mixed_stream(g, 14, 2, 12, 0.5, 0.5, 1)
    else:
        g = W.random_small(160, 0.04, 1000, seed=13, directed=True)
        ups = W.mixed_stream(g, 14, 1000, 14, 0.5, 0.5, 1)
    assert all(up.kind == "edge" for up in ups)
    ctx = make_ctx(g.n, slots=16)
    ctx.set_schedule(**sch)
    gr = ctx.load_graph(g)
    cur = g
    deferred = 0
    for i, up in enumerate(ups):
        gr.update(up)
        deferred += gr.stats()["deferred_sources"]
        cur = W.apply_update(cur, up)
        check_preds(gr, cur, range(g.n), f"{case} {sch} #{i}")
    assert deferred > 16 * 2, "the stream should defer sources past the paired ones"
    say(f"[{case} {sch}] {len(ups)} arc updates, {deferred} deferred sources, all predecessors checked after each")
    ctx.close()
