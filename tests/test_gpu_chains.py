"""Long stored-predecessor chains on the GPU: sources whose union sub-DAG
outgrows the DAG kernel's LDS table.

The graph is a unit-weight path with a few two-hop bypasses (each makes the
vertex after it a vertex with two DAG in-arcs) and side leaves.  The updates
shortcut or double the path far from the source, so a source's changed
targets sit at the end of chains of 40 single-predecessor vertices and the
old sub-DAG holds 160 to 285 vertices (the 128-slot table takes 96 and the
256-slot table 192).  The backward walk then follows the chains lane by lane,
takes E* scan rounds only at the bypass merges, and in the old pass reads the
changed targets' stored predecessors too.  Whole state (D, sigma, E*, BC), the
DAGs of several sources and the stored predecessors of every source are
checked against the oracle after every update, under schedules with either
table and with the wide kernel taking most sources.
"""
from __future__ import annotations

import numpy as np
import pytest

from gpu_util import check_full, check_preds, make_ctx, say
from paper_1311_2147_amd import workloads as W

pytestmark = pytest.mark.gpu

SCHEDULES = [
    {"block": 128, "table": 128, "big_b": 1024, "wide_block": 1024},
    {"block": 64, "table": 256, "big_b": 1024, "wide_block": 512},
    {"block": 256, "table": 128, "big_b": 4, "wide_block": 512},
]


def chain_graph(length: int = 260, bypass_every: int = 40, leaf_every: int = 7) -> W.Graph:
    src, dst = [], []
    n = length
    for i in range(length - 1):
        src.append(i)
        dst.append(i + 1)
    for i in range(bypass_every, length - 1, bypass_every):
        x = n  # i-1 -> x -> i+1 beside i-1 -> i -> i+1
        n += 1
        src += [i - 1, x]
        dst += [x, i + 1]
    for j in range(0, length, leaf_every):
        src.append(j)
        dst.append(n)
        n += 1
    m = len(src)
    return W.Graph(n, True, np.array(src, np.int32), np.array(dst, np.int32), np.ones(m, np.int64))


UPDATES = [
    W.Update("edge", u=0, v=200, w=3, insert=True),  # shortcut: 70 targets behind 200 vertices
    W.Update("edge", u=99, v=101, w=2, insert=True),  # a tie: sigma doubles behind 101
    W.Update("vertex", v=150, edges=[(150, 240, 1), (30, 150, 2)]),
    W.Update("edge", u=10, v=60, w=5, insert=True),
]


@pytest.mark.parametrize("sch", SCHEDULES, ids=["t128", "t256", "wide"])
def test_long_chains_past_the_lds_table(sch):
    g = chain_graph()
    ctx = make_ctx(g.n, slots=16)
    ctx.set_schedule(**sch)
    gr = ctx.load_graph(g)
    cur = g
    for i, up in enumerate(UPDATES):
        say(f"chains {sch}: update {i} {up.kind} {up.u} {up.v} {up.edges}")
        gr.update(up)
        cur = W.apply_update(cur, up)
        check_full(gr, cur, f"chains #{i}", dags=(0, 5, 50, 98, 150))
        check_preds(gr, cur, range(g.n), f"chains #{i}")
    ctx.close()
