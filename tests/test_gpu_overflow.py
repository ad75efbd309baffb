"""Overflow raised by an update, and long candidates that lose.

The device stores distances in 31 bits and path counts in 64 (the reading of
the paper's exact arithmetic taken for storage).  A finite distance that no
longer fits, or a path count past 2^64 - 1, is a sticky error of the graph:
raised by the update that causes it, reported at the next synchronising call,
and cleared only by bc_recompute on a graph whose true state fits again.  A
candidate sum of 2^31 - 1 or more that is not shortest is no error at all.
Every case is forced from the host through ordinary updates; no kernel is made
to fault.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle
from gpu_util import check_full, make_ctx, say
from paper_1311_2147_amd import workloads as W

pytestmark = pytest.mark.gpu

W_MAX = 2**31 - 2  # largest weight the boundary accepts
INF32 = 2**31 - 1


def _bc():
    from paper_1311_2147_amd import bcinc

    return bcinc


def directed_grid(r, c, heavy=()):
    """Unit-weight grid with arcs right and down only; arcs in `heavy` get
    weight 2."""
    src, dst, w = [], [], []
    for i in range(r):
        for j in range(c):
            v = i * c + j
            for (ii, jj) in ((i, j + 1), (i + 1, j)):
                if ii < r and jj < c:
                    u = ii * c + jj
                    src.append(v)
                    dst.append(u)
                    w.append(2 if (v, u) in heavy else 1)
    return W.Graph(r * c, True, np.asarray(src, np.int32), np.asarray(dst, np.int32), np.asarray(w, np.int64))


def arcs_graph(n, arcs, directed=True):
    a = np.asarray([x[0] for x in arcs], np.int32)
    b = np.asarray([x[1] for x in arcs], np.int32)
    w = np.asarray([x[2] for x in arcs], np.int64)
    return W.Graph(n, directed, a, b, w)


def test_sigma_overflow_raised_by_an_update_then_recovered():
    bcinc = _bc()
    r = 35
    corner_in = ((r - 2) * r + (r - 1), (r - 1) * r + (r - 1))  # (33,34) -> (34,34)
    g = directed_grid(r, r, heavy={corner_in})
    ctx = make_ctx(g.n, slots=16)
    say("[ovf-sigma] load 35x35 directed grid, corner arc at weight 2")
    gr = ctx.load_graph(g)
    _, S = gr.rows(0, 1)
    assert int(S[0, g.n - 1]) == math.comb(67, 33)  # fits: only the paths through (34,33)
    lowered = W.Update("edge", u=corner_in[0], v=corner_in[1], w=1)
    cur = W.apply_update(g, lowered)
    with pytest.raises(oracle.SigmaOverflow):
        oracle.brandes(cur, rows=False)  # the oracle agrees: C(68,34) > 2^64 - 1
    say("[ovf-sigma] lower the corner arc to 1: sigma(0, n-1) = C(68,34) > 2^64-1")
    gr.update(lowered)
    with pytest.raises(bcinc.BcError) as e:
        ctx.sync()
    assert e.value.name == "BC_ERR_SIGMA_OVERFLOW"
    with pytest.raises(bcinc.BcError) as e:
        gr.scores()
    assert e.value.name == "BC_ERR_SIGMA_OVERFLOW"
    # a shortcut makes every count fit again; the graph stays halted until
    # it is recomputed
    shortcut = W.Update("edge", u=0, v=g.n - 1, w=1)
    gr.update(shortcut)
    cur = W.apply_update(cur, shortcut)
    with pytest.raises(bcinc.BcError) as e:
        ctx.sync()
    assert e.value.name == "BC_ERR_SIGMA_OVERFLOW"
    say("[ovf-sigma] recompute after the shortcut")
    gr.recompute()
    ctx.sync()
    check_full(gr, cur, "after recovery", dags=(0, r + 1), deltas=(0, 1))
    # and it takes updates again
    more = W.Update("edge", u=1, v=g.n - 1, w=1)
    gr.update(more)
    check_full(gr, W.apply_update(cur, more), "update after recovery")
    ctx.close()


def test_distance_overflow_raised_by_an_update_then_recovered():
    bcinc = _bc()
    g = arcs_graph(4, [(0, 1, W_MAX), (2, 3, 10)])
    ctx = make_ctx(4, slots=4)
    gr = ctx.load_graph(g)
    check_full(gr, g, "load")
    bridge = W.Update("edge", u=1, v=2, w=5)
    cur = W.apply_update(g, bridge)
    ref = oracle.brandes(cur)
    assert ref["D"][0, 2] == W_MAX + 5 >= INF32  # a finite distance past 31 bits
    say("[ovf-dist] bridge 1->2: d(0,2) = 2^31 + 3")
    gr.update(bridge)
    with pytest.raises(bcinc.BcError) as e:
        ctx.sync()
    assert e.value.name == "BC_ERR_DIST_OVERFLOW"
    with pytest.raises(bcinc.BcError) as e:
        gr.recompute()  # the graph as it is still does not fit
    assert e.value.name == "BC_ERR_DIST_OVERFLOW"
    short = W.Update("edge", u=0, v=2, w=1)
    gr.update(short)
    cur = W.apply_update(cur, short)
    Dref = oracle.brandes(cur)["D"]
    assert Dref[Dref != oracle.INF].max() < INF32
    say("[ovf-dist] recompute after 0->2 at weight 1")
    gr.recompute()
    ctx.sync()
    check_full(gr, cur, "after recovery", dags=(0, 1), deltas=(0, 1))
    ctx.close()


def test_distance_overflow_of_a_pair_made_reachable_by_an_out_arc():
    """Vertex update whose out-arc reaches a vertex no path reached before,
    at a length past 31 bits (the Out phase of Section 4)."""
    bcinc = _bc()
    g = arcs_graph(4, [(0, 1, W_MAX - 1), (1, 2, 1)])
    ctx = make_ctx(4, slots=4)
    gr = ctx.load_graph(g)
    check_full(gr, g, "load")
    up = W.Update("vertex", v=2, edges=[(2, 3, 7)])
    cur = W.apply_update(g, up)
    assert oracle.brandes(cur)["D"][0, 3] == W_MAX + 7
    gr.update(up)
    with pytest.raises(bcinc.BcError) as e:
        ctx.sync()
    assert e.value.name == "BC_ERR_DIST_OVERFLOW"
    ctx.close()


def test_long_candidates_that_lose_raise_nothing():
    """Candidates of 2^31 - 1 or more that are not shortest: through the
    scan (edge update), row v'' (vertex update with an out-arc), the static
    pass (load and recompute)."""
    ctx = make_ctx(8, slots=4)
    # edge update: d(0,1) + w'(1,2) = 2^31 + 3 loses to d(0,2) = 1
    g = arcs_graph(4, [(0, 1, W_MAX), (0, 2, 1), (2, 3, 1)])
    gr = ctx.load_graph(g)
    up = W.Update("edge", u=1, v=2, w=5)
    gr.update(up)
    cur = W.apply_update(g, up)
    ctx.sync()
    check_full(gr, cur, "edge update")
    gr.recompute()  # the static pass now relaxes 1->2 from d(0,1) = 2^31 - 2
    check_full(gr, cur, "recompute")
    # vertex update at 1 with out-arc (1,3): w'(1,3) + d(3,4) = 2^31 + 7
    # loses to d(1,4) = 2 through 2
    h = arcs_graph(5, [(0, 1, 1), (1, 2, 1), (2, 4, 1), (3, 4, 10)])
    gh = ctx.load_graph(h)
    up = W.Update("vertex", v=1, edges=[(1, 3, W_MAX - 1)])
    gh.update(up)
    cur = W.apply_update(h, up)
    ctx.sync()
    check_full(gh, cur, "vertex update")
    ctx.close()


@pytest.mark.parametrize("directed", [True, False])
def test_heavy_arcs_around_a_light_hub(directed):
    """A hub with light arcs keeps every distance small, while paths over
    two heavy arcs sum past 31 bits: random insertions and decreases of
    heavy arcs, and of light ones, must match the oracle without an error."""
    n = 24
    rs = W.Rng(W.derive_seed(77, 1 if directed else 2))
    arcs = []
    for x in range(1, n):
        arcs.append((0, x, 1 + int(rs.integers(0, 2, 1)[0])))
        if directed:
            arcs.append((x, 0, 1 + int(rs.integers(0, 2, 1)[0])))
    heavy_w = lambda: int(2**30 + rs.integers(0, 2**30 - 8, 1)[0])  # noqa: E731
    seen = {(a, b) for a, b, _ in arcs}
    while len(arcs) < (4 * n if directed else 3 * n):
        a, b = (int(x) for x in rs.integers(1, n - 1, 2))
        key = (a, b) if directed else (min(a, b), max(a, b))
        if a == b or key in seen:
            continue
        seen.add(key)
        arcs.append((key[0], key[1], heavy_w()))
    g = arcs_graph(n, arcs, directed)
    ctx = make_ctx(n, slots=4)
    gr = ctx.load_graph(g)
    check_full(gr, g, "load")
    cur = g
    st = W.ArcStore(g)
    for i in range(14):
        if i % 3 == 2:
            # vertex update at a random x: two heavy arcs (new or lowered)
            x = int(rs.integers(1, n - 1, 1)[0])
            edges = []
            for y in (int(v) for v in rs.integers(1, n - 1, 6)):
                if y == x or any((y in e[:2]) for e in edges):
                    continue
                a, b = (x, y) if (i % 2 or not directed) else (y, x)
                wc = st.get(a, b)
                wn = heavy_w() if wc is None else max(1, wc - 1 - int(rs.integers(0, 1000, 1)[0]))
                if wc is not None and wn >= wc:
                    continue
                edges.append((a, b, wn))
                if len(edges) == 2:
                    break
            if not edges:
                continue
            up = W.Update("vertex", v=x, edges=edges)
        else:
            a, b = (int(v) for v in rs.integers(1, n - 1, 2))
            if a == b:
                continue
            wc = st.get(a, b)
            wn = heavy_w() if wc is None else max(1, wc - 1 - int(rs.integers(0, 2**20, 1)[0]))
            if wc is not None and wn >= wc:
                continue
            up = W.Update("edge", u=a, v=b, w=wn)
        for (a, b, w) in up.edge_list():
            st.set(a, b, w)
        gr.update(up)
        cur = W.apply_update(cur, up)
        ctx.sync()
        check_full(gr, cur, f"update {i} ({up.kind})")
    gr.recompute()
    check_full(gr, cur, "recompute")
    ctx.close()


def test_sticky_status_of_many_graphs_read_back_together():
    """bc_sync and bc_poll gather the sticky status words of up to 64 graphs
    per launch: an error on the 67th of 70 resident graphs is reported by
    bc_sync and by the result of a ticket that holds it, and a ticket without
    it is clean."""
    bcinc = _bc()
    base = arcs_graph(4, [(0, 1, W_MAX), (2, 3, 10)])
    ctx = make_ctx(4, slots=4)
    grs = [ctx.load_graph(base) for _ in range(70)]
    ctx.sync()
    t1 = ctx.submit([(grs[i], W.Update("edge", u=2, v=3, w=7)) for i in range(70) if i != 66])
    ctx.wait(t1)
    assert ctx.poll(t1)["status"] == "BC_OK"
    ctx.sync()
    say("[ovf-many] graph 66 of 70: bridge 1->2 puts d(0,2) past 31 bits")
    grs[66].update(W.Update("edge", u=1, v=2, w=5))
    with pytest.raises(bcinc.BcError) as e:
        ctx.sync()
    assert e.value.name == "BC_ERR_DIST_OVERFLOW"
    t2 = ctx.submit([(grs[i], W.Update("edge", u=0, v=3, w=9)) for i in (0, 63, 64, 65, 67, 69)])
    ctx.wait(t2)  # its graphs are clean: no error
    t3 = ctx.submit([(grs[i], W.Update("edge", u=0, v=2, w=3)) for i in (1, 66, 68)])
    with pytest.raises(bcinc.BcError) as e:
        ctx.wait(t3)
    assert e.value.name == "BC_ERR_DIST_OVERFLOW"
    # an arc among vertices 2 and 3 only (a path through vertex 1, reached by
    # the 2^31 - 2 arc, would overflow)
    t4 = ctx.submit([(grs[i], W.Update("edge", u=3, v=2, w=4)) for i in (2, 66)])
    t5 = ctx.submit([(grs[i], W.Update("edge", u=3, v=2, w=4)) for i in (3, 62)])
    res = {}
    while len(res) < 2:
        for t in (t4, t5):
            if t not in res:
                r = ctx.poll(t)
                if r is not None:
                    res[t] = r["status"]
    assert res == {t4: "BC_ERR_DIST_OVERFLOW", t5: "BC_OK"}
    # the clean graphs reached the oracle's state
    cur = W.apply_update(W.apply_update(base, W.Update("edge", u=2, v=3, w=7)), W.Update("edge", u=0, v=3, w=9))
    check_full(grs[65], cur, "graph 65")
    check_full(grs[62], W.apply_update(W.apply_update(base, W.Update("edge", u=2, v=3, w=7)),
                                       W.Update("edge", u=3, v=2, w=4)), "graph 62")
    ctx.close()
