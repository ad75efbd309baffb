"""The static pass's checked search on dense graphs (Static-BC of Section 6
with an arc set containing E* found by search and check instead of every
arc): the state it reaches equals the oracle's and the full search's, it
relaxes a small part of the arcs, and it takes more rounds when E* arcs are
not among the lightest out-arcs of their tails."""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle
from gpu_util import BC_TOL, bc_err, check_full, make_ctx, say
from paper_1311_2147_amd import workloads as W

pytestmark = pytest.mark.gpu


def _both(g, n_max=None, check_oracle=True, label=""):
    n_max = n_max or g.n
    ctx = make_ctx(n_max)
    full = make_ctx(n_max, full_search=True)
    gr = ctx.load_graph(g)
    gf = full.load_graph(g)
    st = gr.stats()
    arcs = g.m if g.directed else 2 * g.m
    say(f"[{label}] n={g.n} arcs={arcs}: searched {st['search_arcs']} arcs in {st['search_rounds']} rounds; "
        f"E* {st['estar_arcs']}")
    assert gr.state_hash() == gf.state_hash(), "checked and full search reach different D/sigma"
    assert bc_err(gr.scores(), gf.scores()) <= BC_TOL
    a, b, w = gr.estar()
    fa, fb, fw = gf.estar()
    assert set(zip(a.tolist(), b.tolist(), w.tolist())) == set(zip(fa.tolist(), fb.tolist(), fw.tolist()))
    if check_oracle:
        check_full(gr, g, label, dags=(0, g.n - 1), deltas=(0, 1))
    full.close()
    return ctx, gr, st


@pytest.mark.parametrize("n", [300, 701])
def test_checked_search_on_complete_graphs(n):
    g = W.complete_undirected(n, n * n, W.derive_seed(61, n))
    ctx, gr, st = _both(g, label=f"complete n={n}")
    assert st["search_rounds"] >= 1
    assert st["search_arcs"] < 2 * g.m // 4
    ctx.close()


def test_checked_search_on_a_dense_directed_graph():
    n = 400
    rs = W.Rng(W.derive_seed(62, 1))
    a, b = np.nonzero(~np.eye(n, dtype=bool))
    keep = rs.uniform(a.shape[0]) < 0.6
    g = W.Graph(n, True, a[keep].astype(np.int32), b[keep].astype(np.int32),
                rs.integers(1, 5000, int(keep.sum())))
    ctx, gr, st = _both(g, label="dense directed")
    assert st["search_rounds"] >= 1
    ctx.close()


def test_checked_search_adds_e_star_arcs_beyond_the_lightest():
    """Complete graph with weights uniform in [3, n^2], except that vertex 0
    has 40 edges of weight 1 (to 1..40) and one of weight 2 to the last
    vertex.  Every other route to that vertex costs at least 1 + 3, so the
    weight-2 edge is in E*, but it ranks 41st among vertex 0's edges, past
    the first searched arcs: a second search must take it in."""
    n = 200
    rs = W.Rng(W.derive_seed(63, 1))
    src, dst, w = [], [], []
    for x in range(n):
        for y in range(x + 1, n):
            src.append(x)
            dst.append(y)
            if x == 0 and 1 <= y <= 40:
                w.append(1)
            elif x == 0 and y == n - 1:
                w.append(2)
            else:
                w.append(int(rs.integers(3, n * n, 1)[0]))
    g = W.Graph(n, False, np.asarray(src, np.int32), np.asarray(dst, np.int32), np.asarray(w, np.int64))
    k = math.ceil(2 * math.log(n)) + 4
    assert 41 > k  # the weight-2 edge ranks past the first searched arcs of vertex 0
    ctx, gr, st = _both(g, label="hidden E* arc")
    assert st["search_rounds"] >= 2
    ctx.close()


def test_recompute_after_updates_uses_the_checked_search():
    g, ups = W.config3(n=400, n_updates=6, k=16)
    ctx = make_ctx(g.n)
    gr = ctx.load_graph(g)
    cur = g
    for up in ups:
        gr.update(up)
        cur = W.apply_update(cur, up)
    h = gr.state_hash()
    gr.recompute()
    st = gr.stats()
    assert st["search_rounds"] >= 1 and gr.state_hash() == h
    check_full(gr, cur, "recompute after vertex updates")
    ctx.close()


def test_config3_full_size_load_matches_full_search():
    g, _ = W.config3()
    ctx, gr, st = _both(g, check_oracle=False, label="c3 n=2048")
    ref = oracle.brandes(g, rows=False)
    assert bc_err(gr.scores(), ref["bc"]) <= BC_TOL
    ctx.close()
