"""GPU edge cases and error behaviour of the boundary."""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle
from gpu_util import check_full, make_ctx, say
from paper_1311_2147_amd import workloads as W

pytestmark = pytest.mark.gpu


def _bc():
    from paper_1311_2147_amd import bcinc

    return bcinc


@pytest.mark.parametrize("n", [1, 2, 63, 65, 257])
def test_ragged_sizes_and_trivial_graphs(n):
    g = W.random_small(n, 0.08 if n > 2 else 1.0, 5, seed=n, directed=True)
    ctx = make_ctx(n, slots=8)
    gr = ctx.load_graph(g)
    check_full(gr, g, f"n={n} load")
    if n >= 2:
        if n < 8:
            ups = [W.Update("edge", u=0, v=1, w=1), W.Update("edge", u=1, v=0, w=2)]
        else:
            ups = W.mixed_stream(g, 6, 5, n, 0.5, 0.3, 3)
        cur = g
        for up in ups:
            gr.update(up)
            cur = W.apply_update(cur, up)
        check_full(gr, cur, f"n={n} after")
    ctx.close()


def test_empty_graph_then_insertions_connect_components():
    g = W.Graph(10, False, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int64))
    ctx = make_ctx(10, slots=4)
    gr = ctx.load_graph(g)
    assert np.all(gr.scores() == 0)
    cur = g
    for (a, b, w) in [(0, 1, 3), (1, 2, 3), (5, 6, 1), (2, 5, 2), (0, 2, 6), (0, 2, 5)]:
        up = W.Update("edge", u=a, v=b, w=w)
        gr.update(up)
        cur = W.apply_update(cur, up)
        check_full(gr, cur, f"insert {a}-{b}")
    ctx.close()


def test_closing_a_path_into_a_cycle_on_gpu():
    for n in (8, 9):
        k = n // 2
        ctx = make_ctx(n, slots=4)
        gr = ctx.load_graph(W.path_graph(n))
        gr.update_edge(0, n - 1, 1)
        want = (k - 1) ** 2 if n % 2 == 0 else k * (k - 1)
        assert np.abs(gr.scores() - want).max() <= 1e-9
        ctx.close()


def test_invalid_requests_leave_state_unchanged():
    bcinc = _bc()
    g = W.random_small(40, 0.1, 9, seed=8, directed=True)
    ctx = make_ctx(40, slots=8)
    gr = ctx.load_graph(g)
    h0, bc0 = gr.state_hash(), gr.scores()
    a, b, w = int(g.src[0]), int(g.dst[0]), int(g.w[0])
    cases = [
        (lambda: gr.update_edge(a, b, w), "BC_ERR_NOT_INCREMENTAL"),
        (lambda: gr.update_edge(a, b, w + 5), "BC_ERR_NOT_INCREMENTAL"),
        (lambda: gr.update_edge(3, 3, 1), "BC_ERR_SELF_LOOP"),
        (lambda: gr.update_edge(0, 40, 1), "BC_ERR_INVALID_ARG"),
        (lambda: gr.update_edge(0, 1, 0), "BC_ERR_BAD_WEIGHT"),
        (lambda: gr.update_edge(0, 1, 2 ** 31 - 1), "BC_ERR_BAD_WEIGHT"),
        (lambda: gr.update_vertex(5, [(5, 6, 1), (5, 6, 1)]), "BC_ERR_DUPLICATE_EDGE"),
        (lambda: gr.update_vertex(5, [(5, 6, 1), (7, 8, 1)]), "BC_ERR_NOT_INCIDENT"),
    ]
    for fn, name in cases:
        with pytest.raises(bcinc.BcError) as e:
            fn()
        assert e.value.name == name
        assert gr.state_hash() == h0
        assert np.array_equal(gr.scores(), bc0)
    # a batched submit with one bad request applies nothing
    ups = [W.Update("edge", u=1, v=2, w=1), W.Update("edge", u=a, v=b, w=w)]
    with pytest.raises(bcinc.BcError):
        ctx.submit([(gr, up) for up in ups])
    assert gr.state_hash() == h0
    ctx.close()


def test_non_shortest_decrease_changes_only_the_weight():
    g = W.random_small(50, 0.12, 50, seed=31, directed=True)
    ref = oracle.brandes(g)
    for i in range(g.m):
        a, b, w = int(g.src[i]), int(g.dst[i]), int(g.w[i])
        if w > ref["D"][a, b] + 1:
            break
    else:
        pytest.skip("no non-shortest arc")
    ctx = make_ctx(50, slots=8)
    gr = ctx.load_graph(g)
    h0 = gr.state_hash()
    gr.update_edge(a, b, int(ref["D"][a, b]) + 1)
    assert gr.state_hash() == h0
    assert gr.stats()["affected_sources"] == 0
    cur = W.apply_update(g, W.Update("edge", u=a, v=b, w=int(ref["D"][a, b]) + 1))
    check_full(gr, cur, "non-shortest")
    ctx.close()


def test_vertex_update_equals_its_edits_one_at_a_time_and_edge_form():
    g = W.random_small(60, 0.1, 6, seed=44, directed=True)
    v = 7
    st = W.ArcStore(g)
    edges = []
    for x in range(60):
        if x == v:
            continue
        for (a, b) in ((x, v), (v, x)):
            cw = st.get(a, b)
            if cw is None and len(edges) < 10 and (x % 5 == 0):
                edges.append((a, b, 3))
            elif cw is not None and cw >= 2:
                edges.append((a, b, cw - 1))
    ctx = make_ctx(60, slots=8)
    g1 = ctx.load_graph(g)
    g2 = ctx.load_graph(g)
    g1.update_vertex(v, edges)
    for e in edges:
        g2.update_edge(*e)
    assert g1.state_hash() == g2.state_hash()
    assert np.abs(g1.scores() - g2.scores()).max() <= 1e-9 * max(1.0, np.abs(g2.scores()).max())
    cur = W.apply_update(g, W.Update("vertex", v=v, edges=edges))
    check_full(g1, cur, "vertex vs edges")
    ctx.close()


def test_vertex_update_wider_than_one_job():
    """More than 64 arcs per direction: applied as consecutive vertex updates."""
    n = 200
    g = W.random_small(n, 0.02, 9, seed=5, directed=True)
    st = W.ArcStore(g)
    v = 3
    edges = []
    for x in range(n):
        if x != v:
            cw = st.get(x, v)
            edges.append((x, v, (cw - 1) if (cw or 0) >= 2 else 7) if cw != 1 else None)
    edges = [e for e in edges if e is not None][:150]
    ctx = make_ctx(n, slots=16)
    gr = ctx.load_graph(g)
    gr.update_vertex(v, edges)
    check_full(gr, W.apply_update(g, W.Update("vertex", v=v, edges=edges)), "wide vertex update")
    ctx.close()


def test_recompute_equals_incremental_state():
    g, ups = W.config2(n=700, n_updates=30)
    ctx = make_ctx(700, slots=32)
    gr = ctx.load_graph(g)
    for up in ups:
        gr.update(up)
    h, bc = gr.state_hash(), gr.scores()
    gr.recompute()
    assert gr.state_hash() == h
    assert np.abs(gr.scores() - bc).max() <= 1e-10 * max(1.0, np.abs(bc).max())
    ctx.close()


@pytest.mark.parametrize("kind", ["directed", "complete"])
def test_estar_recompute_equals_incremental_and_full_recompute(kind):
    """The static pass restricted to the maintained E* reaches the state of the
    incremental updates and of the full recompute, and the oracle's."""
    if kind == "directed":
        g = W.random_small(300, 0.03, 20, seed=23, directed=True)
        ups = W.mixed_stream(g, 16, 20, 31, 0.35, 0.35, 8)
    else:
        g, ups = W.config3(n=256, n_updates=6, k=16)
    ctx = make_ctx(g.n, slots=32)
    gr = ctx.load_graph(g)
    cur = g
    for up in ups:
        gr.update(up)
        cur = W.apply_update(cur, up)
    h, bc = gr.state_hash(), gr.scores()
    a, b, w = gr.estar()
    before = set(zip(a.tolist(), b.tolist(), w.tolist()))
    say(f"[{kind}] recompute over E* ({len(before)} arcs of {cur.m if cur.directed else 2 * cur.m})")
    gr.recompute_estar()
    assert gr.state_hash() == h
    assert np.abs(gr.scores() - bc).max() <= 1e-10 * max(1.0, np.abs(bc).max())
    a, b, w = gr.estar()
    assert set(zip(a.tolist(), b.tolist(), w.tolist())) == before
    check_full(gr, cur, f"{kind} after E* recompute", dags=(0, 1, g.n // 2))
    gr.recompute()
    assert gr.state_hash() == h
    # and once more over E* right after a full recompute
    gr.recompute_estar()
    check_full(gr, cur, f"{kind} after a second E* recompute", estar=False)
    ctx.close()


def test_estar_recompute_refuses_a_graph_with_a_sticky_error():
    bcinc = _bc()
    g = W.random_small(64, 0.1, 9, seed=2, directed=True)
    ctx = make_ctx(64, slots=4)
    probe = ctx.load_graph(g)
    mstar = probe.stats()["estar_arcs"]
    probe.free()
    gr = ctx.load_graph(g, estar_capacity=mstar)
    st = W.ArcStore(g)
    a, b = next((a, b) for a in range(64) for b in range(64) if a != b and st.get(a, b) is None)
    # an inserted arc of weight 1 is its own shortest path, so E* outgrows
    # the capacity it was loaded with
    with pytest.raises(bcinc.BcError) as e:
        gr.update_edge(a, b, 1)
        ctx.sync()
        gr.scores()
    assert e.value.name == "BC_ERR_ESTAR_CAPACITY"
    with pytest.raises(bcinc.BcError) as e:
        gr.recompute_estar()
    assert e.value.name == "BC_ERR_ESTAR_CAPACITY"
    ctx.close()


def test_sigma_overflow_is_detected_and_recoverable():
    bcinc = _bc()
    ctx = make_ctx(35 * 35, slots=8)
    g34 = W.grid_graph(34, 34)
    gr = ctx.load_graph(g34)
    D, S = gr.rows(0, 1)
    assert int(S[0, 34 * 34 - 1]) == math.comb(66, 33)
    with pytest.raises(bcinc.BcError) as e:
        ctx.load_graph(W.grid_graph(35, 35))
    assert e.value.name == "BC_ERR_SIGMA_OVERFLOW"
    ctx.close()


def test_capacity_and_admission_errors():
    bcinc = _bc()
    g = W.random_small(64, 0.1, 9, seed=2, directed=True)
    ctx = make_ctx(64, slots=4)
    with pytest.raises(bcinc.BcError) as e:
        ctx.load_graph(g, arc_capacity=g.m - 1)
    assert e.value.name == "BC_ERR_CAPACITY"
    with pytest.raises(bcinc.BcError) as e:
        ctx.load_graph(g, estar_capacity=8)
    assert e.value.name == "BC_ERR_ESTAR_CAPACITY"
    gr = ctx.load_graph(g, arc_capacity=g.m + 1)
    st = W.ArcStore(g)
    ins = [(a, b) for a in range(64) for b in range(64) if a != b and st.get(a, b) is None][:2]
    gr.update_edge(ins[0][0], ins[0][1], 5)
    with pytest.raises(bcinc.BcError) as e:
        gr.update_edge(ins[1][0], ins[1][1], 5)
    assert e.value.name == "BC_ERR_CAPACITY"
    ctx.close()
    tiny = make_ctx(64, slots=4, memory_budget=bcinc.bc_graph_bytes(64, 2 * g.m, 0) + 10)
    tiny.load_graph(g, arc_capacity=2 * g.m)
    with pytest.raises(bcinc.BcError) as e:
        tiny.load_graph(g, arc_capacity=2 * g.m)
    assert e.value.name == "BC_ERR_ADMISSION"
    tiny.close()


def test_lemma1_row_v_column_u_and_undirected_symmetry():
    """Lemma 1: an arc update (u, v) leaves row v and column u as they were;
    an undirected graph's D and sigma stay symmetric through every update."""
    g = W.random_small(90, 0.06, 10, seed=91, directed=True)
    h = W.random_small(80, 0.06, 10, seed=93, directed=False)
    ctx = make_ctx(max(g.n, h.n), slots=8)
    gr = ctx.load_graph(g)
    ups = W.mixed_stream(g, 12, 10, 92, 0.5, 0.5, 4)
    assert all(up.kind == "edge" for up in ups)
    for up in ups:
        D0, S0 = gr.rows()
        gr.update(up)
        D1, S1 = gr.rows()
        assert np.array_equal(D1[up.v], D0[up.v]) and np.array_equal(S1[up.v], S0[up.v]), "row v changed"
        assert np.array_equal(D1[:, up.u], D0[:, up.u]) and np.array_equal(S1[:, up.u], S0[:, up.u]), \
            "column u changed"
    gh = ctx.load_graph(h)
    for up in W.mixed_stream(h, 10, 10, 94, 0.35, 0.35, 4):
        gh.update(up)
        D, S = gh.rows()
        assert np.array_equal(D, D.T) and np.array_equal(S, S.T), "undirected state lost its symmetry"
    ctx.close()


def test_hub_fan_graph_static_pass_and_updates():
    """A unit-weight fan: vertex 0 has 1500 out-arcs to a middle layer, every
    middle vertex has arcs to the same 40 bottom vertices, and each bottom
    vertex one arc on.  The static search's frontier holds 1500 vertices in
    one round (more than one chunk of a workgroup), vertex 0 and every middle
    vertex have more out-arcs than a lane takes alone (a wave each in the sigma
    and delta passes), and the bottom vertices gather 1500 tied paths each.
    Load and a few updates against the oracle, with the DAGs of sources 0, a
    middle vertex and a bottom vertex."""
    mid, bot = 1500, 40
    n = 1 + mid + 2 * bot
    src, dst = [], []
    for m in range(1, mid + 1):
        src.append(0)
        dst.append(m)
        for b in range(bot):
            src.append(m)
            dst.append(1 + mid + b)
    for b in range(bot):
        src.append(1 + mid + b)
        dst.append(1 + mid + bot + b)
    g = W.Graph(n, True, np.asarray(src, np.int32), np.asarray(dst, np.int32), np.ones(len(src), np.int64))
    ctx = make_ctx(n, slots=16)
    gr = ctx.load_graph(g)
    check_full(gr, g, "fan load", dags=(0, 7, 1 + mid + 3), estar=True)
    say(f"[fan] n={n}, {len(src)} arcs: load matches the oracle")
    ups = [W.Update("edge", u=0, v=1 + mid + 5, w=1),        # a shortcut past the fan to one bottom vertex
           W.Update("edge", u=2, v=1 + mid + bot + 7, w=1),  # a middle vertex straight to a last-layer vertex
           W.Update("vertex", v=1 + mid, edges=[(0, 1 + mid, 2), (1 + mid, 1 + mid + bot + 1, 1)])]
    cur = g
    for k, up in enumerate(ups):
        gr.update(up)
        cur = W.apply_update(cur, up)
        check_full(gr, cur, f"fan update {k}", dags=(0, 7), estar=True)
    say("[fan] three updates match the oracle")
    ctx.close()
