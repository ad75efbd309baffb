"""The state check: BC_FLAG_CHECK after every load and update step, bc_check on
demand.

The check tests the device state against the definitions over the current
arcs: distances that no arc shortens and that some in-arc meets, path counts
as sums over the DAG(s) in-arcs of Eq.1, stored predecessors, symmetry of
undirected graphs, and E* as the tight arcs.  Runs through every entry path
(single updates, split vertex updates, batched submits with several steps per
graph, clones, the request queue) must pass it, and still match the oracle.
A state broken from the host (one path count or one stored predecessor
changed in the arena, which the caller owns) must fail it, name the pair,
halt the graph and recover with bc_recompute.  Only data is changed, never
an index: nothing reads a path count or a predecessor as an address here.
"""
from __future__ import annotations

import time

import numpy as np
import pytest
import torch

from gpu_util import check_full, make_ctx, say
from paper_1311_2147_amd import workloads as W

pytestmark = pytest.mark.gpu


def _bc():
    from paper_1311_2147_amd import bcinc

    return bcinc


def assert_clean(gr, label):
    st = gr.stats()
    assert st["check_failures"] == 0, f"{label}: {st}"
    assert st["check_kind"] == 0 and st["check_source"] == -1, f"{label}: {st}"
    return st


def wide_vertex_update(g, v, k, seed):
    """A vertex update at v with k arcs in and k arcs out (more than one job's
    64 per direction): existing arcs lowered by one where they can be, missing
    ones inserted with weight 1..5."""
    cur = {(int(a), int(b)): int(w) for a, b, w in zip(*g.arcs())}
    rs = np.random.default_rng(seed)
    others = [x for x in range(g.n) if x != v]
    edges = []
    for x in rs.choice(others, size=k, replace=False):
        for a, b in ((int(x), v), (v, int(x))):
            w = cur.get((a, b))
            if w is None:
                edges.append((a, b, int(rs.integers(1, 6))))
            elif w > 1:
                edges.append((a, b, w - 1))
    return W.Update("vertex", v=v, edges=edges)


def test_check_mode_passes_on_every_entry_path():
    ctx = make_ctx(512, slots=16, check=True)
    # undirected: edge updates one at a time (the symmetry check applies)
    g1, ups1 = W.config1()
    say(f"check: {g1.name} n={g1.n}, {len(ups1)} updates")
    gr1 = ctx.load_graph(g1)
    st = assert_clean(gr1, "after load")
    assert st["check_rows"] == g1.n  # the load checks every source
    cur1 = g1
    for up in ups1:
        gr1.update(up)
        cur1 = W.apply_update(cur1, up)
    st = assert_clean(gr1, "config 1 stream")
    assert st["check_rows"] == g1.n + st["total_affected"]  # every affected source, once per update
    check_full(gr1, cur1, "config 1 under the check")

    # directed Chung-Lu: mixed edge and vertex updates, then a vertex update
    # split into two jobs, through single calls, a batched submit with several
    # steps per graph, a clone and the request queue
    g2 = W.chung_lu_directed(300, 2.5, 6.0, 20, 7)
    ups2 = W.mixed_stream(g2, 24, 20, 7, 0.4, 0.3, 6)
    say(f"check: chung-lu n={g2.n} m={g2.m}, {len(ups2)} mixed updates")
    gr2 = ctx.load_graph(g2)
    cur2 = g2
    for up in ups2[:8]:
        gr2.update(up)
        cur2 = W.apply_update(cur2, up)
    big = wide_vertex_update(cur2, 5, 80, 11)
    assert sum(1 for a, b, _ in big.edges if b == 5) > 64 and sum(1 for a, b, _ in big.edges if a == 5) > 64
    gr2.update(big)
    cur2 = W.apply_update(cur2, big)
    assert_clean(gr2, "split vertex update")
    twin = gr2.clone()
    cur_twin = cur2
    reqs = []
    for up in ups2[8:16]:
        reqs.append((gr2, up))
        cur2 = W.apply_update(cur2, up)
    for up in ups2[16:20]:
        reqs.append((twin, up))
        cur_twin = W.apply_update(cur_twin, up)
    ctx.wait(ctx.submit(reqs))
    assert_clean(gr2, "batched submit")
    assert_clean(twin, "batched submit on the clone")
    tickets = ctx.enqueue([(gr2, up) for up in ups2[20:]])
    while ctx.step():
        pass
    for t in tickets:
        ctx.wait(t)
    for up in ups2[20:]:
        cur2 = W.apply_update(cur2, up)
    st = assert_clean(gr2, "queued requests")
    assert st["updates_applied"] == 9 + len(ups2[8:16]) + len(ups2[20:])
    ctx.sync()
    gr2.check()
    twin.check()
    check_full(gr2, cur2, "chung-lu under the check", dags=(0, 5))
    check_full(twin, cur_twin, "clone under the check")
    ctx.close()


def _arena_views(gr):
    """The arena's D, sigma and stored-predecessor regions as host arrays
    (they lead the arena in that order, each on a 256-byte boundary), checked
    against bc_get_rows and bc_get_preds before anything is changed."""
    n = gr.n
    t = gr._arena
    off = ((t.data_ptr() + 255) & ~255) - t.data_ptr()
    host = t.cpu().numpy()
    a256 = lambda x: (x + 255) // 256 * 256  # noqa: E731
    o_d, o_s = off, off + a256(4 * n * n)
    o_p = o_s + a256(8 * n * n)
    D = host[o_d:o_d + 4 * n * n].view(np.int32).reshape(n, n)
    S = host[o_s:o_s + 8 * n * n].view(np.uint64).reshape(n, n)
    P = host[o_p:o_p + 4 * n * n].view(np.int32).reshape(n, n)
    Dr, Sr = gr.rows()
    assert np.array_equal(np.where(D == 2**31 - 1, np.iinfo(np.int64).max, D.astype(np.int64)), Dr)
    assert np.array_equal(S, Sr)
    for s in range(0, n, max(1, n // 8)):
        assert np.array_equal(P[s], gr.preds(s))
    return D, S, P, o_s, o_p


def _poke(gr, byte_off, value: np.ndarray):
    raw = torch.from_numpy(np.ascontiguousarray(value).view(np.uint8).copy())
    gr._arena[byte_off:byte_off + raw.numel()] = raw.to(gr._arena.device)
    torch.cuda.synchronize()


def test_check_names_a_broken_path_count_and_recovers():
    bcinc = _bc()
    g = W.random_small(40, 0.15, 3, 5)  # weights 1..3: many ties, counts above 1
    ctx = make_ctx(64, slots=8)
    gr = ctx.load_graph(g)
    gr.check()
    assert gr.stats()["check_rows"] == g.n
    D, S, P, o_s, _ = _arena_views(gr)
    s, t = max(((i, j) for i in range(g.n) for j in range(g.n) if i != j and D[i, j] != 2**31 - 1),
               key=lambda p: int(S[p]))
    say(f"check: sigma[{s},{t}] = {int(S[s, t])} raised by one in the arena")
    _poke(gr, o_s + 8 * (s * g.n + t), np.array([S[s, t] + 1], np.uint64))
    with pytest.raises(bcinc.BcError) as e:
        gr.check()
    assert e.value.code == -14, e.value
    st = gr.stats()
    assert st["check_kind"] == 4 and st["check_source"] == s and st["check_failures"] >= 1, st
    with pytest.raises(bcinc.BcError) as e:
        gr.scores()  # sticky until recomputed
    assert e.value.code == -14
    gr.recompute()
    gr.check()
    assert_clean(gr, "after bc_recompute")
    check_full(gr, g, "recovered")
    ctx.close()


def test_check_names_a_broken_predecessor():
    bcinc = _bc()
    g = W.random_small(40, 0.15, 3, 6)
    ctx = make_ctx(64, slots=8)
    gr = ctx.load_graph(g)
    D, S, P, _, o_p = _arena_views(gr)
    s, t = next((i, j) for i in range(g.n) for j in range(g.n) if P[i, j] >= 0)
    say(f"check: stored predecessor of ({s},{t}) = {int(P[s, t])} set to the several-tails marker")
    _poke(gr, o_p + 4 * (s * g.n + t), np.array([-2], np.int32))
    with pytest.raises(bcinc.BcError) as e:
        gr.check()
    assert e.value.code == -14
    st = gr.stats()
    assert (st["check_kind"], st["check_source"], st["check_target"], st["check_failures"]) == (5, s, t, 1), st
    gr.recompute()
    gr.check()
    assert np.array_equal(gr.preds(s), P[s])  # P was read before the change
    ctx.close()


def test_check_mode_stops_the_update_that_meets_a_broken_row():
    """Under BC_FLAG_CHECK the step after which a listed source's row is wrong
    fails its call: here a path count of source u, at a pair the arc (u,v)
    inserted next leaves alone, is broken before the update."""
    bcinc = _bc()
    g = W.random_small(40, 0.12, 3, 8)
    ctx = make_ctx(64, slots=8, check=True)
    gr = ctx.load_graph(g)
    D, S, P, o_s, _ = _arena_views(gr)
    INF = 2**31 - 1
    cur = {(int(a), int(b)) for a, b in zip(g.src, g.dst)}
    # an absent arc (u,v) with d(u,v) >= 3, inserted with weight 1, lists u
    # as affected; a target t with d(u,t) < 1 + d(v,t) keeps its pair
    u, v = next((a, b) for a in range(g.n) for b in range(g.n)
                if a != b and (a, b) not in cur and D[a, b] != INF and D[a, b] >= 3)
    t = next(x for x in range(g.n) if x != u and D[u, x] != INF and S[u, x] >= 1
             and (D[v, x] == INF or int(D[u, x]) < 1 + int(D[v, x])))
    say(f"check: sigma[{u},{t}] broken, then arc ({u},{v}) inserted with weight 1")
    _poke(gr, o_s + 8 * (u * g.n + t), np.array([S[u, t] + 1], np.uint64))
    with pytest.raises(bcinc.BcError) as e:
        gr.update_edge(u, v, 1)
    assert e.value.code == -14, e.value
    st = gr.stats()
    assert st["check_kind"] == 4 and st["check_source"] == u, st
    assert u in set(gr.affected().tolist())
    gr.recompute()
    assert_clean(gr, "after bc_recompute")
    g2 = W.Graph(g.n, True, np.append(g.src, np.int32(u)), np.append(g.dst, np.int32(v)),
                 np.append(g.w, np.int64(1)))
    check_full(gr, g2, "recovered with the arc")
    ctx.close()


def test_check_mode_through_full_size_streams():
    """Every step of three workloads checked on the device, which covers every
    affected source's row, stored predecessors and E* at each step (the oracle
    comparisons elsewhere sample them): the out-degree-8 stream at n = 4096
    (256 edge updates), vertex updates of 32 edges on a complete graph, and
    eight graphs of both kinds advanced together, one batched submit per
    step.  BC, which the check leaves out, is compared with the oracle at the
    end of each."""
    ctx = make_ctx(4096, check=True)
    g, ups = W.config2()
    say(f"check: {g.name} m={g.m}, {len(ups)} updates")
    gr = ctx.load_graph(g)
    cur = g
    for i, up in enumerate(ups):
        gr.update(up)
        cur = W.apply_update(cur, up)
        if i % 64 == 63:
            say(f"check: {g.name} update {i} |A|={gr.stats()['affected_sources']}")
    st = assert_clean(gr, g.name)
    assert st["check_rows"] == g.n + st["total_affected"]
    check_full(gr, cur, f"{g.name} under the check")
    gr.free()

    g3, ups3 = W.config3(n=512, n_updates=24, k=32)
    say(f"check: {g3.name}, {len(ups3)} vertex updates")
    gr3 = ctx.load_graph(g3)
    cur3 = g3
    for up in ups3:
        gr3.update(up)
        cur3 = W.apply_update(cur3, up)
    st = assert_clean(gr3, g3.name)
    assert st["check_rows"] == g3.n + st["total_affected"]
    check_full(gr3, cur3, f"{g3.name} under the check", dags=(ups3[-1].v,))

    work = W.config4(count=8, n_updates=8, lo=256, hi=1024)
    say(f"check: eight graphs {[g4.n for g4, _ in work]}, 8 updates each, one submit per step")
    grs = [ctx.load_graph(g4) for g4, _ in work]
    curs = [g4 for g4, _ in work]
    for k in range(8):
        reqs = [(grs[i], work[i][1][k]) for i in range(len(work)) if k < len(work[i][1])]
        ctx.wait(ctx.submit(reqs))
        for i in range(len(work)):
            if k < len(work[i][1]):
                curs[i] = W.apply_update(curs[i], work[i][1][k])
    for i, (g4, _) in enumerate(work):
        st = assert_clean(grs[i], g4.name)
        assert st["check_rows"] == g4.n + st["total_affected"]
        check_full(grs[i], curs[i], f"{g4.name} under the check")
    ctx.close()


@pytest.mark.slow
def test_check_mode_complete_graph_full_size():
    """The complete-graph workload at n = 2048 under the check: vertex
    updates of 32 edges, every step's affected sources checked over all n^2
    arcs, then BC and the whole state against the oracle."""
    g, ups = W.config3()
    ctx = make_ctx(g.n, check=True)
    t0 = time.time()
    gr = ctx.load_graph(g)
    say(f"check: {g.name} loaded and checked in {time.time() - t0:.1f} s")
    cur = g
    for i, up in enumerate(ups):
        t0 = time.time()
        gr.update(up)
        cur = W.apply_update(cur, up)
        say(f"check: {g.name} vertex update {i} |A|={gr.stats()['affected_sources']} in {time.time() - t0:.1f} s")
    st = assert_clean(gr, g.name)
    assert st["check_rows"] == g.n + st["total_affected"]
    check_full(gr, cur, f"{g.name} under the check", dags=(ups[-1].v,))
    ctx.close()


def test_check_degenerate_graphs_and_bad_ids():
    """One vertex, no arcs (every pair but (s,s) unreachable), a graph that
    becomes connected by insertions, and a freed graph's id."""
    bcinc = _bc()
    ctx = make_ctx(64, slots=8, check=True)
    empty = lambda n, directed: W.Graph(n, directed, np.zeros(0, np.int32), np.zeros(0, np.int32),  # noqa: E731
                                        np.zeros(0, np.int64))
    one = ctx.load_graph(empty(1, True))
    one.check()
    assert_clean(one, "one vertex")
    g = empty(9, False)
    gr = ctx.load_graph(g)
    gr.check()
    cur = g
    for i in range(8):
        up = W.Update("edge", u=i, v=i + 1, w=1 + i % 3, insert=True)
        gr.update(up)
        cur = W.apply_update(cur, up)
    st = assert_clean(gr, "path by insertions")
    assert st["check_rows"] == 2 * g.n + st["total_affected"]  # the load, bc_check, then each update
    check_full(gr, cur, "path by insertions")
    gr.free()
    with pytest.raises(bcinc.BcError) as e:
        gr.check()
    assert e.value.code == -1
    ctx.close()


def test_check_mode_autotuner_clones():
    """The autotuner's runs on device clones take the same checked steps (its
    clones carry the arc copy the checks advance); the resident graph is
    left as it was and then updates under the tuned schedule, checked."""
    ctx = make_ctx(1024, slots=16, check=True)
    g = W.random_small(300, 0.02, 20, seed=91, directed=True)
    gr = ctx.load_graph(g)
    h0 = gr.state_hash()
    sample = [(gr, up) for up in W.mixed_stream(g, 6, 20, 92, 0.35, 0.35, 6)]
    say(f"check: autotune over {len(sample)} sample updates on clones of n={g.n}")
    ctx.autotune(sample)
    assert gr.state_hash() == h0, "the autotuner changed the resident graph"
    assert_clean(gr, "after tuning")
    cur = g
    for up in W.mixed_stream(g, 8, 20, 93, 0.35, 0.35, 6):
        gr.update(up)
        cur = W.apply_update(cur, up)
    st = assert_clean(gr, "tuned updates")
    assert st["check_rows"] == g.n + st["total_affected"]
    check_full(gr, cur, "tuned updates under the check")
    ctx.close()


@pytest.mark.slow
def test_check_mode_unit_weights():
    """The tie regime: a unit-weight power-law graph (every arc in E*, most
    vertices with several DAG in-arcs, the per-source passes in their slots)
    under the check after every step, then against the oracle."""
    g = W.chung_lu_directed(4096, 2.5, 16.0, 1, W.derive_seed(5, 0, 77), "cl-unit-4096")
    ups = W.mixed_stream(g, 16, 1, 78, 0.5, 0.0, 16)
    ctx = make_ctx(g.n, check=True)
    gr = ctx.load_graph(g)
    cur = g
    for i, up in enumerate(ups):
        gr.update(up)
        cur = W.apply_update(cur, up)
        if i % 4 == 3:
            say(f"check: unit weights, update {i} |A|={gr.stats()['affected_sources']}")
    st = assert_clean(gr, "unit weights")
    assert st["check_rows"] == g.n + st["total_affected"]
    check_full(gr, cur, "unit weights under the check")
    ctx.close()
