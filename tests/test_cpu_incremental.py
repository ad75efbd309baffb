"""The multi-core CPU comparator (Lemma 2 for an arc, Section 4's two-phase
rule for a vertex update, the partial dependency over the changed pairs'
ancestors) against the oracle: distances and path
counts bit-exact and BC within the parity tolerance after every update, on
undirected, directed, tie-heavy and complete graphs with edge and vertex
updates; the thread count changes nothing but the BC summation order; bad
requests leave the state as it was."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_1311_2147_amd import workloads as W
from paper_1311_2147_amd.cpu import CpuError, CpuIncremental

BC_TOL = 1e-10


def bc_err(got, ref):
    return float(np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1.0))) if len(ref) else 0.0


def start(g, threads):
    ref = oracle.brandes(g)
    c = CpuIncremental(g, threads=threads)
    c.set_rows(0, ref["D"], ref["sigma"])
    c.set_scores(ref["bc"])
    return c


def check(c, g, label):
    ref = oracle.brandes(g)
    D, S = c.rows()
    assert np.array_equal(D, ref["D"]), f"{label}: distances differ"
    assert np.array_equal(S, ref["sigma"]), f"{label}: path counts differ"
    e = bc_err(c.scores(), ref["bc"])
    assert e <= BC_TOL, f"{label}: BC error {e}"


def cases():
    yield "config1", *W.config1()
    g = W.random_small(90, 0.06, 2, seed=21, directed=True)
    yield "ties", g, W.mixed_stream(g, 14, 2, 22, 0.35, 0.35, 6)
    g = W.random_small(110, 0.05, 1000, seed=23, directed=True)
    yield "spread", g, W.mixed_stream(g, 14, 1000, 24, 0.35, 0.35, 6)
    g = W.random_small(70, 0.08, 5, seed=25, directed=False)
    yield "undirected", g, W.mixed_stream(g, 10, 5, 26, 0.35, 0.35, 5)
    yield "complete", *W.config3(n=48, n_updates=4, k=8)


@pytest.mark.parametrize("name,g,ups", list(cases()), ids=[c[0] for c in cases()])
def test_matches_oracle_after_every_update(name, g, ups):
    c = start(g, threads=4)
    cur = g
    for i, up in enumerate(ups):
        c.update(up)
        cur = W.apply_update(cur, up)
        check(c, cur, f"{name} #{i} {up.kind}")
    c.close()


def test_thread_count_changes_nothing_but_summation_order():
    g = W.random_small(80, 0.07, 3, seed=31, directed=True)
    ups = W.mixed_stream(g, 10, 3, 32, 0.35, 0.35, 6)
    a, b = start(g, threads=1), start(g, threads=6)
    for up in ups:
        a.update(up)
        b.update(up)
    Da, Sa = a.rows()
    Db, Sb = b.rows()
    assert np.array_equal(Da, Db) and np.array_equal(Sa, Sb)
    assert bc_err(a.scores(), b.scores()) <= BC_TOL


def test_bad_requests_leave_the_state_unchanged():
    g = W.random_small(40, 0.1, 10, seed=41, directed=True)
    c = start(g, threads=2)
    D0, S0 = c.rows()
    bc0 = c.scores()
    a, b, w = int(g.src[0]), int(g.dst[0]), int(g.w[0])
    bad = [W.Update("edge", u=a, v=b, w=w),            # not a decrease
           W.Update("edge", u=a, v=a, w=1),            # self-loop
           W.Update("edge", u=a, v=g.n, w=1),          # no such vertex
           W.Update("edge", u=a, v=b, w=0),            # weight below 1
           W.Update("vertex", v=a, edges=[(b, g.n - 1 if b != g.n - 1 else 0, 1)])]  # not incident to v
    for up in bad:
        with pytest.raises(CpuError):
            c.update(up)
    D1, S1 = c.rows()
    assert np.array_equal(D0, D1) and np.array_equal(S0, S1) and np.array_equal(bc0, c.scores())
    c.close()


@pytest.mark.parametrize("n", [1, 2, 3, 17])
def test_trivial_and_ragged_graphs(n):
    """A lone vertex, a single arc, a path piece and a sparse graph with
    unreachable pairs: insertions that connect pieces, then a vertex update."""
    if n == 1:
        g = W.Graph(1, True, np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int64))
        c = start(g, threads=2)
        check(c, g, "lone vertex")
        c.close()
        return
    src = np.arange(0, n - 1, 2, dtype=np.int32)
    g = W.Graph(n, True, src, src + 1, np.full(len(src), 5, np.int64))
    c = start(g, threads=3)
    cur = g
    ups = [W.Update("edge", u=n - 1, v=0, w=2, insert=True)]
    if n > 2:
        ups.append(W.Update("edge", u=1, v=2, w=1, insert=True))
        ups.append(W.Update("vertex", v=0, edges=[(0, n - 1, 3), (2, 0, 1)]))
    for i, up in enumerate(ups):
        c.update(up)
        cur = W.apply_update(cur, up)
        check(c, cur, f"n={n} #{i}")
    c.close()
