"""Helpers of the GPU parity tests: run the HIP path and compare it with the oracle."""
from __future__ import annotations

import os
import sys

import numpy as np

import oracle
from paper_1311_2147_amd import workloads as W

BC_TOL = 1e-10  # |BC_gpu - BC_ref| <= BC_TOL * max(|BC_ref|, 1)


def say(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def bc_err(got, ref):
    return float((np.abs(got - ref) / np.maximum(np.abs(ref), 1.0)).max(initial=0.0))


def dag_set(a, b):
    return set(zip(np.asarray(a).tolist(), np.asarray(b).tolist()))


def expected_preds(n, dag_a, dag_b):
    """Stored-predecessor row from the oracle's DAG(s) arcs: the only tail
    into x, -2 for two or more, -1 for none."""
    a = np.asarray(dag_a, dtype=np.int64)
    b = np.asarray(dag_b, dtype=np.int64)
    cnt = np.bincount(b, minlength=n)
    out = np.full(n, -1, dtype=np.int32)
    one = cnt[b] == 1
    out[b[one]] = a[one]
    out[cnt >= 2] = -2
    return out


def check_preds(gr, g, sources, label=""):
    """Stored predecessors of the listed sources against the oracle's DAGs."""
    for s in sources:
        one = oracle.source(g, int(s))
        want = expected_preds(g.n, one["dag_a"], one["dag_b"])
        got = gr.preds(int(s))
        bad = np.flatnonzero(got != want)
        assert bad.size == 0, (f"{label}: stored predecessors of source {s} differ at {bad.size} vertices, first "
                               f"{[(int(x), int(got[x]), int(want[x])) for x in bad[:3]]}")


def check_full(gr, g, label="", dags=(), deltas=(), estar=True):
    """Whole-state parity: D and sigma bit-exact, BC within BC_TOL, E* and
    the DAGs of the listed sources as sets (and their stored predecessors),
    delta rows within BC_TOL."""
    ref = oracle.brandes(g, estar=estar)
    D, S = gr.rows()
    assert D.shape == ref["D"].shape
    bad = np.argwhere(D != ref["D"])
    assert bad.shape[0] == 0, f"{label}: {bad.shape[0]} distance mismatches, first {bad[:3].tolist()}"
    bad = np.argwhere(S != ref["sigma"])
    assert bad.shape[0] == 0, f"{label}: {bad.shape[0]} sigma mismatches, first {bad[:3].tolist()}"
    bc = gr.scores()
    e = bc_err(bc, ref["bc"])
    assert e <= BC_TOL, f"{label}: BC error {e}"
    if estar:
        a, b, w = gr.estar()
        got = set(zip(a.tolist(), b.tolist(), w.tolist()))
        want = oracle.estar_arcs(g)
        assert got == want, f"{label}: E* differs ({len(got ^ want)} arcs)"
    for s in dags:
        one = oracle.source(g, s)
        a, b = gr.dag(s)
        assert dag_set(a, b) == dag_set(one["dag_a"], one["dag_b"]), f"{label}: DAG({s}) differs"
    check_preds(gr, g, dags, label)
    for s in deltas:
        one = oracle.source(g, s)
        e = bc_err(gr.delta(s), one["delta"])
        assert e <= BC_TOL, f"{label}: delta row {s} error {e}"
    return ref


def check_sampled(gr, g, sources, label=""):
    """Sampled parity on large graphs: rows and stored predecessors of the
    listed sources."""
    r = oracle.rows(g, sources)
    for i, s in enumerate(sources):
        D, S = gr.rows(int(s), 1)
        assert np.array_equal(D[0], r["D"][i]), f"{label}: distance row {s} differs"
        assert np.array_equal(S[0], r["sigma"][i]), f"{label}: sigma row {s} differs"
        e = bc_err(gr.delta(int(s)), r["delta"][i])
        assert e <= BC_TOL, f"{label}: delta row {s} error {e}"
    check_preds(gr, g, sources, label)


def make_ctx(n_max, slots=0, **kw):
    from paper_1311_2147_amd import bcinc

    return bcinc.Context(device=0, n_max=n_max, slots=slots, **kw)
