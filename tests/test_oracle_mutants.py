"""Pin strength: plant plausible mistakes in a copy of the oracle's C code (on
the CPU) and check that the pins reject every one of them.

Each mutant is a textual edit of oracle/brandes.c compiled with gcc into a
temporary library; the pins below are a compact subset of the ones in
test_oracle_pins.py (brute force, closed forms, library distances).
"""
from __future__ import annotations

import math
import os
import subprocess

import numpy as np
import pytest

import oracle
from brute import brute
from paper_1311_2147_amd import workloads as W

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "brandes.c")

MUTANTS = {
    "dropped_one_in_eq4": ("(1.0 + wk->delta[x])", "(wk->delta[x])"),
    "inverted_sigma_ratio": ("(double)wk->sigma[a] / (double)wk->sigma[x]", "(double)wk->sigma[x] / (double)wk->sigma[a]"),
    "tie_overwrites_count": ("if (__builtin_add_overflow(wk->sigma[b], wk->sigma[a], &wk->sigma[b])) return OR_SIGMA_OVERFLOW;",
                             "wk->sigma[b] = wk->sigma[a];"),
    "strict_relax_became_weak": ("if (nd < wk->dist[b]) {", "if (nd <= wk->dist[b]) {"),
    "source_counted_in_bc": ("if (x != s && bc) bc[x] += wk->delta[x];", "if (bc) bc[x] += wk->delta[x];"),
    "predecessor_test_loosened": ("wk->dist[a] + g->in_w[e] == wk->dist[x])\n                wk->delta[a]",
                                  "wk->dist[a] + g->in_w[e] >= wk->dist[x])\n                wk->delta[a]"),
    "reverse_arc_transposed": ("g->out_dst[o] = a; g->out_w[o] = w[i];", "g->out_dst[o] = b; g->out_w[o] = w[i];"),
    "weight_off_by_one": ("int64_t nd = wk->dist[a] + g->out_w[e];", "int64_t nd = wk->dist[a] + g->out_w[e] + 1;"),
}


def _pins_pass() -> bool:
    try:
        for directed in (True, False):
            for seed in range(4):
                g = W.random_small(7, 0.45, 3, seed=500 + seed, directed=directed)
                ref = brute(g)
                got = oracle.brandes(g)
                for s in range(g.n):
                    for t in range(g.n):
                        want = ref["D"][s][t]
                        if got["D"][s, t] != (oracle.INF if want is None else want):
                            return False
                        if int(got["sigma"][s, t]) != ref["sigma"][s][t]:
                            return False
                if np.abs(got["bc"] - np.array([float(x) for x in ref["bc"]])).max() > 1e-10:
                    return False
        n = 9
        got = oracle.brandes(W.path_graph(n))
        if np.abs(got["bc"] - 2 * np.arange(n) * (n - 1 - np.arange(n))).max() > 1e-10:
            return False
        got = oracle.brandes(W.cycle_graph(8))
        if np.abs(got["bc"] - 9).max() > 1e-10:
            return False
        grid = oracle.source(W.grid_graph(5, 5), 0)
        if int(grid["sigma"][24]) != math.comb(8, 4):
            return False
    except oracle.OracleError:
        return False
    return True


def test_unmutated_oracle_passes_the_compact_pins():
    assert _pins_pass()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation anchor for {name} not found exactly once"
    mutated = tmp_path / "mutant.c"
    mutated.write_text(text.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O1", "-std=c11", "-shared", "-fPIC", "-pthread", str(mutated), "-o", str(lib)],
                   check=True, capture_output=True)
    prev = oracle.use_library(str(lib))
    try:
        assert not _pins_pass(), f"mutant {name} survived the pins"
    finally:
        oracle.restore_library(prev)
