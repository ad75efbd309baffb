"""Row-update paths by the size of the candidate-target list T.

An arc insertion (u, v, 1) into a graph where v reaches exactly k sinks
(weight 1) that u reaches only at weight 1000 makes v and the k sinks the
candidates (w' + d(v,t) <= d(u,t) holds there and nowhere else), so |T| =
k + 1, and the 600 sources that reach u are affected.  The sizes cover every
lane-group width of the wave-level path (|T| <= 64: 1, 2, 8, 16, 32 and 64
lanes per row) and the workgroup path with the list (|T| > 64), all in one
batched step, under a schedule that lists every source and one that defers
all but the smallest.
"""
from __future__ import annotations

import numpy as np
import pytest

from gpu_util import check_full, make_ctx, say
from paper_1311_2147_amd import workloads as W

pytestmark = pytest.mark.gpu

N = 1024
U, V = 600, 601
KS = [0, 1, 6, 15, 31, 40, 63, 64, 100]


def fan_graph(k: int, seed: int) -> W.Graph:
    rng = np.random.default_rng(seed)
    src, dst, w = [], [], []
    for s in range(U):
        src.append(s)
        dst.append(U)
        w.append(1 + s % 7)
    for j in range(k):
        t = V + 1 + j
        src += [U, V]
        dst += [t, t]
        w += [1000, 1]
    # unrelated arcs among the remaining vertices (they reach neither u nor v)
    rest = np.arange(V + 1 + k, N)
    for _ in range(3 * len(rest)):
        a, b = rng.choice(rest, 2, replace=False)
        src.append(int(a))
        dst.append(int(b))
        w.append(int(rng.integers(1, 50)))
    keys = {}
    for a, b, c in zip(src, dst, w):
        keys.setdefault((a, b), c)
    a = np.array([x for x, _ in keys], np.int32)
    b = np.array([y for _, y in keys], np.int32)
    return W.Graph(N, True, a, b, np.array(list(keys.values()), np.int64))


@pytest.mark.parametrize("big_b", [512, 4])
def test_every_candidate_list_size_in_one_step(big_b):
    graphs = [fan_graph(k, 100 + k) for k in KS]
    ctx = make_ctx(N, slots=64)
    ctx.set_schedule(big_b=big_b)
    grs = [ctx.load_graph(g) for g in graphs]
    up = W.Update("edge", u=U, v=V, w=1, insert=True)
    ctx.wait(ctx.submit([(gr, up) for gr in grs]))
    for k, g, gr in zip(KS, graphs, grs):
        st = gr.stats()
        say(f"|T| = {k + 1}: |A| = {st['affected_sources']}, changed pairs {st['changed_pairs']}, "
            f"deferred {st['deferred_sources']}")
        assert st["affected_sources"] == U + 1
        check_full(gr, W.apply_update(g, up), f"|T|={k + 1} big_b={big_b}", dags=(0, U), deltas=(0, 5))
    ctx.close()
