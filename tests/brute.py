"""Brute-force enumeration of all simple paths, for pinning the oracle on tiny graphs.

Every quantity comes straight from its definition (Section 2 of the paper), by
listing paths, never by a recurrence:
  d(s,t)       minimum weight over all s-t paths;
  sigma_st     number of s-t paths of that weight (sigma_ss = 1);
  sigma_st(v)  number of those passing through v (Eq.2 as a count);
  BC(v)        sum over ordered s != v != t with sigma_st > 0 of
               sigma_st(v) / sigma_st (Eq.3);
  DAG(s)       last arcs of the shortest s-t paths, over all t (which is
               what the predecessor sets of Eq.1 collect);
  delta_s.(v)  sum over t of sigma_st(v) / sigma_st.
Positive weights make every shortest path simple, so simple paths suffice.
Exponential time: graphs of at most ~9 vertices.
"""
from __future__ import annotations

from fractions import Fraction

INF = None


def _adjacency(g):
    adj = {v: [] for v in range(g.n)}
    for a, b, w in zip(g.src.tolist(), g.dst.tolist(), g.w.tolist()):
        adj[a].append((b, w))
        if not g.directed:
            adj[b].append((a, w))
    return adj


def all_simple_paths(g, s):
    """Yield (path vertex list, weight) for every simple path starting at s."""
    adj = _adjacency(g)
    path, on = [s], {s}

    def rec(x, wsum):
        yield list(path), wsum
        for y, w in adj[x]:
            if y in on:
                continue
            path.append(y)
            on.add(y)
            yield from rec(y, wsum + w)
            path.pop()
            on.discard(y)

    yield from rec(s, 0)


def brute(g):
    """Exact D, sigma, BC (as Fractions), DAG(s) arc sets and delta rows."""
    n = g.n
    D = [[INF] * n for _ in range(n)]
    S = [[0] * n for _ in range(n)]
    paths_by = [[[] for _ in range(n)] for _ in range(n)]
    for s in range(n):
        for p, wsum in all_simple_paths(g, s):
            paths_by[s][p[-1]].append((p, wsum))
    bc = [Fraction(0)] * n
    delta = [[Fraction(0)] * n for _ in range(n)]
    dags = []
    for s in range(n):
        arcs = set()
        for t in range(n):
            ps = paths_by[s][t]
            if not ps:
                continue
            best = min(wsum for _, wsum in ps)
            shortest = [p for p, wsum in ps if wsum == best]
            D[s][t] = best
            S[s][t] = len(shortest)
            for p in shortest:
                if len(p) >= 2:
                    arcs.add((p[-2], p[-1]))
            if t == s:
                continue
            for v in range(n):
                if v == s or v == t:
                    continue
                through = sum(1 for p in shortest if v in p)
                if through:
                    frac = Fraction(through, len(shortest))
                    bc[v] += frac
                    delta[s][v] += frac
        dags.append(arcs)
    return {"D": D, "sigma": S, "bc": bc, "dag": dags, "delta": delta}
