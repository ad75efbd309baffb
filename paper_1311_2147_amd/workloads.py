"""Seeded synthetic graphs and incremental-update streams.

This module only draws random structure: graphs, weights, update requests and
arrival times.  It holds none of the betweenness arithmetic (no distances, no
path counts, no dependencies), so the CPU oracle and the GPU path can both be
fed from it without sharing any of the method.

Randomness is SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014) evaluated counter-style: draw i of a stream
with seed k is mix64(k + (i + 1) * GOLDEN).  Stream seeds are derived as
mix64 chains over (0x13112147, config, graph index, purpose), so every graph,
weight vector, update stream and arrival sequence is reproducible in isolation.

Graph model (Section 2 of the paper): directed graphs with positive weights;
an undirected graph is handled as its directed double G_D (Section 3,
undirected paragraph), but is *stored* here once per unordered pair with a < b.
Weights are integers, which keeps the tie tests of Lemma 2 and Lemma 4 exact.

Update model (Section 1, problem statement): an incremental edge update either
lowers the weight of an existing edge or inserts a missing one; a vertex
update does that on any subset of the edges incident to one vertex.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

MASK64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15
ROOT_SEED = 0x13112147

PURPOSE = {"structure": 1, "weights": 2, "updates": 3, "arrivals": 4, "sizes": 5}


def mix64(z: int) -> int:
    """SplitMix64 output function on a Python int (mod 2^64)."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def derive_seed(*parts: int) -> int:
    s = ROOT_SEED
    for p in parts:
        s = mix64((s ^ (int(p) & MASK64)) + GOLDEN)
    return s


def _mix64_np(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= np.uint64(0xBF58476D1CE4E5B9)
        z ^= z >> np.uint64(27)
        z *= np.uint64(0x94D049BB133111EB)
        z ^= z >> np.uint64(31)
    return z


class Rng:
    """Counter-based SplitMix64 stream with a position that advances per draw."""

    def __init__(self, seed: int):
        self.seed = seed & MASK64
        self.pos = 0

    def raw(self, k: int) -> np.ndarray:
        idx = np.arange(self.pos + 1, self.pos + 1 + k, dtype=np.uint64)
        self.pos += k
        with np.errstate(over="ignore"):
            z = np.uint64(self.seed) + idx * np.uint64(GOLDEN)
        return _mix64_np(z)

    def uniform(self, k: int) -> np.ndarray:
        """k doubles in [0, 1) from the top 53 bits."""
        return (self.raw(k) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)

    def integers(self, lo: int, hi: int, k: int) -> np.ndarray:
        """k integers uniform in [lo, hi] (inclusive); multiply-shift on 53-bit draws."""
        span = hi - lo + 1
        assert span >= 1
        return lo + np.floor(self.uniform(k) * span).astype(np.int64)

    def integer(self, lo: int, hi: int) -> int:
        return int(self.integers(lo, hi, 1)[0])

    def choice_without_replacement(self, pool_size: int, k: int) -> np.ndarray:
        """k distinct indices from range(pool_size) (partial Fisher-Yates)."""
        k = min(k, pool_size)
        if pool_size <= 4 * k or pool_size <= 4096:
            perm = np.arange(pool_size, dtype=np.int64)
            r = self.uniform(k)
            for i in range(k):
                j = i + int(r[i] * (pool_size - i))
                perm[i], perm[j] = perm[j], perm[i]
            return perm[:k].copy()
        out: list[int] = []
        seen: set[int] = set()
        while len(out) < k:
            for x in self.integers(0, pool_size - 1, 2 * (k - len(out))):
                x = int(x)
                if x not in seen:
                    seen.add(x)
                    out.append(x)
                    if len(out) == k:
                        break
        return np.asarray(out, dtype=np.int64)

    def shuffle(self, items: list) -> list:
        items = list(items)
        r = self.uniform(max(len(items), 1))
        for i in range(len(items) - 1, 0, -1):
            j = int(r[i] * (i + 1))
            items[i], items[j] = items[j], items[i]
        return items


# ----------------------------------------------------------------------------
# Graph container
# ----------------------------------------------------------------------------


@dataclass
class Graph:
    """Edge list of a weighted graph.

    directed=True: arcs (src[i] -> dst[i]).  directed=False: one entry per
    unordered edge, src[i] < dst[i], standing for both arcs of G_D.
    """

    n: int
    directed: bool
    src: np.ndarray  # int32
    dst: np.ndarray  # int32
    w: np.ndarray  # int64
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.src.shape[0])

    def arcs(self):
        """All directed arcs (of G_D when undirected) as three arrays."""
        if self.directed:
            return self.src, self.dst, self.w
        return (np.concatenate([self.src, self.dst]), np.concatenate([self.dst, self.src]),
                np.concatenate([self.w, self.w]))

    def copy(self) -> "Graph":
        return Graph(self.n, self.directed, self.src.copy(), self.dst.copy(), self.w.copy(), self.name)


@dataclass
class Update:
    """One incremental update request.

    kind == "edge":   (u, v, w) lowers or inserts arc/edge (u, v) to weight w.
    kind == "vertex": v plus a list of (a, b, w) edges, each incident to v.
    """

    kind: str
    u: int = -1
    v: int = -1
    w: int = 0
    edges: list = field(default_factory=list)
    insert: bool = False  # edge form only: the edge did not exist before

    def edge_list(self):
        if self.kind == "edge":
            return [(self.u, self.v, self.w)]
        return list(self.edges)


class ArcStore:
    """Current weights of a graph while an update stream is being drawn.

    Keys are a*n+b (directed) or min*n+max (undirected).  Base edges sit in a
    sorted numpy array; inserted edges in an overlay dict.
    """

    def __init__(self, g: Graph):
        self.n = g.n
        self.directed = g.directed
        a, b = g.src.astype(np.int64), g.dst.astype(np.int64)
        if not g.directed:
            a, b = np.minimum(a, b), np.maximum(a, b)
        keys = a * g.n + b
        order = np.argsort(keys, kind="stable")
        self.keys = keys[order]
        self.w = g.w.astype(np.int64)[order].copy()
        self.overlay: dict[int, int] = {}
        self.overlay_keys: list[int] = []
        if g.directed:
            by_dst = np.argsort(b * g.n + a, kind="stable")
            self.in_keys = (b * g.n + a)[by_dst]
            self.in_src = a[by_dst]
        self._base_index: dict[int, int] | None = None

    def key(self, a: int, b: int) -> int:
        if not self.directed and a > b:
            a, b = b, a
        return a * self.n + b

    def get(self, a: int, b: int):
        k = self.key(a, b)
        if k in self.overlay:
            return self.overlay[k]
        i = int(np.searchsorted(self.keys, k))
        if i < self.keys.shape[0] and int(self.keys[i]) == k:
            return int(self.w[i])
        return None

    def set(self, a: int, b: int, w: int):
        k = self.key(a, b)
        if k in self.overlay:
            self.overlay[k] = w
            return
        i = int(np.searchsorted(self.keys, k))
        if i < self.keys.shape[0] and int(self.keys[i]) == k:
            self.w[i] = w
        else:
            self.overlay[k] = w
            self.overlay_keys.append(k)

    def count(self) -> int:
        return int(self.keys.shape[0]) + len(self.overlay_keys)

    def edge_at(self, idx: int):
        if idx < self.keys.shape[0]:
            k, w = int(self.keys[idx]), int(self.w[idx])
        else:
            k = self.overlay_keys[idx - self.keys.shape[0]]
            w = self.overlay[k]
        return k // self.n, k % self.n, w

    def out_neighbours(self, v: int) -> list[int]:
        lo = int(np.searchsorted(self.keys, v * self.n))
        hi = int(np.searchsorted(self.keys, (v + 1) * self.n))
        res = [int(k) % self.n for k in self.keys[lo:hi]]
        res += [k % self.n for k in self.overlay_keys if k // self.n == v]
        if not self.directed:
            res += self.in_neighbours_undirected(v)
        return res

    def in_neighbours_undirected(self, v: int) -> list[int]:
        # undirected edges {a, v} with a < v: keys a*n + v
        cand = np.nonzero(self.keys % self.n == v)[0]
        res = [int(self.keys[i]) // self.n for i in cand]
        res += [k // self.n for k in self.overlay_keys if k % self.n == v]
        return res

    def in_neighbours(self, v: int) -> list[int]:
        assert self.directed
        lo = int(np.searchsorted(self.in_keys, v * self.n))
        hi = int(np.searchsorted(self.in_keys, (v + 1) * self.n))
        res = [int(a) for a in self.in_src[lo:hi]]
        res += [k // self.n for k in self.overlay_keys if k % self.n == v]
        return res

    def to_graph(self, name: str = "") -> Graph:
        ks = np.concatenate([self.keys, np.asarray(self.overlay_keys, dtype=np.int64)])
        ws = np.concatenate([self.w, np.asarray([self.overlay[k] for k in self.overlay_keys], dtype=np.int64)])
        order = np.argsort(ks, kind="stable")
        ks, ws = ks[order], ws[order]
        return Graph(self.n, self.directed, (ks // self.n).astype(np.int32), (ks % self.n).astype(np.int32),
                     ws.astype(np.int64), name)


def apply_update(g: Graph, up: Update) -> Graph:
    """Edge list after an update (host bookkeeping only)."""
    st = ArcStore(g)
    for a, b, w in up.edge_list():
        st.set(a, b, w)
    return st.to_graph(g.name)


# ----------------------------------------------------------------------------
# Graph families
# ----------------------------------------------------------------------------


def gnp_undirected(n: int, avg_deg: float, wmax: int, seed: int, name: str = "gnp") -> Graph:
    """Undirected G(n, p) with p = avg_deg/(n-1); weights uniform in {1..wmax}."""
    rs = Rng(derive_seed(seed, PURPOSE["structure"]))
    p = avg_deg / (n - 1)
    iu, ju = np.triu_indices(n, k=1)
    keep = rs.uniform(iu.shape[0]) < p
    src, dst = iu[keep].astype(np.int32), ju[keep].astype(np.int32)
    w = Rng(derive_seed(seed, PURPOSE["weights"])).integers(1, wmax, src.shape[0])
    return Graph(n, False, src, dst, w, name)


def directed_out_degree(n: int, k: int, wmax: int, seed: int, name: str = "outdeg") -> Graph:
    """Each vertex gets k distinct uniform out-targets (no self-loops)."""
    rs = Rng(derive_seed(seed, PURPOSE["structure"]))
    src = np.repeat(np.arange(n, dtype=np.int64), k)
    dst = np.empty(n * k, dtype=np.int64)
    for a in range(n):
        picks = rs.choice_without_replacement(n - 1, k)
        picks = picks + (picks >= a)  # skip the self-loop slot
        dst[a * k:(a + 1) * k] = np.sort(picks)
    w = Rng(derive_seed(seed, PURPOSE["weights"])).integers(1, wmax, n * k)
    return Graph(n, True, src.astype(np.int32), dst.astype(np.int32), w, name)


def complete_undirected(n: int, wmax: int, seed: int, name: str = "complete") -> Graph:
    """K_n with weights uniform in {1..wmax} (wmax = n^2 in the dense workloads)."""
    iu, ju = np.triu_indices(n, k=1)
    w = Rng(derive_seed(seed, PURPOSE["weights"])).integers(1, wmax, iu.shape[0])
    return Graph(n, False, iu.astype(np.int32), ju.astype(np.int32), w, name)


def chung_lu_directed(n: int, beta: float, avg_deg: float, wmax: int, seed: int,
                      name: str = "chunglu") -> Graph:
    """Directed Chung-Lu graph with power-law expected degrees.

    theta_i ~ (i+1)^(-1/(beta-1)); independent random vertex permutations for
    the out- and in-sequences; m = avg_deg*n distinct arcs sampled with source
    ~ theta_out and target ~ theta_in, self-loops and duplicates rejected.
    """
    rs = Rng(derive_seed(seed, PURPOSE["structure"]))
    m = int(round(avg_deg * n))
    theta = (np.arange(1, n + 1, dtype=np.float64)) ** (-1.0 / (beta - 1.0))
    cdf = np.cumsum(theta)
    cdf /= cdf[-1]
    perm_out = np.argsort(rs.uniform(n), kind="stable")
    perm_in = np.argsort(rs.uniform(n), kind="stable")
    seen = np.zeros(0, dtype=np.int64)
    got_keys: list[np.ndarray] = []
    have = 0
    seen_set = set()
    while have < m:
        batch = max(2 * (m - have), 1024)
        a = perm_out[np.minimum(np.searchsorted(cdf, rs.uniform(batch), side="right"), n - 1)]
        b = perm_in[np.minimum(np.searchsorted(cdf, rs.uniform(batch), side="right"), n - 1)]
        keys = a.astype(np.int64) * n + b.astype(np.int64)
        keys = keys[a != b]
        # keep first occurrences in draw order
        _, first = np.unique(keys, return_index=True)
        keys = keys[np.sort(first)]
        fresh = []
        for kk in keys.tolist():
            if kk not in seen_set:
                seen_set.add(kk)
                fresh.append(kk)
                if have + len(fresh) == m:
                    break
        got_keys.append(np.asarray(fresh, dtype=np.int64))
        have += len(fresh)
    del seen
    keys = np.concatenate(got_keys)
    w = Rng(derive_seed(seed, PURPOSE["weights"])).integers(1, wmax, m)
    return Graph(n, True, (keys // n).astype(np.int32), (keys % n).astype(np.int32), w, name)


# Closed-form families (used to pin the oracle).


def path_graph(n: int, c: int = 1, directed: bool = False) -> Graph:
    s = np.arange(n - 1, dtype=np.int32)
    return Graph(n, directed, s, s + 1, np.full(n - 1, c, dtype=np.int64), "path")


def cycle_graph(n: int, c: int = 1, directed: bool = False) -> Graph:
    s = np.arange(n, dtype=np.int32)
    d = (s + 1) % n
    if not directed:
        a, b = np.minimum(s, d), np.maximum(s, d)
        return Graph(n, False, a, b, np.full(n, c, dtype=np.int64), "cycle")
    return Graph(n, True, s, d.astype(np.int32), np.full(n, c, dtype=np.int64), "dcycle")


def star_graph(n: int, c: int = 1) -> Graph:
    leaves = np.arange(1, n, dtype=np.int32)
    return Graph(n, False, np.zeros(n - 1, dtype=np.int32), leaves, np.full(n - 1, c, dtype=np.int64), "star")


def complete_graph_equal(n: int, c: int = 1) -> Graph:
    iu, ju = np.triu_indices(n, k=1)
    return Graph(n, False, iu.astype(np.int32), ju.astype(np.int32), np.full(iu.shape[0], c, dtype=np.int64),
                 "kn")


def grid_graph(r: int, c: int, wt: int = 1) -> Graph:
    src, dst = [], []
    for i in range(r):
        for j in range(c):
            v = i * c + j
            if j + 1 < c:
                src.append(v)
                dst.append(v + 1)
            if i + 1 < r:
                src.append(v)
                dst.append(v + c)
    return Graph(r * c, False, np.asarray(src, dtype=np.int32), np.asarray(dst, dtype=np.int32),
                 np.full(len(src), wt, dtype=np.int64), "grid")


def random_small(n: int, p: float, wmax: int, seed: int, directed: bool = True) -> Graph:
    """Small random graph for brute-force checks (ties frequent when wmax is small)."""
    rs = Rng(derive_seed(seed, PURPOSE["structure"]))
    if directed:
        a, b = np.nonzero(~np.eye(n, dtype=bool))
    else:
        a, b = np.triu_indices(n, k=1)
    keep = rs.uniform(a.shape[0]) < p
    src, dst = a[keep].astype(np.int32), b[keep].astype(np.int32)
    w = Rng(derive_seed(seed, PURPOSE["weights"])).integers(1, wmax, src.shape[0])
    return Graph(n, directed, src, dst, w, "small")


# ----------------------------------------------------------------------------
# Update streams
# ----------------------------------------------------------------------------


def _draw_insertion(st: ArcStore, rs: Rng, wmax: int, avoid=()):
    n = st.n
    for _ in range(100000):
        a, b = (int(x) for x in rs.integers(0, n - 1, 2))
        if a == b or st.get(a, b) is not None or st.key(a, b) in avoid:
            continue
        return a, b, rs.integer(1, wmax)
    return None


def _draw_decrease(st: ArcStore, rs: Rng):
    cnt = st.count()
    for _ in range(100000):
        a, b, w = st.edge_at(rs.integer(0, cnt - 1))
        if w >= 2:
            return a, b, rs.integer(1, w - 1)
    return None


def _draw_vertex(st: ArcStore, rs: Rng, k: int, wmax: int, fill_insert: bool = True):
    """Vertex update at a uniform v: up to k existing incident edges with w >= 2,
    each lowered to U[1, w-1]; if fewer than k qualify, the rest are insertions
    (direction 50/50 for directed graphs)."""
    n = st.n
    v = rs.integer(0, n - 1)
    cands = []
    if st.directed:
        cands += [(v, x) for x in st.out_neighbours(v)]
        cands += [(x, v) for x in st.in_neighbours(v)]
    else:
        if st.count() == n * (n - 1) // 2:  # complete graph: every x is a neighbour
            xs = rs.choice_without_replacement(n - 1, 4 * k)
            cands = [(v, int(x) + (int(x) >= v)) for x in xs]
        else:
            cands = [(v, x) for x in st.out_neighbours(v)]
    cands = [(a, b) for (a, b) in cands if (st.get(a, b) or 0) >= 2]
    picks = rs.choice_without_replacement(len(cands), k) if cands else []
    edges, used = [], set()
    for i in picks:
        a, b = cands[int(i)]
        w = st.get(a, b)
        edges.append((a, b, rs.integer(1, w - 1)))
        used.add(st.key(a, b))
    tries = 0
    while fill_insert and len(edges) < k and tries < 10000:
        tries += 1
        x = rs.integer(0, n - 1)
        if x == v:
            continue
        a, b = (v, x) if (not st.directed or rs.uniform(1)[0] < 0.5) else (x, v)
        kk = st.key(a, b)
        if st.get(a, b) is not None or kk in used:
            continue
        edges.append((a, b, rs.integer(1, wmax)))
        used.add(kk)
    return Update("vertex", v=v, edges=edges)


def edge_stream(g: Graph, n_ins: int, n_dec: int, wmax: int, seed: int) -> list[Update]:
    """n_ins insertions and n_dec decreases in a seeded shuffled order, drawn
    sequentially against the evolving graph."""
    rs = Rng(derive_seed(seed, PURPOSE["updates"]))
    kinds = rs.shuffle(["ins"] * n_ins + ["dec"] * n_dec)
    st = ArcStore(g)
    out = []
    for kd in kinds:
        if kd == "ins":
            a, b, w = _draw_insertion(st, rs, wmax)
            out.append(Update("edge", u=a, v=b, w=w, insert=True))
        else:
            a, b, w = _draw_decrease(st, rs)
            out.append(Update("edge", u=a, v=b, w=w))
        st.set(a, b, w)
    return out


def vertex_stream(g: Graph, count: int, k: int, wmax: int, seed: int) -> list[Update]:
    rs = Rng(derive_seed(seed, PURPOSE["updates"]))
    st = ArcStore(g)
    out = []
    for _ in range(count):
        up = _draw_vertex(st, rs, k, wmax)
        for a, b, w in up.edges:
            st.set(a, b, w)
        out.append(up)
    return out


def mixed_stream(g: Graph, count: int, wmax: int, seed: int, p_ins: float, p_dec: float, k_vertex: int,
                 rs: Rng | None = None, st: ArcStore | None = None) -> list[Update]:
    """Mix of insertions (p_ins), decreases (p_dec) and vertex updates (rest)."""
    rs = rs or Rng(derive_seed(seed, PURPOSE["updates"]))
    st = st or ArcStore(g)
    out = []
    for _ in range(count):
        full = st.count() == (g.n * (g.n - 1) if g.directed else g.n * (g.n - 1) // 2)
        r = rs.uniform(1)[0]
        if r < p_ins + p_dec:
            drawn = _draw_insertion(st, rs, wmax) if (r < p_ins and not full) else _draw_decrease(st, rs)
            if drawn is None:  # nothing left to lower or insert
                continue
            a, b, w = drawn
            up = Update("edge", u=a, v=b, w=w, insert=st.get(a, b) is None)
        else:
            up = _draw_vertex(st, rs, k_vertex, wmax)
        for a, b, w in up.edge_list():
            st.set(a, b, w)
        out.append(up)
    return out


def poisson_arrivals(count: int, rate_per_s: float, seed: int) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process with the given rate."""
    u = Rng(derive_seed(seed, PURPOSE["arrivals"])).uniform(count)
    gaps = -np.log1p(-u) / rate_per_s
    return np.cumsum(gaps)


# ----------------------------------------------------------------------------
# The five workloads
# ----------------------------------------------------------------------------


def config1(seed: int = 0):
    """Undirected G(64, 4/63), weights {1..10}; 8 insertions + 8 decreases."""
    g = gnp_undirected(64, 4.0, 10, derive_seed(1, 0, seed), "c1-gnp64")
    ups = edge_stream(g, 8, 8, 10, derive_seed(1, 0, seed))
    return g, ups


def config2(seed: int = 0, n: int = 4096, n_updates: int = 256):
    """Directed out-degree-8 graph, weights {1..100}; half insertions, half decreases."""
    g = directed_out_degree(n, 8, 100, derive_seed(2, 0, seed), f"c2-outdeg8-n{n}")
    ups = edge_stream(g, n_updates // 2, n_updates - n_updates // 2, 100, derive_seed(2, 0, seed))
    return g, ups


def config3(seed: int = 0, n: int = 2048, n_updates: int = 64, k: int = 32):
    """Complete undirected graph, weights {1..n^2}; vertex updates lowering k incident edges."""
    g = complete_undirected(n, n * n, derive_seed(3, 0, seed), f"c3-complete-n{n}")
    ups = vertex_stream(g, n_updates, k, n * n, derive_seed(3, 0, seed))
    return g, ups


def config4_sizes(count: int = 64, seed: int = 0, lo: int = 256, hi: int = 4096) -> list[int]:
    u = Rng(derive_seed(4, 0, seed, PURPOSE["sizes"])).uniform(count)
    return [int(round(math.exp(math.log(lo) + x * (math.log(hi) - math.log(lo))))) for x in u]


def config4(seed: int = 0, count: int = 64, n_updates: int = 32, lo: int = 256, hi: int = 4096):
    """Many independent graphs: first half directed out-degree 8 (weights {1..100}),
    second half complete undirected (weights {1..n^2}); each with its own stream of
    70% edge updates and 30% vertex updates touching 16 incident edges."""
    sizes = config4_sizes(count, seed, lo, hi)
    out = []
    for gi, n in enumerate(sizes):
        if gi < count // 2:
            g = directed_out_degree(n, 8, 100, derive_seed(4, gi, seed), f"c4-outdeg8-n{n}")
            ups = mixed_stream(g, n_updates, 100, derive_seed(4, gi, seed), 0.35, 0.35, 16)
        else:
            g = complete_undirected(n, n * n, derive_seed(4, gi, seed), f"c4-complete-n{n}")
            ups = mixed_stream(g, n_updates, n * n, derive_seed(4, gi, seed), 0.0, 0.70, 16)
        out.append((g, ups))
    return out


C5_SIZES = (4096, 8192, 16384, 32768)


def config5_graph(n: int, gi: int, seed: int = 0) -> Graph:
    """Directed Chung-Lu graph, degree exponent 2.5, mean degree 16, weights {1..1000}."""
    return chung_lu_directed(n, 2.5, 16.0, 1000, derive_seed(5, gi, seed), f"c5-chunglu-n{n}-g{gi}")


def config5_stream(graphs: list[Graph], count: int, seed: int = 0):
    """Updates spread uniformly over the graphs: 35% insertions, 35% decreases,
    30% vertex updates touching 16 incident arcs.  Returns (graph index, update)."""
    rs = Rng(derive_seed(5, 1000, seed, PURPOSE["updates"]))
    stores = [ArcStore(g) for g in graphs]
    out = []
    for _ in range(count):
        gi = rs.integer(0, len(graphs) - 1)
        up = mixed_stream(graphs[gi], 1, 1000, 0, 0.35, 0.35, 16, rs=rs, st=stores[gi])[0]
        out.append((gi, up))
    return out
