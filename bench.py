#!/usr/bin/env python3
"""Benchmark: incremental betweenness-centrality updates per second at n = 32768.

Workload (synthetic, seeded): six resident directed Chung-Lu graphs with
n = 32768 (17.2 GB of state each), degree exponent 2.5, mean out-degree 16 (m = 16n arcs), integer
weights uniform in {1..1000}; each graph gets its own stream of updates drawn
35% insertions, 35% decreases to a uniform lower weight, 30% vertex updates
touching 16 incident arcs.  Inputs are resident in HBM before timing starts;
every leg's requests are marshalled into their C arrays beforehand, and
timed regions run with Python's garbage collector paused.

A step is one pass of the whole update path over one batch: one update on
each resident graph, processed together by one batched launch sequence (scan,
row v'', E* merge, per-source kernels, E* filter, commit) replayed from
captured HIP graphs.  value = updates completed per second over the timed
steps.

Besides the headline the run measures:
  * the plain path on the same updates: device clones of the graphs taken
    before the timed window get the same requests one at a time, with the
    library's default schedule, synchronised after each, launched directly
    (no HIP graph, no batching); both legs must reach the same state;
  * the same with two graphs per step (the two n = 32768 graphs of the
    served workload), batched and plain, on 300 more updates of graphs 0
    and 1;
  * the row kernel's achieved HBM bandwidth over the timed window;
  * a full GPU recompute (the static pass) and the recompute over E*;
  * loads of dense graphs (complete, weights up to n^2) by the checked
    search over a subset containing E*, against the search over every arc;
  * a dedicated 1000-update stream on one freshly loaded graph;
  * the 64-graph batched workload (n from 256 to 4096), batched against the
    plain path on clones;
  * the out-degree-8 stream at n = 4096 and the complete graph's vertex
    updates at n = 2048, one update per step and one at a time, beside the
    oracle's time per update;
  * the served workload at full shape: 8 resident Chung-Lu graphs (n = 4096,
    8192, 16384, 32768, two of each), a closed loop for the saturation rate
    (and the plain path on its requests, on clones), and Poisson streams over
    them, served by
    continuous batching at 0.5, 0.8 (10,000 updates) and 0.95 times the
    closed-loop saturation rate, p50/p99 per graph size; then admission
    under a memory budget that holds only some graphs at once;
  * the multi-core CPU incremental comparator on a short sample;
  * the CPU oracle (from-scratch Brandes): one complete BC recompute of the
    n = 32768 graph on all host cores, and a one-core figure on a sample.
Prints one JSON line, which also names the system (GPU, ROCm and HIP
versions, host CPU and threads, the GPU clocks rocm-smi reports once idle).
"""
from __future__ import annotations

import argparse
import contextlib
import gc
import hashlib
import json
import os
import platform
import re
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_rows_chunglu_n32768_traffic.md")
KERNEL_SOURCES = ("paper_1311_2147_amd/csrc/bc_kernels.hip", "paper_1311_2147_amd/csrc/bc_device.h")


@contextlib.contextmanager
def quiet_gc():
    """A timed region with Python's cyclic garbage collector paused (after a
    collection), as timeit runs: a collection over the bench's own heap is
    no cost of the library.  Requests are marshalled before the region."""
    gc.collect()
    gc.disable()
    try:
        yield
    finally:
        gc.enable()


def kernel_sources_sha256():
    """SHA-256 of the kernel sources' code: comments and whitespace are
    dropped first, so that only a change of the code itself invalidates the
    committed counter figures."""
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel)) as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()


def committed_traffic(graphs: int, n: int):
    """HBM bytes per row-kernel launch from the committed counter summary,
    or None when there is none, the kernel sources changed since, or it was
    taken on another workload (graphs per launch, n)."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    text = open(TRAFFIC_FILE).read()
    sha = re.search(r"kernel_sources_sha256:\s*([0-9a-f]{64})", text)
    val = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", text)
    g = re.search(r"graphs_per_launch:\s*(\d+)", text)
    nn = re.search(r"vertices:\s*(\d+)", text)
    if not sha or not val or not g or not nn or sha.group(1) != kernel_sources_sha256():
        return None
    if int(g.group(1)) != graphs or int(nn.group(1)) != n:
        return None
    return float(val.group(1))


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def system_info():
    """Where the run happened: the GPU, the runtime versions, the host CPU and
    the clocks rocm-smi reports once the work is done (the idle power state,
    not the clocks under load; None where a figure is not available)."""
    import torch

    p = torch.cuda.get_device_properties(0)
    info = {"gpu": p.name, "arch": getattr(p, "gcnArchName", None), "compute_units": p.multi_processor_count,
            "hbm_gib": round(p.total_memory / 2**30, 1), "hip": torch.version.hip, "torch": torch.__version__,
            "rocm": None, "cpu": cpu_model(), "host_threads": len(os.sched_getaffinity(0)),
            "clocks_idle_after_run": None}
    try:
        with open("/opt/rocm/.info/version") as f:
            info["rocm"] = f.read().strip()
    except OSError:
        pass
    try:
        res = subprocess.run(["rocm-smi", "--showclocks", "--json"], capture_output=True, text=True, timeout=30)
        cards = json.loads(res.stdout)
        info["clocks_idle_after_run"] = {k.rstrip(":"): v for card in cards.values() if isinstance(card, dict)
                          for k, v in card.items() if "clk" in k.lower()}
    except (OSError, ValueError, subprocess.SubprocessError):
        pass
    return info


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=150)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--n", type=int, default=32768)
    ap.add_argument("--graphs", type=int, default=6)
    ap.add_argument("--legs",
                    default="batched,plain,two,recompute,loader,single,served,budget,c4,c2c3,cpuinc,cpu,copy")
    ap.add_argument("--served-updates", type=int, default=10000, help="updates of the 0.8x served run")
    ap.add_argument("--cpu-updates", type=int, default=12, help="updates of the CPU incremental comparator's sample")
    ap.add_argument("--cpu-one-core-sources", type=int, default=512, help="sources of the one-core oracle sample")
    ap.add_argument("--single", type=int, default=1000, help="updates of the dedicated single-graph stream")
    ap.add_argument("--tune-sample", type=int, default=8, help="updates per graph in the autotuner's sample (0: no tuning)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the incremental path is "
              "measured on one MI355X and its multi-GPU sharding is a design note, not a measured path.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1311_2147_amd import bcinc
    from paper_1311_2147_amd import serve
    from paper_1311_2147_amd import workloads as W

    legs = set(args.legs.split(","))
    n, G, K, Wm = args.n, args.graphs, args.steps, args.warmup

    # ---------------------------------------------------------------- inputs
    t = time.perf_counter()
    sizes = list(W.C5_SIZES)
    gidx = [i for i in range(4 * G) if sizes[i % 4] == n][:G] if n in sizes else list(range(G))
    graphs = [W.config5_graph(n, gi) for gi in gidx]
    per_graph = Wm + K + 8
    # the two-graph leg continues the streams of graphs 0 and 1 (a longer
    # stream starts with the same updates)
    two = "two" in legs and G >= 2
    streams = [W.mixed_stream(g, per_graph + (K if two and i < 2 else 0), 1000, W.derive_seed(5, 2000 + gi),
                              0.35, 0.35, 16) for i, (g, gi) in enumerate(zip(graphs, gidx))]
    log(f"generated {G} graphs n={n} m={graphs[0].m} and {per_graph} updates each in {time.perf_counter() - t:.1f}s")
    cursor = [0] * G

    def take(i):
        up = streams[i][cursor[i]]
        cursor[i] += 1
        return up

    ctx = bcinc.Context(device=0, n_max=n, timing=True)
    t = time.perf_counter()
    grs = [ctx.load_graph(g) for g in graphs]
    ctx.sync()
    load_s = (time.perf_counter() - t) / G
    log(f"loaded (static GPU Brandes) {load_s:.3f}s per graph; E* arcs {grs[0].stats()['estar_arcs']}")

    # --------------------------------------------------------------- autotune
    # The schedule autotuner replays a separately drawn sample of updates
    # (same mix, different seed) on device clones of the graphs; the chosen
    # schedule serves the batched and served legs, the plain leg keeps the
    # library default.
    default_sched = ctx.schedule()
    tuned = default_sched
    tune_s = 0.0
    if args.tune_sample > 0:
        samples = [W.mixed_stream(g, args.tune_sample, 1000, W.derive_seed(5, 4000 + gi), 0.35, 0.35, 16)
                   for g, gi in zip(graphs, gidx)]
        sample = [(grs[i], samples[i][k]) for k in range(args.tune_sample) for i in range(G)]
        t = time.perf_counter()
        tuned = ctx.autotune(sample)
        tune_s = time.perf_counter() - t
        log(f"autotune over {len(sample)} sample updates in {tune_s:.2f}s: {tuned} (default {default_sched})")

    # ---------------------------------------------------------------- warmup
    for _ in range(Wm):
        ctx.wait(ctx.submit([(grs[i], take(i)) for i in range(G)]))
    ctx.sync()

    # ---------------------------------------------------------------- batched
    # the plain leg's twins: device clones of both graphs at this point
    twins = [gr.clone() for gr in grs] if "plain" in legs else []
    ctx.sync()
    before = [gr.stats() for gr in grs]
    reqs = []
    for _ in range(K):
        for i in range(G):
            reqs.append((grs[i], take(i)))
    stream = ctx.stream
    batch = ctx.batch(reqs)
    ctx.reset_timing()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    with quiet_gc():
        t0 = time.perf_counter()
        ev0.record(stream)
        ticket = ctx.submit(batch)
        ev1.record(stream)
        ctx.wait(ticket)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    window_timing = ctx.timing()
    after = [gr.stats() for gr in grs]
    ctx.sync()
    value = K * G / wall
    aff_b = sum(after[i]['total_affected'] - before[i]['total_affected'] for i in range(G))
    chg_b = sum(after[i]['total_changed'] - before[i]['total_changed'] for i in range(G))
    alg_bytes = sum(after[i]['total_scan_bytes'] - before[i]['total_scan_bytes'] for i in range(G))
    log(f"batched: {K} steps x {G} graphs in {wall * 1e3:.1f} ms wall ({gpu_ms:.1f} ms stream) -> {value:.1f} updates/s; "
        f"|A| per update {aff_b / (K * G):.0f}, changed pairs per update {chg_b / (K * G):.0f}")

    # ------------------------------------------------------------ row kernel
    # HIP events on the library's stream bracket the row kernel in every step
    # of the timed window (one launch per step); its algorithmic bytes (the
    # device counts them per update: 4n per affected row scanned, or 4 per
    # candidate target when the candidates are scanned instead, plus 8 per
    # changed pair) are summed over the same updates.
    rows_ms = window_timing["rows_ms"]
    launches = max(window_timing["steps"], 1)
    achieved = alg_bytes / (rows_ms / 1e3) / 1e9 if rows_ms > 0 else 0.0
    log(f"row kernel over the timed window: {launches} launches, avg {rows_ms / launches:.3f} ms, "
        f"{alg_bytes / launches / 1e6:.1f} MB/launch -> {achieved:.1f} GB/s "
        f"({100 * achieved / HBM_PEAK_GBS:.2f}% of HBM peak); per-source kernels avg "
        f"{window_timing['source_ms'] / launches:.3f} ms, step avg {window_timing['step_ms'] / launches:.3f} ms")

    comparators = {"batched_window": {"updates": K * G, "affected_per_update": aff_b / (K * G),
                                      "changed_pairs_per_update": chg_b / (K * G)}}
    # ---------------------------------------------------------------- plain
    # the same requests, in the same order, on the twins: one update at a
    # time, default schedule, synchronised after each, no HIP graph
    if "plain" in legs:
        tb = [tw.stats() for tw in twins]
        calls = [twins[grs.index(gr)].prepare(up) for gr, up in reqs]
        ctx.set_schedule(**default_sched)
        torch.cuda.synchronize()
        with quiet_gc():
            t0 = time.perf_counter()
            for call in calls:
                call()
                ctx.sync()
            plain_s = time.perf_counter() - t0
        ctx.set_schedule(**tuned)
        ta = [tw.stats() for tw in twins]
        same = all(twins[i].state_hash() == grs[i].state_hash() for i in range(G))
        aff_p = sum(ta[i]['total_affected'] - tb[i]['total_affected'] for i in range(G))
        chg_p = sum(ta[i]['total_changed'] - tb[i]['total_changed'] for i in range(G))
        comparators["plain_updates_per_s"] = len(reqs) / plain_s
        comparators["batched_over_plain"] = value / (len(reqs) / plain_s)
        comparators["plain_window"] = {"updates": len(reqs), "affected_per_update": aff_p / len(reqs),
                                       "changed_pairs_per_update": chg_p / len(reqs), "same_state_as_batched": same}
        log(f"plain (same {len(reqs)} updates on clones): {len(reqs) / plain_s:.1f} updates/s, batched/plain "
            f"{comparators['batched_over_plain']:.3f}, |A| {aff_p / len(reqs):.0f}, same state {same}")
        for tw in twins:
            tw.free()
        del twins
        torch.cuda.empty_cache()

    # ---------------------------------------------------------------- two graphs
    # The same measurement with two graphs per step (the two n = 32768 graphs
    # of the served workload): graphs 0 and 1 continue their streams for K
    # more steps, batched, and device clones taken before get the same
    # updates one at a time (default schedule, synchronised after each).
    if two:
        pair = grs[:2]
        twins2 = [gr.clone() for gr in pair]
        reqs2 = [(pair[i], take(i)) for _ in range(K) for i in range(2)]
        batch2 = ctx.batch(reqs2)
        calls2 = [twins2[pair.index(gr)].prepare(up) for gr, up in reqs2]
        ctx.sync()
        torch.cuda.synchronize()
        with quiet_gc():
            t0 = time.perf_counter()
            ctx.wait(ctx.submit(batch2))
            torch.cuda.synchronize()
            two_b = len(reqs2) / (time.perf_counter() - t0)
        ctx.set_schedule(**default_sched)
        torch.cuda.synchronize()
        with quiet_gc():
            t0 = time.perf_counter()
            for call in calls2:
                call()
                ctx.sync()
            two_p = len(reqs2) / (time.perf_counter() - t0)
        ctx.set_schedule(**tuned)
        two_same = all(twins2[i].state_hash() == pair[i].state_hash() for i in range(2))
        comparators["two_graphs"] = {"updates": len(reqs2), "batched_updates_per_s": two_b,
                                     "plain_updates_per_s": two_p, "batched_over_plain": two_b / two_p,
                                     "same_state": two_same}
        log(f"two graphs per step ({len(reqs2)} more updates on graphs 0 and 1): batched {two_b:.1f} updates/s, "
            f"plain {two_p:.1f} updates/s, batched/plain {two_b / two_p:.3f}, same state {two_same}")
        for tw in twins2:
            tw.free()
        del twins2
        torch.cuda.empty_cache()

    # ---------------------------------------------------------------- recompute
    if "recompute" in legs:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        grs[0].recompute()
        ctx.sync()
        rec_s = time.perf_counter() - t0
        comparators["full_gpu_recompute_s"] = rec_s
        comparators["full_gpu_recompute_updates_per_s"] = 1.0 / rec_s
        comparators["batched_over_recompute"] = value * rec_s
        log(f"full GPU recompute: {rec_s:.3f}s -> {1 / rec_s:.3f} updates/s")
        # the same static pass with the distance search over the maintained E*
        # only (Section 6); the state it reaches is the same
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        grs[0].recompute_estar()
        ctx.sync()
        est_s = time.perf_counter() - t0
        comparators["estar_gpu_recompute_s"] = est_s
        comparators["batched_over_estar_recompute"] = value * est_s
        log(f"GPU recompute over E*: {est_s:.3f}s")

    # ---------------------------------------------------------------- loader
    # Loading dense graphs: the complete n=2048 workload (weights up to n^2)
    # and the largest complete graph of the 64-graph batched workload, by the
    # static pass's checked search over a subset containing E* (Section 6)
    # and, in a second context, by the search over every arc.
    if "loader" in legs:
        dense = [("complete n=2048 (the vertex-update workload)", W.config3()[0])]
        c4n = W.config4_sizes()
        gi = max(range(32, 64), key=lambda i: c4n[i])  # graphs 32..63 are the complete ones
        big = W.complete_undirected(c4n[gi], c4n[gi] ** 2, W.derive_seed(4, gi, 0), f"c4-complete-n{c4n[gi]}")
        dense.append((f"complete n={big.n} (largest of the 64-graph workload)", big))
        loads = []
        full_ctx = bcinc.Context(device=0, n_max=max(g.n for _, g in dense), slots=0, full_search=True)
        for name, g in dense:
            row = {"graph": name, "n": g.n, "arcs": 2 * g.m}
            for label, c in (("checked", ctx), ("full", full_ctx)):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                gl = c.load_graph(g)
                c.sync()
                row[f"{label}_load_s"] = time.perf_counter() - t0
                st = gl.stats()
                row[f"{label}_searched_arcs"] = st["search_arcs"]
                row[f"{label}_search_rounds"] = st["search_rounds"]
                row[f"{label}_hash"] = gl.state_hash()
                gl.free()
                torch.cuda.empty_cache()
            row["same_state"] = row.pop("checked_hash") == row.pop("full_hash")
            loads.append(row)
            log(f"load {name}: checked search {row['checked_load_s']:.2f}s ({row['checked_searched_arcs']} arcs, "
                f"{row['checked_search_rounds']} rounds), full search {row['full_load_s']:.2f}s; same state "
                f"{row['same_state']}")
        full_ctx.close()
        torch.cuda.empty_cache()
        comparators["dense_loads"] = loads

    # ---------------------------------------------------------------- single
    # A dedicated stream of the same mix on one freshly loaded n-vertex graph:
    # the whole stream in one submit (one job per step, captured steps, tuned
    # schedule), and the same stream one update at a time on a device clone
    # taken before it (default schedule, synchronised).  Both must reach the
    # same D and sigma.
    if "single" in legs and args.single > 0:
        S = args.single
        sstream = W.mixed_stream(graphs[0], S, 1000, W.derive_seed(5, 6000 + gidx[0]), 0.35, 0.35, 16)
        fresh = ctx.load_graph(graphs[0])
        twin = fresh.clone()
        sbatch = ctx.batch([(fresh, up) for up in sstream])
        scalls = [twin.prepare(up) for up in sstream]
        ctx.sync()
        torch.cuda.synchronize()
        with quiet_gc():
            t0 = time.perf_counter()
            ctx.wait(ctx.submit(sbatch))
            ctx.sync()
            s_batched = time.perf_counter() - t0
        ctx.set_schedule(**default_sched)
        torch.cuda.synchronize()
        with quiet_gc():
            t0 = time.perf_counter()
            for call in scalls:
                call()
                ctx.sync()
            s_plain = time.perf_counter() - t0
        ctx.set_schedule(**tuned)
        same = fresh.state_hash() == twin.state_hash()
        comparators["single_graph_stream"] = {
            "updates": S, "batched_updates_per_s": S / s_batched, "plain_updates_per_s": S / s_plain,
            "batched_over_plain": s_plain / s_batched, "same_state": same}
        log(f"single-graph stream of {S} updates: batched {S / s_batched:.1f} updates/s, plain {S / s_plain:.1f} "
            f"updates/s, same state {same}")
        twin.free()
        fresh.free()
        torch.cuda.empty_cache()

    # ------------------------------------------------------- cpu incremental
    # The multi-core CPU comparator (Lemma 2 for an arc, the two-phase rule of
    # Section 4 for a vertex update, the partial dependency over the changed
    # pairs' ancestors) on the same graph: its state is read back from a
    # freshly loaded GPU copy, a short sample of the same mix is applied on
    # CPU threads, and the same updates on the GPU copy must give the same
    # rows (sampled) and BC.
    if "cpuinc" in legs and args.cpu_updates > 0:
        from paper_1311_2147_amd.cpu import CpuIncremental

        C = args.cpu_updates
        threads = min(16, os.cpu_count() or 1)
        cstream = W.mixed_stream(graphs[0], C, 1000, W.derive_seed(5, 7000 + gidx[0]), 0.35, 0.35, 16)
        base = ctx.load_graph(graphs[0])
        ctx.sync()
        t0 = time.perf_counter()
        cpu_inc = CpuIncremental(graphs[0], threads=threads)
        chunk = 1024
        for s0 in range(0, n, chunk):
            Dc, Sc = base.rows(s0, min(chunk, n - s0))
            cpu_inc.set_rows(s0, Dc, Sc)
        cpu_inc.set_scores(base.scores())
        del Dc, Sc
        fill_s = time.perf_counter() - t0
        t_edge = t_vertex = 0.0
        n_edge = n_vertex = 0
        for up in cstream:
            t0 = time.perf_counter()
            cpu_inc.update(up)
            dt = time.perf_counter() - t0
            if up.kind == "edge":
                t_edge += dt
                n_edge += 1
            else:
                t_vertex += dt
                n_vertex += 1
        ctx.set_schedule(**default_sched)
        for up in cstream:
            base.update(up)
        ctx.sync()
        ctx.set_schedule(**tuned)
        probe = np.linspace(0, n - 1, 64).astype(np.int64)
        same = True
        for s in probe:
            Dg, Sg = base.rows(int(s), 1)
            Dh, Sh = cpu_inc.rows(int(s), 1)
            same = same and np.array_equal(Dg, Dh) and np.array_equal(Sg, Sh)
        bg, bh = base.scores(), cpu_inc.scores()
        same = same and float(np.max(np.abs(bg - bh) / np.maximum(np.abs(bg), 1.0))) <= 1e-10
        cpu_inc.close()
        base.free()
        torch.cuda.empty_cache()
        rate = C / (t_edge + t_vertex)
        comparators["cpu_incremental"] = {
            "updates": C, "threads": threads, "updates_per_s": rate,
            "edge_updates_per_s": n_edge / t_edge if n_edge else None,
            "vertex_updates_per_s": n_vertex / t_vertex if n_vertex else None,
            "batched_over_cpu_incremental": value / rate, "same_state_sampled": bool(same),
            "state_fill_s": fill_s,
            "note": "C/OpenMP over the sources, the same update rules (Lemma 2, Section 4) on the host"}
        log(f"cpu incremental comparator: {C} updates ({n_edge} edge, {n_vertex} vertex) on {threads} threads -> "
            f"{rate:.2f} updates/s (edge {n_edge / max(t_edge, 1e-9):.2f}/s, vertex {n_vertex / max(t_vertex, 1e-9):.2f}/s); "
            f"same sampled state as the GPU: {same}; state read back in {fill_s:.1f}s")

    # the headline graphs are done with; the oracle leg needs only their arcs
    cur0 = graphs[0]
    for up in streams[0][:cursor[0]]:
        cur0 = W.apply_update(cur0, up)
    for gr in grs:
        gr.free()
    del grs
    torch.cuda.empty_cache()

    # ---------------------------------------------------------------- served
    # The served workload at full shape: 8 resident Chung-Lu graphs and one
    # seeded stream over them, cut into consecutive parts (each part is valid
    # on the graphs as the parts before it left them): a closed loop (every
    # request there at the start) for the saturation rate, then Poisson
    # arrivals at 0.5, 0.8 and 0.95 of it.
    served = None
    if "served" in legs:
        c5 = [W.config5_graph(W.C5_SIZES[i % 4], i) for i in range(8)]
        n_sat, n_lo, n_hi = 2000, 3000, 3000
        total = n_sat + n_lo + args.served_updates + n_hi + 1000
        t = time.perf_counter()
        c5_stream = W.config5_stream(c5, total)
        log(f"served workload: 8 graphs {[g.n for g in c5]}, {total} updates drawn in {time.perf_counter() - t:.1f}s")
        t = time.perf_counter()
        sg = [ctx.load_graph(g) for g in c5]
        ctx.sync()
        c5_load_s = time.perf_counter() - t
        log(f"served workload loaded in {c5_load_s:.1f}s")
        pos = 0

        def part(cnt):
            nonlocal pos
            out = c5_stream[pos:pos + cnt]
            pos += cnt
            return out

        def run(reqs, rate, seed):
            arrivals = np.zeros(len(reqs)) if rate is None else W.poisson_arrivals(len(reqs), rate, seed)
            srv = serve.Server(ctx, sg, max_in_flight=2)
            with quiet_gc():
                lat, _, wall_s = srv.run(arrivals, reqs)
            ctx.sync()
            res = {"updates": len(reqs), "served_updates_per_s": len(reqs) / wall_s,
                   "mean_requests_per_step": srv.stepped_requests / max(srv.steps, 1), **serve.percentiles(lat)}
            by_n = {}
            for nn in W.C5_SIZES:
                sel = [k for k, (gi, _) in enumerate(reqs) if c5[gi].n == nn]
                if sel:
                    pp = serve.percentiles(lat[sel])
                    by_n[str(nn)] = {"updates": len(sel), "p50": pp["p50"], "p99": pp["p99"]}
            res["by_n"] = by_n
            return res

        # the plain path on the closed loop's requests: device clones of the 8
        # graphs taken before it get the same requests one at a time (in the
        # order they were queued, which keeps each graph's order), default
        # schedule, bc_update_* and bc_sync after each; both must end in the
        # same state
        c5_twins = [gr.clone() for gr in sg]
        ctx.sync()
        sat_reqs = part(n_sat)
        sat = run(sat_reqs, None, 0)
        sat_rate = sat["served_updates_per_s"]
        log(f"served closed loop: {sat_rate:.1f} updates/s, {sat['mean_requests_per_step']:.2f} requests per step")
        c5_calls = [c5_twins[gi].prepare(up) for gi, up in sat_reqs]
        ctx.set_schedule(**default_sched)
        torch.cuda.synchronize()
        with quiet_gc():
            t0 = time.perf_counter()
            for call in c5_calls:
                call()
                ctx.sync()
            c5_plain_s = time.perf_counter() - t0
        ctx.set_schedule(**tuned)
        c5_same = all(c5_twins[i].state_hash() == sg[i].state_hash() for i in range(len(sg)))
        sat["plain_updates_per_s"] = len(sat_reqs) / c5_plain_s
        sat["served_over_plain"] = sat_rate / sat["plain_updates_per_s"]
        sat["plain_same_state"] = c5_same
        log(f"plain path on the closed loop's {len(sat_reqs)} requests (clones): {sat['plain_updates_per_s']:.1f} "
            f"updates/s; served/plain {sat['served_over_plain']:.2f}, same state {c5_same}")
        for tw in c5_twins:
            tw.free()
        del c5_twins
        torch.cuda.empty_cache()
        sweep = []
        for frac, cnt, seed in ((0.5, n_lo, 5101), (0.8, args.served_updates, 5102), (0.95, n_hi, 5103)):
            res = run(part(cnt), frac * sat_rate, W.derive_seed(5, seed))
            res["offered_fraction"] = frac
            res["offered_updates_per_s"] = frac * sat_rate
            sweep.append(res)
            log(f"served at {frac:.2f} x saturation ({frac * sat_rate:.0f}/s, {cnt} updates): "
                f"{res['served_updates_per_s']:.0f}/s served, p50 {res['p50']:.2f} ms, p99 {res['p99']:.2f} ms; "
                + ", ".join(f"n={k} p50 {v['p50']:.2f} p99 {v['p99']:.2f}" for k, v in res["by_n"].items()))
        served = {"graphs": [g.n for g in c5], "load_s": c5_load_s, "saturation": sat, "sweep": sweep}
        comparators["served_over_plain"] = sat["served_over_plain"]

        # admission under a memory budget: the 8 graphs' arenas less half an
        # n=4096 arena, so one graph stays off the device at any time;
        # requests for it wait until an idle graph of its size is evicted
        # (its arcs kept on the host) and it is loaded again by the static
        # pass
        if "budget" in legs:
            nbytes = [gr.nbytes + 256 for gr in sg]
            budget = sum(nbytes) - nbytes[0] // 2
            # the resident graphs stay but for graph 0 (n=4096): the two
            # n=4096 graphs share one place, and a request for the one that
            # is out waits until the other is idle, is evicted and it is
            # loaded again
            res_mgr = serve.Resident(ctx, [None] * len(sg), budget, lambda i: nbytes[i])
            for i, gr in enumerate(sg):
                res_mgr.live[i] = gr
            evicted = res_mgr.live.pop(0)
            res_mgr.arcs[0] = evicted.arcs()
            evicted.free()
            del sg
            torch.cuda.empty_cache()
            # its own saturation first (closed loop), then half of it offered
            creqs = part(300)
            srv = serve.Server(ctx, resident=res_mgr, max_in_flight=2)
            lat, _, wall_s = srv.run(np.zeros(len(creqs)), creqs)
            bsat = len(creqs) / wall_s
            ev0, ld0, lds0 = res_mgr.evictions, res_mgr.loads, res_mgr.load_s
            breqs = part(400)
            rate = 0.5 * bsat
            arrivals = W.poisson_arrivals(len(breqs), rate, W.derive_seed(5, 5104))
            srv = serve.Server(ctx, resident=res_mgr, max_in_flight=2)
            lat, _, wall_s = srv.run(arrivals, breqs)
            ctx.sync()
            pp = serve.percentiles(lat)
            served["budget"] = {
                "budget_bytes": budget, "budget_in_16n2_units": budget / sum(16 * g.n * g.n for g in c5),
                "all_graphs_bytes": sum(nbytes), "saturation_updates_per_s": bsat, "updates": len(breqs),
                "offered_updates_per_s": rate, "served_updates_per_s": len(breqs) / wall_s,
                "loads": res_mgr.loads - ld0, "evictions": res_mgr.evictions - ev0, "load_s": res_mgr.load_s - lds0,
                **pp}
            b = served["budget"]
            log(f"served under a {budget / 1e9:.2f} GB budget (all graphs {sum(nbytes) / 1e9:.2f} GB): saturation "
                f"{bsat:.0f}/s; at {rate:.0f}/s offered: {b['evictions']} evictions, {b['loads']} loads "
                f"({b['load_s']:.1f}s), {b['served_updates_per_s']:.0f}/s served, p50 {pp['p50']:.2f} ms "
                f"p99 {pp['p99']:.2f} ms")
            for i in list(res_mgr.live):
                res_mgr.live.pop(i).free()
        else:
            for gr in sg:
                gr.free()
        torch.cuda.empty_cache()

    # ---------------------------------------------------------------- many graphs
    # The 64-graph batched workload (n log-uniform in [256, 4096], half
    # directed with out-degree 8, half complete with weights up to n^2, 32
    # updates each): every step's 64 updates in one batched launch sequence
    # under the autotuner's choice per size bucket (tuned on a separately
    # drawn sample of eight graphs, on clones), then the same updates one at a
    # time on clones of the graphs (default schedule, bc_sync after each);
    # both must end in the same states.
    if "c4" in legs:
        t = time.perf_counter()
        work = W.config4()
        c4g = [ctx.load_graph(g) for g, _ in work]
        ctx.sync()
        c4_load_s = time.perf_counter() - t
        sample = []
        for i in range(0, len(work), 8):
            g = work[i][0]
            if g.directed:
                ups4 = W.mixed_stream(g, 4, 100, W.derive_seed(4, 9000 + i), 0.35, 0.35, 16)
            else:
                ups4 = W.mixed_stream(g, 4, g.n * g.n, W.derive_seed(4, 9000 + i), 0.0, 0.70, 16)
            sample += [(c4g[i], up) for up in ups4]
        t = time.perf_counter()
        c4_pick = ctx.autotune(sample)
        c4_tune_s = time.perf_counter() - t
        c4_twins = [gr.clone() for gr in c4g]
        ctx.sync()
        n_steps = len(work[0][1])
        reqs4 = [(c4g[i], ups4[k]) for k in range(n_steps) for i, (_, ups4) in enumerate(work)]
        batch4 = ctx.batch(reqs4)
        calls4 = [c4_twins[i].prepare(ups4[k]) for k in range(n_steps) for i, (_, ups4) in enumerate(work)]
        torch.cuda.synchronize()
        ctx.reset_timing()
        with quiet_gc():
            t0 = time.perf_counter()
            ctx.wait(ctx.submit(batch4))
            torch.cuda.synchronize()
            c4_b = len(reqs4) / (time.perf_counter() - t0)
        c4_dev = ctx.timing()
        ctx.set_schedule(**default_sched)
        torch.cuda.synchronize()
        with quiet_gc():
            t0 = time.perf_counter()
            for call in calls4:
                call()
                ctx.sync()
            c4_p = len(reqs4) / (time.perf_counter() - t0)
        ctx.set_schedule(**tuned)
        c4_same = all(c4_twins[i].state_hash() == c4g[i].state_hash() for i in range(len(work)))
        comparators["many_graphs"] = {
            "workload": "64 graphs, n log-uniform in [256, 4096], half directed out-degree 8 (weights 1..100), "
                        "half complete undirected (weights 1..n^2), 32 updates each, one update per graph per step",
            "updates": len(reqs4), "load_s": c4_load_s, "autotune_s": c4_tune_s,
            "batched_updates_per_s": c4_b, "plain_updates_per_s": c4_p, "batched_over_plain": c4_b / c4_p,
            "same_state": c4_same, "schedule": c4_pick, "steps": c4_dev["steps"],
            "device_ms_per_step": c4_dev["step_ms"] / max(c4_dev["steps"], 1)}
        log(f"64-graph batched workload ({len(reqs4)} updates, loaded in {c4_load_s:.1f}s, tuned in {c4_tune_s:.1f}s): "
            f"batched {c4_b:.0f} updates/s, plain {c4_p:.0f} updates/s, batched/plain {c4_b / c4_p:.2f}, "
            f"same state {c4_same}; {c4_dev['steps']} steps, {c4_dev['step_ms'] / max(c4_dev['steps'], 1):.3f} ms "
            f"per step on the device; schedule {c4_pick}")
        for gr in c4_twins + c4g:
            gr.free()
        del c4_twins, c4g
        torch.cuda.empty_cache()

    # ------------------------------------------------------------ C2 and C3
    # The out-degree-8 stream at n = 4096 (256 arc updates) and the complete
    # graph at n = 2048 (64 vertex updates of 32 edges each): one graph each,
    # so its stream runs one update per step (bc_submit of the whole stream,
    # under the autotuner's schedule for the graph's size bucket, tuned on a
    # separately drawn sample unless a bucket has one) and, on a device clone,
    # one update at a time (default schedule, synchronised after each); both
    # must end in the same state.  The CPU leg times the oracle on the final
    # graphs.
    small_finals = []
    if "c2c3" in legs:
        small = {}
        for name, (g, ups) in (("out-degree-8 n=4096, 256 arc updates", W.config2()),
                               ("complete n=2048, 64 vertex updates of 32 edges", W.config3())):
            gr = ctx.load_graph(g)
            if g.directed:
                tsample = W.edge_stream(g, 4, 4, 100, W.derive_seed(2, 9000))
            else:
                tsample = W.vertex_stream(g, 4, 32, g.n * g.n, W.derive_seed(3, 9000))
            ctx.autotune([(gr, up) for up in tsample])
            tw = gr.clone()
            sb = ctx.batch([(gr, up) for up in ups])
            calls = [tw.prepare(up) for up in ups]
            ctx.sync()
            torch.cuda.synchronize()
            with quiet_gc():
                t0 = time.perf_counter()
                ctx.wait(ctx.submit(sb))
                torch.cuda.synchronize()
                b_rate = len(ups) / (time.perf_counter() - t0)
            b_sched = ctx.schedule()
            ctx.set_schedule(**default_sched)
            torch.cuda.synchronize()
            with quiet_gc():
                t0 = time.perf_counter()
                for call in calls:
                    call()
                    ctx.sync()
                p_rate = len(ups) / (time.perf_counter() - t0)
            ctx.set_schedule(**tuned)
            st = gr.stats()
            same = gr.state_hash() == tw.state_hash()
            cur = g
            for up in ups:
                cur = W.apply_update(cur, up)
            small_finals.append((name, cur))
            small[name] = {"updates": len(ups), "batched_updates_per_s": b_rate, "plain_updates_per_s": p_rate,
                           "schedule": b_sched, "same_state": same, "affected_per_update": st["total_affected"] / len(ups),
                           "changed_pairs_per_update": st["total_changed"] / len(ups)}
            log(f"{name}: batched {b_rate:.0f} updates/s, plain {p_rate:.0f} updates/s, same state {same}, "
                f"|A| {st['total_affected'] / len(ups):.0f}, schedule {b_sched}")
            tw.free()
            gr.free()
            torch.cuda.empty_cache()
        comparators["small_configs"] = small

    # ------------------------------------------------------------------ copy
    # A plain device-to-device copy of 1 GiB: the achievable HBM bandwidth on
    # this box (read + write bytes over time), and the calibration kernel of
    # the HBM counter runs.
    copy_gbs = None
    if "copy" in legs:
        nb = 1 << 30
        a = torch.empty(nb, dtype=torch.uint8, device="cuda:0")
        b = torch.empty_like(a)
        a.fill_(1)
        b.copy_(a)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        copy_gbs = 2 * nb * 5 / (e0.elapsed_time(e1) / 1e3) / 1e9
        del a, b
        torch.cuda.empty_cache()
        log(f"device copy of 1 GiB: {copy_gbs:.0f} GB/s (read + write)")

    # ---------------------------------------------------------------- cpu oracle
    # One complete from-scratch recompute of BC (every source, no rows kept)
    # of the n = 32768 graph as the updates left it, on all host cores; and
    # the same Brandes pass for a sample of sources on one core, scaled to all
    # n sources.
    cpu = None
    if "cpu" in legs:
        import oracle

        threads = oracle.default_threads()
        t0 = time.perf_counter()
        oracle.brandes(cur0, rows=False, threads=threads)
        full_s = time.perf_counter() - t0
        S1 = min(args.cpu_one_core_sources, n)
        srcs = np.linspace(0, n - 1, S1).astype(np.int32)
        t0 = time.perf_counter()
        oracle.rows(cur0, srcs, threads=1)
        one_s = time.perf_counter() - t0
        one_full = one_s * n / S1
        cpu = {"value": 1.0 / full_s, "unit": "updates/s", "cores": threads, "kind": "oracle",
               "sample": f"one complete from-scratch Brandes BC recompute (Dijkstra from all {n} sources + "
                         f"dependency accumulation) of the updated n={n} graph in {full_s:.1f}s on {threads} threads "
                         f"({cpu_model()})",
               "one_core": {"value": 1.0 / one_full, "unit": "updates/s", "cores": 1,
                            "sample": f"{S1} of {n} sources in {one_s:.2f}s on one thread, scaled by n/{S1} to "
                                      f"{one_full:.0f}s per recompute (extrapolated)"}}
        log(f"cpu oracle: complete recompute {full_s:.1f}s on {threads} threads -> {1 / full_s:.4f} updates/s; "
            f"one core {S1} sources in {one_s:.2f}s -> {one_full:.0f}s per recompute (extrapolated)")
        # the oracle's time per update on the two single-graph workloads: a
        # from-scratch BC recompute of the final graph on all host cores (every
        # source for n = 4096; for the complete graph, whose Dijkstra relaxes
        # n^2 arcs per source, a 128-source sample scaled to n)
        per_cfg = {}
        for name, cur in small_finals:
            if cur.m <= 64 * cur.n:
                t0 = time.perf_counter()
                oracle.brandes(cur, rows=False, threads=threads)
                o_s = time.perf_counter() - t0
                note = f"complete recompute of all {cur.n} sources"
            else:
                S2 = 128
                t0 = time.perf_counter()
                oracle.rows(cur, np.linspace(0, cur.n - 1, S2).astype(np.int32), threads=threads)
                o_s = (time.perf_counter() - t0) * cur.n / S2
                note = f"{S2} of {cur.n} sources scaled by n/{S2} (extrapolated)"
            per_cfg[name] = {"s_per_update": o_s, "updates_per_s": 1.0 / o_s, "cores": threads, "sample": note}
            log(f"cpu oracle, {name}: {o_s:.2f}s per update on {threads} threads ({note})")
        if per_cfg:
            cpu["small_configs"] = per_cfg

    line = {
        "metric": "BC updates/sec at n=32768 (batched incremental path)",
        "value": value,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": wall / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32 distances, uint64 path counts, f64 BC",
        "data": "synthetic (seeded Chung-Lu graphs and update streams)",
        "config": {
            "workload": f"{G} resident directed Chung-Lu graphs, n={n}, mean degree 16, exponent 2.5, "
                        f"weights 1..1000; per graph 35% insertions, 35% decreases, 30% vertex updates "
                        f"of 16 arcs; one update per graph per step",
            "n": n, "graphs": G, "updates_per_step": G, "parallelism": "1 GPU",
            "load_s_per_graph": load_s,
            "schedule": tuned, "plain_schedule": default_sched, "autotune_s": tune_s,
        },
        "comparators": comparators,
        "latency_ms": served["sweep"][1] if served else None,
        "served": served,
        "roofline": {
            "kernel": "k_rows (row update: distance filter and Lemma 4 pair update over the affected rows)",
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": committed_traffic(G, n),
            "copy_gbs": copy_gbs,
            "window": "the timed batched steps",
            "avg_launch_ms": rows_ms / launches,
            "launches": launches,
            "bytes_per_launch": alg_bytes / launches,
            "per_source_kernels_avg_ms": window_timing["source_ms"] / launches,
            "step_avg_ms": window_timing["step_ms"] / launches,
        },
        "cpu_baseline": cpu,
        "system": system_info(),
    }
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
