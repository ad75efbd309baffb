#!/usr/bin/env python3
"""Benchmark: incremental betweenness-centrality updates per second at n = 32768.

Workload (synthetic, seeded): two resident directed Chung-Lu graphs with
n = 32768, degree exponent 2.5, mean out-degree 16 (m = 16n arcs), integer
weights uniform in {1..1000}; each graph gets its own stream of updates drawn
35% insertions, 35% decreases to a uniform lower weight, 30% vertex updates
touching 16 incident arcs.  Inputs are resident in HBM before timing starts.

A step is one pass of the whole update path over one batch: one update on
each resident graph, processed together by one batched launch sequence (scan,
row v'', E* merge, per-source kernel, E* filter, commit) replayed from a
captured HIP graph.  value = updates completed per second over the timed steps.

Besides the headline the run measures, on the same graphs and stream:
  * the plain path: the same kernels, one update at a time, synchronised
    after each, launched directly (no HIP graph, no batching);
  * a full GPU recompute (static Brandes on the GPU, the loader);
  * p50/p99 latency of a served Poisson stream at 0.8x the batched rate;
  * a dedicated 1000-update stream on one freshly loaded graph;
  * the multi-core CPU incremental comparator (the same update rules on CPU
    threads) on a short sample, its state checked against the GPU's;
  * the CPU oracle (from-scratch Brandes) on a bounded sample of sources.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_rows_chunglu_n32768_traffic.md")
KERNEL_SOURCES = ("paper_1311_2147_amd/csrc/bc_kernels.hip", "paper_1311_2147_amd/csrc/bc_device.h")


def kernel_sources_sha256():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def committed_traffic():
    """HBM bytes per row-kernel launch from the committed counter summary,
    or None when there is none or the kernel sources changed since."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    text = open(TRAFFIC_FILE).read()
    sha = re.search(r"kernel_sources_sha256:\s*([0-9a-f]{64})", text)
    val = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not sha or not val or sha.group(1) != kernel_sources_sha256():
        return None
    return float(val.group(1))


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--n", type=int, default=32768)
    ap.add_argument("--graphs", type=int, default=2)
    ap.add_argument("--plain", type=int, default=None, help="updates on the plain path (default steps*graphs)")
    ap.add_argument("--latency-requests", type=int, default=160)
    ap.add_argument("--cpu-sources", type=int, default=4096)
    ap.add_argument("--legs", default="batched,plain,recompute,latency,single,cpuinc,cpu,copy")
    ap.add_argument("--cpu-updates", type=int, default=12, help="updates of the CPU incremental comparator's sample")
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
    P = args.plain if args.plain is not None else K * G
    R = args.latency_requests

    # ---------------------------------------------------------------- inputs
    t = time.perf_counter()
    sizes = list(W.C5_SIZES)
    gidx = [i for i in range(8) if sizes[i % 4] == n][:G] if n in sizes else list(range(G))
    graphs = [W.config5_graph(n, gi) for gi in gidx]
    per_graph = Wm + K + (P + G - 1) // G + (R + G - 1) // G + 8
    streams = [W.mixed_stream(g, per_graph, 1000, W.derive_seed(5, 2000 + gi), 0.35, 0.35, 16)
               for g, gi in zip(graphs, gidx)]
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
    before = [gr.stats() for gr in grs]
    reqs = []
    for _ in range(K):
        for i in range(G):
            reqs.append((grs[i], take(i)))
    stream = ctx.stream
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    ticket = ctx.submit(reqs)
    ev1.record(stream)
    ctx.wait(ticket)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    after = [gr.stats() for gr in grs]
    ctx.sync()
    value = K * G / wall
    log(f"batched: {K} steps x {G} graphs in {wall * 1e3:.1f} ms wall ({gpu_ms:.1f} ms stream) -> {value:.1f} updates/s")

    log(f"batched window: |A| per update "
        f"{sum(after[i]['total_affected'] - before[i]['total_affected'] for i in range(G)) / (K * G):.0f}, changed "
        f"pairs per update {sum(after[i]['total_changed'] - before[i]['total_changed'] for i in range(G)) / (K * G):.0f}")

    comparators = {}
    # ---------------------------------------------------------------- plain
    if "plain" in legs and P > 0:
        ctx.set_schedule(**default_sched)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(P):
            i = k % G
            grs[i].update(take(i))
            ctx.sync()
        plain_s = time.perf_counter() - t0
        ctx.set_schedule(**tuned)
        comparators["plain_updates_per_s"] = P / plain_s
        comparators["batched_over_plain"] = value / (P / plain_s)
        log(f"plain: {P} updates one at a time -> {P / plain_s:.1f} updates/s")

    # ---------------------------------------------------------------- latency
    latency = None
    if "latency" in legs and R > 0:
        rate = 0.8 * value
        arrivals = W.poisson_arrivals(R, rate, W.derive_seed(5, 3000))
        pick = W.Rng(W.derive_seed(5, 3001)).integers(0, G - 1, R)
        requests = []
        for gi in pick:
            gi = int(gi)
            if cursor[gi] >= len(streams[gi]):
                gi = int(np.argmin(cursor))
            requests.append((gi, take(gi)))
        srv = serve.Server(ctx, grs, max_in_flight=2)
        lat, _, lwall = srv.run(arrivals, requests)
        latency = serve.percentiles(lat)
        latency["offered_updates_per_s"] = rate
        latency["served_updates_per_s"] = R / lwall
        log(f"served {R} Poisson requests at {rate:.1f}/s: p50 {latency['p50']:.2f} ms, p99 {latency['p99']:.2f} ms")
    ctx.sync()

    # ------------------------------------------------------------ row kernel
    # HIP events on the library's stream bracket every launch of the row
    # kernel in this run (warmup, batched, plain and served updates: one launch
    # per step); its algorithmic bytes (the device counts them per update:
    # 4n per affected row scanned, or 4 per candidate target when the
    # candidates are scanned instead, plus 8 per changed pair) are summed over
    # the same updates.
    timing = ctx.timing()
    alg_bytes = sum(gr.stats()["total_scan_bytes"] for gr in grs)
    rows_ms = timing["rows_ms"]
    launches = max(timing["steps"], 1)
    achieved = alg_bytes / (rows_ms / 1e3) / 1e9 if rows_ms > 0 else 0.0
    log(f"row kernel over the run: {launches} launches, avg {rows_ms / launches:.3f} ms, "
        f"{alg_bytes / launches / 1e6:.1f} MB/launch -> {achieved:.1f} GB/s "
        f"({100 * achieved / HBM_PEAK_GBS:.2f}% of HBM peak); all per-source kernels avg "
        f"{timing['source_ms'] / launches:.3f} ms, step avg {timing['step_ms'] / launches:.3f} ms")

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
        ctx.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.wait(ctx.submit([(fresh, up) for up in sstream]))
        ctx.sync()
        s_batched = time.perf_counter() - t0
        ctx.set_schedule(**default_sched)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for up in sstream:
            twin.update(up)
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
    # pairs' ancestors) on the
    # same graph: its state is read back from a freshly loaded GPU copy, a
    # short sample of the same mix is applied on CPU threads, and the same
    # updates on the GPU copy must give the same rows (sampled) and BC.
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
    cpu = None
    if "cpu" in legs and args.cpu_sources > 0:
        import oracle

        cur = graphs[0]
        for up in streams[0][:cursor[0]]:
            cur = W.apply_update(cur, up)
        S = min(args.cpu_sources, n)
        srcs = np.linspace(0, n - 1, S).astype(np.int32)
        threads = oracle.default_threads()
        t0 = time.perf_counter()
        oracle.rows(cur, srcs, threads=threads)
        cs = time.perf_counter() - t0
        full_s = cs * n / S
        cpu = {"value": 1.0 / full_s, "unit": "updates/s", "cores": threads, "kind": "oracle",
               "sample": f"from-scratch Brandes (Dijkstra + dependency accumulation) for {S} of {n} sources "
                         f"of the updated graph in {cs:.2f}s on {threads} threads, scaled by n/{S} to one "
                         f"full recompute ({full_s:.1f}s) per update"}
        log(f"cpu oracle: {S} sources in {cs:.2f}s on {threads} threads -> {1 / full_s:.4f} updates/s (extrapolated)")

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
        "latency_ms": latency,
        "roofline": {
            "kernel": "k_rows (row update: distance filter and Lemma 4 pair update over the affected rows)",
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": committed_traffic(),
            "copy_gbs": copy_gbs,
            "avg_launch_ms": rows_ms / launches,
            "launches": launches,
            "bytes_per_launch": alg_bytes / launches,
            "per_source_kernels_avg_ms": timing["source_ms"] / launches,
            "step_avg_ms": timing["step_ms"] / launches,
        },
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
