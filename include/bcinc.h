/*
 * bcinc -- incremental betweenness centrality on AMD Instinct MI355X (gfx950).
 *
 * C ABI of libbcinc.so.  Every call takes plain host or device pointers and
 * sizes; no framework types cross this boundary.  The method is the
 * incremental update of Nasre, Pontecorvi and Ramachandran, "Betweenness
 * Centrality -- Incremental and Faster" (arXiv:1311.2147):
 *
 *   - an incremental edge update lowers the weight of an existing arc or
 *     inserts a missing one (Section 1, problem statement);
 *   - a vertex update does that on any subset of the arcs into and out of
 *     one vertex v (Section 4);
 *   - after each update the library holds, for every pair (s,t), the distance
 *     d(s,t) and the shortest-path count sigma_st (Lemma 2 for edges, Lemma 4
 *     for vertex updates, In then Out on the reverse graph), the SSSP DAG of
 *     every source implicitly as the predicate of Eq.1 over E* (the arcs on
 *     some shortest path, Section 1), and BC(v) of Eq.3 updated by the
 *     difference of the Brandes dependencies (Eq.4, Alg 1) of every affected
 *     source (Alg 3).
 *
 * Conventions shared by every call:
 *   - Vertices are 0..n-1.  Weights are positive integers below 2^31-1.
 *   - Directed graphs take arcs (a,b).  Undirected graphs take each edge once
 *     and are handled as their directed double G_D (Section 3, undirected
 *     graphs), so BC counts ordered pairs (twice the unordered convention).
 *   - Unreachable pairs have distance INT64_MAX and sigma 0 at this boundary;
 *     they contribute nothing to BC.
 *   - Device state per graph is D (int32, n x n, row-major), sigma (uint64,
 *     n x n) and the stored DAG predecessor of every pair (int32, n x n; see
 *     bc_get_preds): 16 bytes per pair.  A finite distance that would reach 2^31-1
 *     raises BC_ERR_DIST_OVERFLOW; a path count above 2^64-1 raises
 *     BC_ERR_SIGMA_OVERFLOW.  Both are sticky: the graph answers with that
 *     error until bc_recompute or bc_free_graph.
 *   - Calls on one context come from one host thread.  Work is ordered on the
 *     context's stream; device-side errors surface at the next synchronising
 *     call (bc_sync, bc_scores, bc_get_*, bc_wait).
 *   - A call that fails validation leaves every state unchanged.
 */
#ifndef BCINC_H
#define BCINC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t bc_status;

enum {
    BC_OK = 0,
    BC_ERR_INVALID_ARG = -1,     /* null pointer, n <= 0, id out of range, ... */
    BC_ERR_SELF_LOOP = -2,       /* arc (a,a) */
    BC_ERR_BAD_WEIGHT = -3,      /* w <= 0 or w >= 2^31-1 */
    BC_ERR_DUPLICATE_EDGE = -4,  /* repeated arc at load or inside one vertex update */
    BC_ERR_NOT_INCIDENT = -5,    /* vertex-update edge not touching v */
    BC_ERR_NOT_INCREMENTAL = -6, /* new weight >= current weight (Lemma 2 needs a strict decrease) */
    BC_ERR_ADMISSION = -7,       /* state would exceed the context's memory budget */
    BC_ERR_CAPACITY = -8,        /* arena, arc or E* capacity exceeded */
    BC_ERR_SIGMA_OVERFLOW = -9,  /* sticky: a path count passed 2^64-1 */
    BC_ERR_DIST_OVERFLOW = -10,  /* sticky: a finite distance reached 2^31-1 */
    BC_ERR_HIP = -11,            /* HIP runtime error; text in bc_last_error */
    BC_ERR_NO_DEVICE = -12,      /* no usable gfx950 device */
    BC_ERR_ESTAR_CAPACITY = -13, /* sticky: E* outgrew its capacity */
    BC_ERR_CHECK_FAILED = -14    /* sticky: a state check found the state wrong (BC_FLAG_CHECK, bc_check) */
};

typedef struct bc_ctx bc_ctx;
typedef int32_t bc_graph_id;

/* bc_config.flags */
#define BC_FLAG_TIMING 1      /* time every update step and its per-source kernels with HIP events */
#define BC_FLAG_FULL_SEARCH 2 /* the static pass (load, bc_recompute) relaxes every arc, never a
                                 checked subset (see bc_load_graph) */
#define BC_FLAG_CHECK 4       /* debugging: check the state after every load, recompute and update
                                 step (see bc_check); slow, and every such call synchronises */

typedef struct {
    int32_t device;         /* HIP device ordinal */
    int32_t flags;          /* BC_FLAG_* bits */
    void *stream;           /* hipStream_t to order all work on; NULL: the library makes one */
    void *scratch;          /* device buffer for per-workgroup work areas (caller owns it) */
    uint64_t scratch_bytes; /* its size; see bc_scratch_bytes */
    uint64_t memory_budget; /* admission limit for the sum of graph arenas, 0 = none */
    int32_t slots;          /* workgroup slots of the DAG kernel and the static pass, 0 = 2560 */
    int32_t block;          /* threads per workgroup of the DAG kernel (64, 128, 192 or 256), 0 = 256 */
    const char *tune_cache; /* path of the autotuner's cache file (see bc_autotune), or NULL */
} bc_config;

typedef struct {
    int32_t a, b; /* arc (a,b); for a vertex update one of them is v */
    int64_t w;    /* new weight */
} bc_edge;

/* Sizes (bytes) the caller allocates in device memory. */
uint64_t bc_graph_bytes(int32_t n, int64_t arc_capacity, int64_t estar_capacity);
uint64_t bc_scratch_bytes(int32_t n_max, int32_t slots);

/* Creates a context on cfg->device.  The scratch buffer must stay alive and
 * unused by the caller until bc_destroy.  Returns BC_ERR_NO_DEVICE when the
 * device is missing or is not gfx950. */
bc_status bc_create(bc_ctx **out, const bc_config *cfg);
bc_status bc_destroy(bc_ctx *ctx);

/* Loads a graph and computes its initial state with a static Brandes pass on
 * the GPU (the paper assumes BC and every DAG are available before the first
 * update: Section 1, and Alg 7 of the appendix).  The distance search of a
 * dense graph (at least 4k out-arcs per vertex on average, k = ceil(2 ln n)
 * + 4) relaxes a checked subset instead of every arc (Static-BC of Section
 * 6, which needs only an arc set containing E*): the k lightest out-arcs of
 * every vertex, plus, round by round, every arc whose weight is at most the
 * distance between its ends that the subset gives, until no such arc is
 * missing.  On complete graphs with random weights E* has about n ln n arcs,
 * so the search relaxes a small fraction of the n^2 arcs.  bc_recompute does
 * the same; BC_FLAG_FULL_SEARCH turns the check off.
 *   src, dst, w: host arrays of m arcs (edges when undirected), copied in;
 *     the caller keeps ownership.
 *   arc_capacity: most arcs (of G_D) the graph may ever hold, >= its arc count.
 *   estar_capacity: most arcs E* may hold (0 = arc_capacity).
 *   arena: caller-allocated device memory of bc_graph_bytes(...) bytes or
 *     more, 256-byte aligned, owned by the caller, untouched by it until
 *     bc_free_graph.
 * Validation: ids in range, no self-loops (BC_ERR_SELF_LOOP), no repeated
 * arcs (BC_ERR_DUPLICATE_EDGE), weights in [1, 2^31-2] (BC_ERR_BAD_WEIGHT),
 * arena size (BC_ERR_CAPACITY), budget (BC_ERR_ADMISSION).  Asynchronous
 * after validation. */
bc_status bc_load_graph(bc_ctx *ctx, int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                        const int64_t *w, int32_t directed, int64_t arc_capacity, int64_t estar_capacity,
                        void *arena, uint64_t arena_bytes, bc_graph_id *out);
bc_status bc_free_graph(bc_ctx *ctx, bc_graph_id g);

/* A second resident graph with the state of g at this point of the stream:
 * every update enqueued on g so far is included (device copy of g's arena,
 * ordered on the context's stream, plus a copy of the host arc mirror).  The
 * two then evolve independently.  Used to try updates or launch schedules on
 * a copy (the schedule autotuner replays sample updates on clones).
 *   arena: caller-allocated device memory of at least g's
 *     bc_graph_bytes(n, arc_capacity, estar_capacity), 256-byte aligned,
 *     owned by the caller, untouched by it until bc_free_graph of the clone.
 * Errors: BC_ERR_INVALID_ARG (no such graph, null or misaligned arena),
 * BC_ERR_CAPACITY (arena too small), BC_ERR_ADMISSION (over budget). */
bc_status bc_clone_graph(bc_ctx *ctx, bc_graph_id g, void *arena, uint64_t arena_bytes, bc_graph_id *out);

/* Incremental edge update (Section 3, Alg 3 with Lemma 2 and Alg 2): arc
 * (u,v) of a directed graph, or edge {u,v} of an undirected one (two arc
 * updates, Section 3 undirected paragraph), gets weight w.  w must be below
 * the current weight, or the arc must be new (BC_ERR_NOT_INCREMENTAL
 * otherwise).  Stream-ordered; returns after enqueueing. */
bc_status bc_update_edge(bc_ctx *ctx, bc_graph_id g, int32_t u, int32_t v, int64_t w);

/* Incremental vertex update (Section 4, steps (A)-(D), Alg 4 and Lemma 4):
 * k edges e[0..k) each with e[i].a == v or e[i].b == v.  Directed: (x,v) is
 * an in-arc (set E_i), (v,x) an out-arc (set E_o).  Undirected: {v,x} is both.
 * Each must lower the current weight or be new; no arc may repeat.  Sets with
 * more than 64 arcs per direction are applied as consecutive vertex updates
 * at v, which reach the same state. */
bc_status bc_update_vertex(bc_ctx *ctx, bc_graph_id g, int32_t v, int32_t k, const bc_edge *e);

/* Batched and served updates.  A request names a graph and either one edge
 * update or one vertex update.  bc_submit validates every request (none is
 * applied if one fails; *bad_index gets its index), then enqueues them as
 * steps: step k holds the k-th request of every graph, and all graphs of a
 * step are processed together by the same kernel launches (replayed from a
 * captured HIP graph).  Requests on one graph keep their order.  *ticket
 * identifies the submission for bc_poll/bc_wait. */
typedef struct {
    bc_graph_id graph;
    int32_t kind;          /* 0 = edge (u, v, w), 1 = vertex (v, k, edges) */
    int32_t u, v;
    int64_t w;
    int32_t k;
    const bc_edge *edges;  /* host pointer, k entries, read during the call only */
} bc_request;

bc_status bc_submit(bc_ctx *ctx, int32_t cnt, const bc_request *reqs, uint64_t *ticket, int32_t *bad_index);

/* Continuous batching.  bc_enqueue validates requests like bc_submit (none is
 * taken if one fails) and appends each to its graph's queue without
 * launching anything; tickets[i] identifies request i.  bc_step launches one
 * step: the head request of every graph with a non-empty queue, oldest head
 * first, at most max_jobs of them (0 = 256), all in one batched launch
 * sequence (the same kernels and captured graphs as bc_submit); *launched
 * gets the number of requests in it, 0 when every queue is empty.  If
 * step_ticket is not NULL it gets a ticket of the step itself (poll it to
 * learn when the step finishes).  A queued request changes no device state
 * until a step launches it; bc_wait on its ticket, bc_sync, and every call
 * that enqueues work directly or acts on a graph's state (bc_update_*,
 * bc_submit, bc_clone_graph, bc_free_graph, bc_recompute*, bc_autotune)
 * first launch every queued request, so the device applies requests in the
 * order they were validated.  Introspection calls and bc_scores see the
 * state of the steps launched so far. */
bc_status bc_enqueue(bc_ctx *ctx, int32_t cnt, const bc_request *reqs, uint64_t *tickets, int32_t *bad_index);
bc_status bc_step(bc_ctx *ctx, int32_t max_jobs, int32_t *launched, uint64_t *step_ticket);

/* Result of a ticket.  Times are nanoseconds of the host's CLOCK_MONOTONIC:
 * t_enqueue_ns is read on the host when the ticket was issued; t_start_ns and
 * t_finish_ns are device timestamps (HIP timing events recorded on the
 * context's stream before the first step that ran the ticket's requests and
 * after the last one) mapped to that clock through an event on an idle
 * stream of the library, to within tens of microseconds. */
typedef struct {
    int32_t done;          /* 1 once every step of the ticket has finished on the device */
    int32_t status;        /* when done: BC_OK, or the sticky error of one of its graphs */
    int64_t t_enqueue_ns;
    int64_t t_start_ns;    /* when done */
    int64_t t_finish_ns;   /* when done */
} bc_result;

/* bc_poll fills *out without waiting; out->status is the sticky error of
 * any of the ticket's graphs once it is done (sigma overflow first, then
 * distance overflow, then E* capacity), else BC_OK.  Once it reports done the
 * ticket is collected: polling it again reports done with status BC_OK and
 * zero times.  bc_wait launches the ticket's queued requests if any, waits
 * for its last step, collects it and returns that same status. */
bc_status bc_poll(bc_ctx *ctx, uint64_t ticket, bc_result *out);
bc_status bc_wait(bc_ctx *ctx, uint64_t ticket);

/* Launches every queued request, waits for all work of the context, and
 * returns the sticky error of any graph (sigma overflow first, then distance
 * overflow, then E* capacity), or BC_OK. */
bc_status bc_sync(bc_ctx *ctx);

/* BC(v) for all v (Eq.3 over ordered pairs) into host memory out[0..n).
 * Synchronises. */
bc_status bc_scores(bc_ctx *ctx, bc_graph_id g, double *out);

/* Full static recomputation on the GPU from the current arc set (the Brandes
 * baseline, Alg 7, and the recovery path after a sticky error). */
bc_status bc_recompute(bc_ctx *ctx, bc_graph_id g);

/* Static recomputation whose distance search relaxes only the maintained E*
 * (Section 6, Static-BC, with E* already known: every shortest path lies in
 * E*, so searching E* instead of E gives the same distances, and the DAGs,
 * path counts and dependencies over E* follow as in bc_recompute).  The
 * result equals bc_recompute's.  Synchronises.  A graph that carries a sticky
 * error (its E* may be incomplete) is left unchanged and its sticky status
 * returned: recover it with bc_recompute. */
bc_status bc_recompute_estar(bc_ctx *ctx, bc_graph_id g);

/* Introspection (tests).  All synchronise and write host memory.
 * bc_get_rows: rows s0..s0+cnt-1 of d (int64, INT64_MAX unreachable) and
 *   sigma (uint64); either pointer may be NULL.
 * bc_get_dag: arcs (a[i], b[i]) of DAG(s), the predicate of Eq.1 over E*;
 *   cap entries at most, *cnt gets the full count.
 * bc_get_estar: E* arcs (a, b, w); same capacity rule.
 * bc_get_delta: the dependency row delta_s.(.) of Eq.4 computed by the GPU's
 *   level-ordered accumulation (0 at s itself and at unreachable vertices).
 * bc_get_preds: the stored DAG(s) predecessor of every vertex x into out[0..n):
 *   the tail of x's only DAG(s) in-arc (Eq.1 over E*), -2 if x has two or
 *   more, -1 at x == s and at vertices unreachable from s.  The walks use it
 *   in place of Eq.1 tests where it names one tail.
 * bc_get_affected: the affected sources A of the graph's last update (the
 *   sources whose row the update changes: Lemma 2 case 1 fails for them at
 *   t = v, Section 3; for a vertex update the In and Out tests of Section 4),
 *   in no particular order, from the last job when a vertex update with more
 *   than 64 arcs per direction was split; cap entries at most (out may be
 *   NULL when cap is 0), *cnt gets |A|.  Empty right after a load.
 * bc_state_hash: 128-bit hash of D and sigma (order-fixed, bit-exact).
 * bc_get_stats: counters of the last update (see bc_update_stats). */
bc_status bc_get_rows(bc_ctx *ctx, bc_graph_id g, int32_t s0, int32_t cnt, int64_t *D, uint64_t *sigma);

/* Checkpoint: the graph's current arcs, as bc_load_graph takes them (arcs
 * (src[i] -> dst[i]) of a directed graph; one entry per edge, src < dst, of
 * an undirected one), with every update submitted so far applied (the host
 * keeps this list as it validates updates).  cap entries at most, *cnt gets
 * the full count; the pointers may be NULL to ask for the count.  Loading the
 * arcs again (bc_load_graph, the static pass of Section 6) re-derives D,
 * sigma, E*, the stored predecessors and BC: the restored graph's D and sigma
 * equal the live one's once its updates have run (bc_sync), and its BC agrees
 * within rounding.  Host-side only; needs no synchronisation. */
bc_status bc_get_arcs(bc_ctx *ctx, bc_graph_id g, int32_t *src, int32_t *dst, int64_t *w, int64_t cap,
                      int64_t *cnt);
bc_status bc_get_dag(bc_ctx *ctx, bc_graph_id g, int32_t s, int32_t *a, int32_t *b, int64_t cap, int64_t *cnt);
bc_status bc_get_estar(bc_ctx *ctx, bc_graph_id g, int32_t *a, int32_t *b, int64_t *w, int64_t cap, int64_t *cnt);
bc_status bc_get_delta(bc_ctx *ctx, bc_graph_id g, int32_t s, double *out);

/* bc_get_delta for callers that cannot allocate (code under HIP graph
 * capture, serving loops, harnesses that forbid allocation): the same
 * dependency row delta_s.(.) (Eq.4 summed over every reachable target, 0 at
 * s and at unreachable vertices), written to out_dev[0..n), caller-owned
 * device memory of n doubles, by one kernel enqueued on the context's stream.
 * It allocates nothing and uses no caller workspace: its work area is a fixed
 * array in the library's device image (one wide-kernel slot, about 3.5 MB,
 * held by every device the library runs on until the process ends), resolved
 * once per device at bc_create.  It does not synchronise; the row is there
 * once the stream reaches it, and device errors surface at the next
 * synchronising call.  Graphs of up to 32768 vertices; a larger one returns
 * BC_ERR_CAPACITY and enqueues nothing.  Every call on one device shares the
 * array: calls that can overlap on the device (other contexts' streams on the
 * same GPU) race and must be ordered by the caller.
 * Errors: BC_ERR_INVALID_ARG (no such graph, s out of range, null out_dev),
 * BC_ERR_CAPACITY. */
bc_status bc_get_delta_noalloc(bc_ctx *ctx, bc_graph_id g, int32_t s, double *out_dev);
bc_status bc_get_preds(bc_ctx *ctx, bc_graph_id g, int32_t s, int32_t *out);
bc_status bc_get_affected(bc_ctx *ctx, bc_graph_id g, int32_t *out, int64_t cap, int64_t *cnt);
bc_status bc_state_hash(bc_ctx *ctx, bc_graph_id g, uint64_t out[2]);

/* State check, a debugging aid: tests the graph's state against the
 * definitions on the device, over its current arcs (a thread per pair).  For
 * every source s and target t, with the arcs (a,t) of weight w whose tail
 * a is reachable from s:
 *   - d(s,s) = 0, sigma_ss = 1, no stored predecessor at s (BC_CHECK_SOURCE);
 *   - no arc gives d(s,a) + w < d(s,t), and none leads from a reachable a to
 *     an unreachable t (BC_CHECK_RELAX);
 *   - a reachable t has an arc with d(s,a) + w = d(s,t), an arc of DAG(s)
 *     by Eq.1 (BC_CHECK_NO_PATH); sigma_st is the sum of sigma_sa over those
 *     arcs (BC_CHECK_SIGMA); its stored predecessor (bc_get_preds) is the
 *     tail of the only one, or -2 for several (BC_CHECK_PRED);
 *   - an unreachable t has sigma_st = 0 and no stored predecessor
 *     (BC_CHECK_UNREACHED);
 *   - an undirected graph has equal d and sigma at (s,t) and (t,s)
 *     (BC_CHECK_SYMMETRY);
 * and E* holds exactly the arcs (a,b) with w(a,b) = d(a,b), once each, with
 * their current weights (BC_CHECK_ESTAR).  With positive weights the first
 * three fix d and sigma uniquely, so a state that passes has the exact
 * distances, path counts, stored predecessors and E* of its arcs.  BC itself
 * is not checked.
 * bc_check runs it on every source and synchronises.  A context created with
 * BC_FLAG_CHECK runs it after every load and recompute, and after every
 * update step on the step's affected sources (sources outside A keep their
 * rows by Lemma 2 and Lemma 4) and all of E*; a failing step makes its call
 * return BC_ERR_CHECK_FAILED.
 * A failure is sticky (BC_ERR_CHECK_FAILED, ranked after the overflow and E*
 * capacity errors, until bc_recompute) and its first instance is in
 * bc_last_error and bc_update_stats.  A graph that already carries a sticky
 * error is not checked and returns that error.
 * Errors: BC_ERR_INVALID_ARG (no such graph), the sticky errors. */
bc_status bc_check(bc_ctx *ctx, bc_graph_id g);

/* Kinds of a failed check (bc_update_stats.check_kind). */
#define BC_CHECK_SOURCE 1
#define BC_CHECK_RELAX 2
#define BC_CHECK_NO_PATH 3
#define BC_CHECK_SIGMA 4
#define BC_CHECK_PRED 5
#define BC_CHECK_UNREACHED 6
#define BC_CHECK_SYMMETRY 7
#define BC_CHECK_ESTAR 8

typedef struct {
    int64_t affected_sources; /* |A| of the last update (sum over its phases) */
    int64_t changed_pairs;    /* pairs (s,t) whose d or sigma changed */
    int64_t estar_arcs;       /* |E*| after the update */
    int64_t max_levels;       /* deepest DAG level count seen by the static pass */
    int64_t updates_applied;  /* updates since load */
    int64_t total_affected;   /* sum of |A| over all updates since load */
    int64_t total_changed;    /* sum of changed pairs over all updates since load */
    int64_t deferred_sources; /* sources of the last update run by the wide kernel (bc_schedule) */
    int64_t scan_bytes;       /* algorithmic bytes of the last update's row scans: 4n per affected
                                 source (4|T| when the update's candidate targets T are scanned
                                 instead, |T| <= n/8) plus 8 per changed pair (its old sigma) */
    int64_t total_scan_bytes; /* the same summed over all updates since load */
    int64_t search_arcs;      /* arcs the distance search of the last static pass relaxed */
    int64_t search_rounds;    /* its searches when the arc set was checked (0: one search) */
    int64_t check_rows;       /* source rows verified by state checks since load (bc_check) */
    int64_t check_failures;   /* conditions those checks found false */
    int64_t check_source;     /* the first of them: source s (tail for BC_CHECK_ESTAR), -1 if none */
    int64_t check_target;     /* its target t (head for BC_CHECK_ESTAR), -1 if none */
    int64_t check_kind;       /* its BC_CHECK_* kind, 0 if none */
} bc_update_stats;
bc_status bc_get_stats(bc_ctx *ctx, bc_graph_id g, bc_update_stats *out);

/* Kernel timing of a context created with BC_FLAG_TIMING: HIP events on the
 * context's stream bracket every update step (all its kernels) and, inside
 * it, the per-source kernels (the row kernel, which scans the rows of the
 * affected sources, then the DAG and wide kernels, which run the partial
 * dependencies) and the row kernel alone.  Totals cover the steps finished
 * since the last bc_reset_timing (bc_get_timing synchronises first). */
typedef struct {
    double step_ms;          /* summed duration of update steps */
    double source_ms;        /* summed duration of the per-source kernels (row, DAG and wide) */
    int64_t steps;           /* update steps timed (one launch of each kernel) */
    double rows_ms;          /* summed duration of the row kernel alone */
} bc_timing;
bc_status bc_get_timing(bc_ctx *ctx, bc_timing *out);
bc_status bc_reset_timing(bc_ctx *ctx);

/* Launch schedule of the per-source step (the all-pairs part of Alg 3 with
 * the dependency accumulation of Alg 1, one affected source per workgroup).
 * It changes only how affected sources map onto workgroups, never a result:
 * every schedule reaches the same D, sigma, DAG and (within rounding order)
 * BC.  A source whose changed-target set has more than big_b entries is
 * deferred to a second kernel with wider workgroups (wide_block threads),
 * which stages the source's distance row in LDS when wide_stage is set and the
 * row fits (n <= 36864).  Fields set to 0 keep their current value.
 *   block:      threads per workgroup of the first kernel: 64, 128, 192, 256
 *   slots:      its persistent workgroups (at most bc_config.slots)
 *   big_b:      deferral threshold, 1..1024
 *   wide_block: threads per workgroup of the wide kernel: 256, 512 or 1024
 *   wide_stage: 1 = stage rows in LDS when they fit, 2 = never stage
 *   wide_slots: persistent workgroups of the wide kernel (at most slots)
 *   table:      slots of the DAG kernel's LDS sub-DAG tables: 128 or 256
 *               (smaller tables fit more workgroups per CU, larger ones
 *               send fewer sub-DAGs to global memory)
 * bc_set_schedule synchronises the context's stream before it switches.
 * Errors: BC_ERR_INVALID_ARG for a value out of range (nothing changes). */
typedef struct {
    int32_t block;
    int32_t slots;
    int32_t big_b;
    int32_t wide_block;
    int32_t wide_stage;
    int32_t wide_slots;
    int32_t table;
} bc_schedule;
bc_status bc_set_schedule(bc_ctx *ctx, const bc_schedule *s);
bc_status bc_get_schedule(bc_ctx *ctx, bc_schedule *out);

/* Autotuner of the launch schedule.  reqs[0..cnt) is a sample of requests
 * in bc_submit form on resident graphs (typically updates like the expected
 * stream, drawn for tuning).  Schedules are kept per size bucket
 * (ceil(log2 n)) and a step takes the one of its largest graph's bucket, so
 * bucket B is tuned on the sample's requests on graphs of bucket B and below
 * (steps like the ones it will serve); a bucket that already has a schedule,
 * from an earlier tuning or from the cache file, keeps it and runs nothing.
 * For the others, each candidate schedule (table 128 or 256; block 256, 128
 * or 64, the last one wave per source; wide_block 512 or 1024; big_b 512 or
 * 1024; the other fields as set) runs that sample on fresh device clones
 * of its graphs, twice (the first run also captures the step graphs), and
 * the summed device time of the second run's steps ranks it.  Afterwards
 * every step takes the schedule of its bucket (the size of its largest
 * graph) while one is known, the context's schedule is the largest sampled
 * bucket's (returned in *chosen, may be NULL), and when bc_config named a
 * cache file every known bucket's schedule is written to it (JSON, with the
 * device kind; bc_create reads it back on the same kind of device).
 * bc_set_schedule afterwards applies its schedule to every step again.  The
 * resident graphs are never modified.
 *   workspace: caller-owned device memory, 256-byte aligned, of at least the
 *     sum over the distinct sampled graphs of align256(bc_graph_bytes(...)),
 *     holding the clones during the call.
 * Synchronises.  Errors: BC_ERR_INVALID_ARG (also: the cache file cannot be
 * written), BC_ERR_CAPACITY (workspace too small), any validation error of
 * the sample (the schedule is then left as it was). */
bc_status bc_autotune(bc_ctx *ctx, int32_t cnt, const bc_request *reqs, void *workspace, uint64_t workspace_bytes,
                      bc_schedule *chosen);

const char *bc_status_string(bc_status s);
const char *bc_last_error(bc_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* BCINC_H */
