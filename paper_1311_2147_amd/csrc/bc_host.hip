// Host side of libbcinc: the C ABI declared in include/bcinc.h.
//
// Responsibilities: validation of every request against a host mirror of the
// arcs (so a rejected call leaves all state unchanged), carving each graph's
// caller-provided device arena, staging update jobs, launching the kernel
// sequence (directly for single updates, replayed from a captured HIP graph
// for batched steps) and introspection copies.  All arithmetic of the method
// runs in the kernels of bc_kernels.hip.
#include <time.h>

#include <cmath>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <set>
#include <mutex>
#include <tuple>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/bcinc.h"
#include "bc_device.h"

// The kernels live in bc_kernels.hip, compiled in the same translation unit
// (see bcinc.hip).

using namespace bcinc;

namespace {
// size of the fixed scratch array below (one wide-kernel slot, n <= 32768)
constexpr size_t FIXED_BYTES = wide_layout(32768).total;
}  // namespace

// Fixed device scratch of bc_get_delta_noalloc (see fixed_scratch_setup).
static __device__ __align__(256) char bc_fixed_scratch[FIXED_BYTES];

namespace {

constexpr int RING = 4;            // job staging slots in flight
constexpr int JCAP = 256;          // jobs per staging slot
constexpr size_t MISC_BYTES = 4096;
constexpr int DEFAULT_SLOTS = 2560; // 10 persistent 128-thread workgroups per CU of an MI355X (5 waves per SIMD)
constexpr int WIDE_SLOTS_MAX = 256; // wide-kernel slots: one per CU
constexpr int DEFAULT_BLOCK = 256;  // 4 waves per affected source
constexpr int DEFAULT_WIDE_BLOCK = 512;
constexpr int64_t W_MAX = (int64_t)INF32 - 1;
constexpr int STATUS_BATCH = 256;   // graph status words read back per copy batch
constexpr int64_t CLOCK_REFRESH_NS = 10000000000ll;  // re-map the device clock after 10 s

// Fixed scratch of the allocation-free entry point (bc_get_delta_noalloc):
// one wide-kernel work slot laid out for graphs of up to FIXED_N_MAX vertices,
// in the library's device image.  Each device holds its own copy until the
// process ends; host code reaches it only through the address
// hipGetSymbolAddress returns for that device (the array's name in host code
// is not a device address).
constexpr int32_t FIXED_N_MAX = 32768;
constexpr size_t FIXED_SCRATCH_BYTES = wide_layout(FIXED_N_MAX).total;
static_assert(FIXED_SCRATCH_BYTES == FIXED_BYTES, "fixed scratch sized for another n");
constexpr int FIXED_MAX_DEVICES = 64;

std::mutex fixed_mu;
void *fixed_addr[FIXED_MAX_DEVICES] = {};  // per device, resolved once

size_t ring_slot_bytes() { return align256(256 + sizeof(UpdateJob) * JCAP); }
size_t ring_bytes() { return RING * ring_slot_bytes(); }

struct Mirror {
    // Arcs of G (G_D when undirected) as a CSR by tail, heads sorted, plus an
    // overlay of arcs inserted since the last rebuild.
    int32_t n = 0;
    std::vector<int64_t> ptr;
    std::vector<int32_t> dst;
    std::vector<int32_t> w;
    std::unordered_map<uint64_t, int32_t> extra;
    int64_t arcs = 0;

    uint64_t key(int32_t a, int32_t b) const { return (uint64_t)a * (uint64_t)n + (uint64_t)b; }

    // current weight of (a,b), or -1 when absent
    int64_t find(int32_t a, int32_t b) const {
        auto first = dst.begin() + ptr[a], last = dst.begin() + ptr[a + 1];
        auto it = std::lower_bound(first, last, b);
        if (it != last && *it == b) return w[it - dst.begin()];
        auto e = extra.find(key(a, b));
        return e == extra.end() ? -1 : e->second;
    }

    void set(int32_t a, int32_t b, int32_t wt) {
        auto first = dst.begin() + ptr[a], last = dst.begin() + ptr[a + 1];
        auto it = std::lower_bound(first, last, b);
        if (it != last && *it == b) {
            w[it - dst.begin()] = wt;
            return;
        }
        auto e = extra.find(key(a, b));
        if (e == extra.end()) {
            extra.emplace(key(a, b), wt);
            ++arcs;
        } else {
            e->second = wt;
        }
    }

    // Folds the overlay into the CSR.
    void compact() {
        if (extra.empty()) return;
        std::vector<std::vector<std::pair<int32_t, int32_t>>> add(n);
        for (auto &kv : extra) add[kv.first / n].push_back({(int32_t)(kv.first % n), kv.second});
        std::vector<int64_t> np(n + 1, 0);
        std::vector<int32_t> nd, nw;
        nd.reserve(arcs);
        nw.reserve(arcs);
        for (int32_t a = 0; a < n; ++a) {
            std::vector<std::pair<int32_t, int32_t>> row;
            for (int64_t e = ptr[a]; e < ptr[a + 1]; ++e) row.push_back({dst[e], w[e]});
            row.insert(row.end(), add[a].begin(), add[a].end());
            std::sort(row.begin(), row.end());
            for (auto &p : row) {
                nd.push_back(p.first);
                nw.push_back(p.second);
            }
            np[a + 1] = (int64_t)nd.size();
        }
        ptr.swap(np);
        dst.swap(nd);
        w.swap(nw);
        extra.clear();
    }
};

struct GraphRec {
    bool live = false;
    int32_t n = 0;
    int32_t directed = 1;
    int64_t arc_cap = 0, es_cap = 0;
    char *arena = nullptr;
    uint64_t arena_bytes = 0;
    GraphPtrs P{};
    Mirror mirror;
    uint64_t updates = 0;
    int64_t search_arcs = 0;   // arcs the last static pass's distance search relaxed
    int32_t search_rounds = 0; // searches of its checked search (0: one search over a given set)
    CheckRec *chk = nullptr;   // the state checks' record (in the arena)
    // BC_FLAG_CHECK: the arcs as of the last step launched on the device (the
    // mirror runs ahead by every request validated but not launched yet)
    Mirror dev;
};

struct StepGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

// Timing events recorded on the stream around one update step (before its
// staging copy, after its last kernel); tickets whose requests ran in the
// step hold references to them.
struct StepEvents {
    hipEvent_t begin = nullptr, end = nullptr;
    int refs = 0;
};

// A submission (bc_submit), a queued request (bc_enqueue) or a step
// (bc_step): its first and last step's events, the graphs it touched, and
// its jobs not launched yet.
struct Ticket {
    int64_t t_enqueue_ns = 0;
    StepEvents *first = nullptr, *last = nullptr;
    std::vector<int32_t> graphs;
    int32_t jobs_queued = 0;
};

// A job waiting in its graph's FIFO for bc_step.
struct QueuedJob {
    UpdateJob job;
    uint64_t ticket;
    uint64_t seq;  // enqueue order over all graphs
};

int64_t monotonic_ns() {
    timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (int64_t)ts.tv_sec * 1000000000ll + ts.tv_nsec;
}

}  // namespace

struct bc_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    // second stream (default priority): the wide kernel runs on it beside the
    // DAG kernel, forked after the row kernel and joined before the E* filter
    hipStream_t side = nullptr;
    hipEvent_t fork_ev = nullptr, join_ev = nullptr;
    char *scratch = nullptr;
    uint64_t scratch_bytes = 0;
    uint64_t budget = 0;
    uint64_t in_use = 0;
    int slots = DEFAULT_SLOTS;  // workgroup slots the scratch buffer was sized for
    int cu_count = 256;
    // launch schedule of the per-source step (bc_schedule)
    int block = DEFAULT_BLOCK;
    int run_slots = 0;   // 0: every usable slot
    int big_b = BIG_B;
    int wide_block = DEFAULT_WIDE_BLOCK;
    int wide_stage = 1;
    int wide_slots = 0;  // 0: one workgroup per CU when staging, else two
    int table = 256;     // LDS sub-DAG table slots of the DAG kernel
    size_t wide_lds_limit = 0;  // dynamic LDS the wide kernel may use
    size_t sssp_lds_limit = 0;  // and the static search
    int rows_grid = 1024;       // workgroups of the row kernel (all resident)
    int32_t n_layout = 1;  // slot layout size: the largest graph ever loaded
    bool full_search = false;  // BC_FLAG_FULL_SEARCH: the static pass relaxes every arc
    bool check = false;        // BC_FLAG_CHECK: state check after every load, recompute and step
    // schedules chosen by the autotuner per size bucket (ceil(log2 n) of a
    // step's largest graph), used while use_tuned is set; the cache file
    // keeps them across contexts of the same device kind
    std::map<int, bc_schedule> tuned;
    bool use_tuned = false;
    std::string tune_cache;
    std::string device_tag;
    int32_t src_lds_max = 8192;  // per-source kernel stages rows up to this n in LDS
    std::vector<GraphRec *> graphs;
    std::string last_error;
    // staging
    // pinned host image of each staging slot, laid out as on the device (the
    // job count in a 256-byte header, then the jobs): one copy stages a step
    char *h_ring[RING] = {};
    UpdateJob *h_jobs[RING] = {};
    int32_t *h_njobs[RING] = {};
    hipEvent_t ring_ev[RING] = {};
    bool ring_used[RING] = {};
    int ring_next = 0;
    // timing (BC_FLAG_TIMING): per staging slot, events at step start, around
    // the per-source kernel, and at step end
    bool timing = false;
    hipEvent_t tev[RING][5] = {};  // before parts 0..3 and after part 3
    bool tev_pending[RING] = {};
    double step_ms = 0, source_ms = 0, rows_ms = 0;
    int64_t timed_steps = 0;
    // captured step parts, keyed by everything their launches bake in
    std::map<std::vector<int64_t>, StepGraph> graph_cache;
    // tickets, the step events they refer to, and the FIFOs of queued jobs
    uint64_t next_ticket = 1;
    std::map<uint64_t, Ticket> tickets;
    std::vector<StepEvents *> spare_steps;
    std::map<int32_t, std::deque<QueuedJob>> queues;
    uint64_t queue_seq = 0;
    int64_t queued_jobs = 0;
    // device clock against CLOCK_MONOTONIC: clock_ev completed at host time
    // clock_ns (within half of clock_span_ns); recorded on a stream of its
    // own, which never waits for update work
    hipStream_t clock_stream = nullptr;
    hipEvent_t clock_ev = nullptr;
    int64_t clock_ns = 0, clock_span_ns = 0;
    int32_t *h_status = nullptr;  // pinned: graph status words read back for results
    // this device's copy of the fixed scratch array (see bc_fixed_scratch)
    char *fixed_scratch = nullptr;
};

namespace {

bc_status hip_fail(bc_ctx *ctx, hipError_t e, const char *what) {
    if (ctx) {
        char buf[512];
        snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
        ctx->last_error = buf;
    }
    return BC_ERR_HIP;
}

#define HIPCHK(call)                                           \
    do {                                                       \
        hipError_t e_ = (call);                                \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, #call); \
    } while (0)

bc_status fail(bc_ctx *ctx, bc_status s, const std::string &msg) {
    if (ctx) ctx->last_error = msg;
    return s;
}

char *ring_dev(bc_ctx *ctx, int r) { return ctx->scratch + (size_t)r * ring_slot_bytes(); }
UpdateJob *ring_jobs_dev(bc_ctx *ctx, int r) { return (UpdateJob *)(ring_dev(ctx, r) + 256); }
int32_t *ring_njobs_dev(bc_ctx *ctx, int r) { return (int32_t *)ring_dev(ctx, r); }
char *misc_dev(bc_ctx *ctx) { return ctx->scratch + ring_bytes(); }

// Target pool of an update step (after the misc area): 256 entries per vertex
// of the largest graph, at least 2^20; 16 bytes per entry.
int64_t pool_entries(int32_t n_max) { return std::max<int64_t>(int64_t(1) << 20, 256 * (int64_t)n_max); }
size_t pool_bytes(int32_t n_max) { return align256(16 * (size_t)pool_entries(n_max)); }
char *pool_dev(bc_ctx *ctx) { return ctx->scratch + ring_bytes() + MISC_BYTES; }
// Device staging of the status gather, one area per stream that reads status
// back (the main stream and the clock stream); each holds STATUS_BATCH words.
int32_t *status_dev(bc_ctx *ctx, bool clock) { return (int32_t *)(misc_dev(ctx) + (clock ? 3072 : 1024)); }
static_assert(1024 + 4 * STATUS_BATCH <= 2048 && 3072 + 4 * STATUS_BATCH <= MISC_BYTES, "status staging areas");
StepPool step_pool(bc_ctx *ctx) {
    StepPool p;
    p.cap = pool_entries(ctx->n_layout);
    p.t = (int32_t *)pool_dev(ctx);
    p.d = p.t + p.cap;
    p.s = (uint64_t *)(p.d + p.cap);
    p.next = (unsigned long long *)(misc_dev(ctx) + 2048);
    return p;
}
int wide_slots_for(int slots) { return std::min(slots, WIDE_SLOTS_MAX); }

// The part of the scratch buffer after the pool, laid out for graphs of up to
// n vertices: `src` slots of the DAG kernel and the static pass, then `wide`
// slots of the wide kernel, then as many item regions (changed-pair lists of
// deferred sources whose two passes run apart).  Fewer slots than configured
// when the buffer was sized for a smaller n; zero counts when not even one of
// each fits.
struct ScratchPlan {
    int src = 0, wide = 0;
    size_t src_bytes = 0, wide_bytes = 0, item_bytes = 0;
    char *src_base = nullptr, *wide_base = nullptr, *items_base = nullptr;
};

ScratchPlan plan_scratch(bc_ctx *ctx, int32_t n) {
    ScratchPlan p;
    p.src_bytes = slot_bytes_for(n);
    p.wide_bytes = wide_slot_bytes_for(n);
    p.item_bytes = item_region_bytes(n);
    const uint64_t fixed = ring_bytes() + MISC_BYTES + pool_bytes(n);
    if (ctx->scratch_bytes <= fixed) return p;
    const uint64_t avail = ctx->scratch_bytes - fixed;
    const uint64_t per_wide = p.wide_bytes + p.item_bytes;
    uint64_t w = (uint64_t)wide_slots_for(ctx->slots);
    w = std::min<uint64_t>(w, avail / (per_wide + p.src_bytes));
    if (w < 1) return p;
    const uint64_t s = std::min<uint64_t>((uint64_t)ctx->slots, (avail - w * per_wide) / p.src_bytes);
    if (s < 1) return p;
    p.src = (int)s;
    p.wide = (int)w;
    p.src_base = pool_dev(ctx) + pool_bytes(n);
    p.wide_base = p.src_base + s * p.src_bytes;
    p.items_base = p.wide_base + w * p.wide_bytes;
    return p;
}

int lds_cap_for(int32_t n_max) { return std::min<int32_t>(n_max, LDS_ROW_MAX); }

// Dynamic LDS of the per-source kernels: staged row, XB bytes per thread of
// expansion arrays, and the LDS sub-DAG tables of `table` slots (0: none; the
// wide kernel and the dependency-row kernel use none).
size_t table_bytes(int table) {
    if (table == 256) return std::max(small_dag_bytes<256>(), dual_dag_bytes<256>());
    if (table == 128) return std::max(small_dag_bytes<128>(), dual_dag_bytes<128>());
    return 0;
}
size_t source_lds_bytes(int lds_cap, int block, int table) {
    return align256((size_t)lds_cap * 4) + align256(XB * (size_t)block) + table_bytes(table);
}

// Arena layout of one graph (every piece 256-byte aligned).
struct Carve {
    size_t off = 0;
    size_t take(size_t bytes) {
        size_t o = off;
        off += align256(bytes);
        return o;
    }
};

GraphPtrs carve(char *base, int32_t n, int64_t arc_cap, int64_t es_cap, size_t *total, CheckRec **chk = nullptr) {
    Carve c;
    const size_t nn = (size_t)n * (size_t)n;
    size_t oD = c.take(4 * nn), oS = c.take(8 * nn), oPr = c.take(4 * nn);
    size_t ohi = c.take(8 * (size_t)n), olo = c.take(8 * (size_t)n), odl = c.take(8 * (size_t)n);
    size_t oxp = c.take(4 * ((size_t)n + 1)), oxs = c.take(4 * (size_t)es_cap), oxd = c.take(4 * (size_t)es_cap),
           oxw = c.take(4 * (size_t)es_cap);
    size_t oxcp = c.take(4 * ((size_t)n + 1)), oxcs = c.take(4 * (size_t)es_cap), oxcd = c.take(4 * (size_t)es_cap),
           oxcw = c.take(4 * (size_t)es_cap);
    size_t oyp = c.take(4 * ((size_t)n + 1)), oys = c.take(4 * (size_t)es_cap), oyd = c.take(4 * (size_t)es_cap),
           oyw = c.take(4 * (size_t)es_cap);
    size_t ocnt = c.take(4 * ((size_t)n + 1));
    size_t osc = c.take(sizeof(SrcScal) * (size_t)n), oal = c.take(4 * (size_t)n), obig = c.take(4 * (size_t)n);
    size_t odl2 = c.take(sizeof(DItem) * (size_t)n);
    size_t ofi = c.take(4 * (size_t)n), ofo = c.take(4 * (size_t)n);
    size_t orvd = c.take(4 * (size_t)n), orvs = c.take(8 * (size_t)n);
    size_t orvvd = c.take(4 * (size_t)n), orvvs = c.take(8 * (size_t)n), orvvh = c.take(8 * (size_t)n);
    size_t otl = c.take(4 * (size_t)n), otlr = c.take(4 * (size_t)n), otlrr = c.take(4 * (size_t)n);
    size_t octl = c.take(sizeof(GraphCtl));
    size_t oap = c.take(4 * ((size_t)n + 1)), oad = c.take(4 * (size_t)arc_cap), oaw = c.take(4 * (size_t)arc_cap);
    size_t oip = c.take(4 * ((size_t)n + 1)), ois = c.take(4 * (size_t)arc_cap), oiw = c.take(4 * (size_t)arc_cap);
    size_t ochk = c.take(sizeof(CheckRec));
    *total = c.off;
    GraphPtrs P{};
    if (!base) return P;
    if (chk) *chk = (CheckRec *)(base + ochk);
    P.n = n;
    P.es_cap = es_cap;
    P.D = (int32_t *)(base + oD);
    P.pred = (int32_t *)(base + oPr);
    P.S = (uint64_t *)(base + oS);
    P.bc_hi = (double *)(base + ohi);
    P.bc_lo = (double *)(base + olo);
    P.bc_delta = (double *)(base + odl);
    P.x_ptr = (int32_t *)(base + oxp);
    P.x_src = (int32_t *)(base + oxs);
    P.x_dst = (int32_t *)(base + oxd);
    P.x_w = (int32_t *)(base + oxw);
    P.xc_ptr = (int32_t *)(base + oxcp);
    P.xc_src = (int32_t *)(base + oxcs);
    P.xc_dst = (int32_t *)(base + oxcd);
    P.xc_w = (int32_t *)(base + oxcw);
    P.yc_ptr = (int32_t *)(base + oyp);
    P.yc_src = (int32_t *)(base + oys);
    P.yc_dst = (int32_t *)(base + oyd);
    P.yc_w = (int32_t *)(base + oyw);
    P.es_cnt = (int32_t *)(base + ocnt);
    P.scal = (SrcScal *)(base + osc);
    P.alist = (int32_t *)(base + oal);
    P.biglist = (int32_t *)(base + obig);
    P.dlist = (DItem *)(base + odl2);
    P.f_any = (int32_t *)(base + ofi);
    P.f_out = (int32_t *)(base + ofo);
    P.rv_D = (int32_t *)(base + orvd);
    P.rv_S = (uint64_t *)(base + orvs);
    P.rvv_D = (int32_t *)(base + orvvd);
    P.rvv_S = (uint64_t *)(base + orvvs);
    P.rvv_H = (uint64_t *)(base + orvvh);
    P.tlist = (int32_t *)(base + otl);
    P.tl_rvD = (int32_t *)(base + otlr);
    P.tl_rvvD = (int32_t *)(base + otlrr);
    P.ctl = (GraphCtl *)(base + octl);
    P.arc_ptr = (int32_t *)(base + oap);
    P.arc_dst = (int32_t *)(base + oad);
    P.arc_w = (int32_t *)(base + oaw);
    P.arcin_ptr = (int32_t *)(base + oip);
    P.arcin_src = (int32_t *)(base + ois);
    P.arcin_w = (int32_t *)(base + oiw);
    return P;
}

GraphRec *get_graph(bc_ctx *ctx, bc_graph_id g) {
    if (!ctx || g < 0 || g >= (int)ctx->graphs.size()) return nullptr;
    GraphRec *r = ctx->graphs[g];
    return (r && r->live) ? r : nullptr;
}

// Adds the timed durations of slot r's last step (its events have completed).
bc_status harvest_timing(bc_ctx *ctx, int r) {
    if (!ctx->tev_pending[r]) return BC_OK;
    float a = 0, b = 0, c = 0;
    HIPCHK(hipEventElapsedTime(&a, ctx->tev[r][0], ctx->tev[r][4]));  // whole step
    HIPCHK(hipEventElapsedTime(&b, ctx->tev[r][1], ctx->tev[r][3]));  // per-source kernels
    HIPCHK(hipEventElapsedTime(&c, ctx->tev[r][1], ctx->tev[r][2]));  // row kernel
    ctx->step_ms += a;
    ctx->source_ms += b;
    ctx->rows_ms += c;
    ctx->timed_steps += 1;
    ctx->tev_pending[r] = false;
    return BC_OK;
}

bc_status harvest_all(bc_ctx *ctx) {
    for (int r = 0; r < RING; ++r)
        if (ctx->tev_pending[r]) {
            HIPCHK(hipEventSynchronize(ctx->tev[r][4]));
            bc_status st = harvest_timing(ctx, r);
            if (st) return st;
        }
    return BC_OK;
}

// Acquire a staging slot (waits until its previous use has finished).
bc_status ring_acquire(bc_ctx *ctx, int *slot) {
    int r = ctx->ring_next;
    ctx->ring_next = (r + 1) % RING;
    if (ctx->ring_used[r]) HIPCHK(hipEventSynchronize(ctx->ring_ev[r]));
    ctx->ring_used[r] = false;
    bc_status st = harvest_timing(ctx, r);
    if (st) return st;
    *slot = r;
    return BC_OK;
}

bc_status ring_stage(bc_ctx *ctx, int r, const std::vector<UpdateJob> &jobs) {
    const size_t nj = jobs.size();
    if (nj > (size_t)JCAP) return fail(ctx, BC_ERR_CAPACITY, "too many jobs in one step");
    *ctx->h_njobs[r] = (int32_t)nj;
    if (nj) memcpy(ctx->h_jobs[r], jobs.data(), sizeof(UpdateJob) * nj);
    HIPCHK(hipMemcpyAsync(ring_dev(ctx, r), ctx->h_ring[r], 256 + sizeof(UpdateJob) * nj, hipMemcpyHostToDevice,
                          ctx->stream));
    return BC_OK;
}

bc_status ring_release(bc_ctx *ctx, int r) {
    HIPCHK(hipEventRecord(ctx->ring_ev[r], ctx->stream));
    ctx->ring_used[r] = true;
    return BC_OK;
}

struct LaunchShape {
    int32_t n_max;
    int njobs;
    int slots;
    size_t slot_bytes;
    int lds_cap;      // static pass: rows up to this size are staged in LDS
    int src_lds_cap;  // per-source kernel: rows up to this size are staged in LDS
    int wide_slots;   // workgroups of the wide per-source kernel
    size_t wide_bytes;
    char *src_base, *wide_base, *items_base;
    int item_regions;
    int wide_lds_cap; // and its LDS staging limit
    int32_t n_layout;
};

// The update kernel sequence for the jobs staged in ring slot r, in four
// parts: 0 = begin, scan, row v'', E* merge; 1 = the row kernel; 2 = the DAG
// and wide kernels; 3 = E* filter and commit.
bc_status launch_update_part(bc_ctx *ctx, int r, const LaunchShape &L, int part) {
    const UpdateJob *jobs = ring_jobs_dev(ctx, r);
    const int32_t *nj = ring_njobs_dev(ctx, r);
    hipStream_t st = ctx->stream;
    const int g_elem = (int)std::min<int64_t>(((int64_t)L.n_max + 255) / 256, 2048);
    const int g_wave = (int)std::min<int64_t>(((int64_t)L.n_max * 64 + 255) / 256, 4096);
    const StepPool pool = step_pool(ctx);
    if (part == 0) {
        hipLaunchKernelGGL(k_begin, dim3(1), dim3(64), 0, st, jobs, nj, pool);
        hipLaunchKernelGGL(k_scan, dim3(g_elem, L.njobs), dim3(256), 0, st, jobs, nj);
        hipLaunchKernelGGL(k_targets, dim3(g_elem, L.njobs), dim3(256), 0, st, jobs, nj);
        hipLaunchKernelGGL(k_es_merge, dim3(g_wave, L.njobs), dim3(256), 0, st, jobs, nj);
    } else if (part == 1) {
        hipLaunchKernelGGL(k_rows, dim3(ctx->rows_grid), dim3(256), 0, st, jobs, nj, ctx->big_b, pool);
    } else if (part == 2) {
        // the wide kernel (deferred sources) and the DAG kernel (listed
        // sources) touch disjoint rows and run side by side: the wide one
        // directly behind the row kernel on the main stream, so its few long
        // workgroups (a whole CU each) start first, the DAG kernel on the
        // side stream, filling the remaining CUs
        HIPCHK(hipEventRecord(ctx->fork_ev, st));
        HIPCHK(hipStreamWaitEvent(ctx->side, ctx->fork_ev, 0));
        hipLaunchKernelGGL(k_source_wide, dim3(L.wide_slots), dim3(ctx->wide_block),
                           source_lds_bytes(L.wide_lds_cap, ctx->wide_block, 0), st, jobs, nj, L.wide_base,
                           L.wide_bytes, L.wide_lds_cap, L.n_layout, L.items_base, L.item_regions);
        const size_t lds = source_lds_bytes(L.src_lds_cap, ctx->block, ctx->table);
        if (ctx->table == 128)
            hipLaunchKernelGGL(k_source<128>, dim3(L.slots), dim3(ctx->block), lds, ctx->side, jobs, nj, L.src_base,
                               L.slot_bytes, L.src_lds_cap, L.n_layout, pool);
        else
            hipLaunchKernelGGL(k_source<256>, dim3(L.slots), dim3(ctx->block), lds, ctx->side, jobs, nj, L.src_base,
                               L.slot_bytes, L.src_lds_cap, L.n_layout, pool);
        HIPCHK(hipEventRecord(ctx->join_ev, ctx->side));
        hipLaunchKernelGGL(k_wide_apply, dim3(256), dim3(256), 0, st, jobs, nj, L.items_base, L.item_regions,
                           L.n_layout);
        HIPCHK(hipStreamWaitEvent(st, ctx->join_ev, 0));
    } else {
        hipLaunchKernelGGL(k_es_keep, dim3(g_wave, L.njobs), dim3(256), 0, st, jobs, nj);
        hipLaunchKernelGGL(k_es_wscan, dim3(L.njobs), dim3(1024), 0, st, jobs, nj);
        hipLaunchKernelGGL(k_es_place, dim3(g_wave, L.njobs), dim3(256), 0, st, jobs, nj);
        hipLaunchKernelGGL(k_commit, dim3(g_elem, L.njobs), dim3(256), 0, st, jobs, nj, 0);
    }
    HIPCHK(hipGetLastError());
    return BC_OK;
}

// Captured graph of one part, instantiated once per staging slot and shape.
bc_status part_graph(bc_ctx *ctx, int r, const LaunchShape &L, int part, hipGraphExec_t *exec) {
    // every launch argument that comes from the shape (grid sizes from n_max,
    // slot and region layouts from n_layout, bases and counts of the scratch
    // plan) and the schedule fields read at launch are part of the key
    const std::vector<int64_t> key = {r,
                                      part,
                                      L.njobs,
                                      L.n_max,
                                      L.n_layout,
                                      L.slots,
                                      (int64_t)L.slot_bytes,
                                      L.src_lds_cap,
                                      L.wide_slots,
                                      (int64_t)L.wide_bytes,
                                      L.wide_lds_cap,
                                      L.item_regions,
                                      (int64_t)(uintptr_t)L.src_base,
                                      (int64_t)(uintptr_t)L.wide_base,
                                      (int64_t)(uintptr_t)L.items_base,
                                      ctx->block,
                                      ctx->wide_block,
                                      ctx->table,
                                      ctx->big_b,
                                      ctx->rows_grid};
    auto it = ctx->graph_cache.find(key);
    if (it == ctx->graph_cache.end()) {
        StepGraph sg;
        HIPCHK(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
        bc_status cst = launch_update_part(ctx, r, L, part);
        hipError_t ce = hipStreamEndCapture(ctx->stream, &sg.graph);
        if (cst) return cst;
        if (ce != hipSuccess) return hip_fail(ctx, ce, "hipStreamEndCapture");
        HIPCHK(hipGraphInstantiate(&sg.exec, sg.graph, nullptr, nullptr, 0));
        it = ctx->graph_cache.emplace(key, sg).first;
    }
    *exec = it->second.exec;
    return BC_OK;
}

bc_status shape_for(bc_ctx *ctx, const std::vector<UpdateJob> &jobs, LaunchShape *L) {
    L->n_max = 1;
    for (auto &j : jobs) L->n_max = std::max(L->n_max, j.g.n);
    L->njobs = (int)jobs.size();
    L->n_layout = ctx->n_layout;
    const ScratchPlan sp = plan_scratch(ctx, ctx->n_layout);
    if (sp.src < 1) return fail(ctx, BC_ERR_CAPACITY, "scratch too small for one work slot at this n");
    L->slots = sp.src;
    L->slot_bytes = sp.src_bytes;
    L->src_base = sp.src_base;
    L->wide_bytes = sp.wide_bytes;
    L->wide_base = sp.wide_base;
    L->items_base = sp.items_base;
    L->item_regions = sp.wide;
    if (ctx->run_slots > 0) L->slots = std::min(L->slots, ctx->run_slots);
    L->lds_cap = lds_cap_for(L->n_max);
    // the row is staged only when it fits; otherwise no LDS is reserved for it
    L->src_lds_cap = L->n_max <= ctx->src_lds_max ? L->n_max : 0;
    // wide kernel: the row is staged when it fits beside the expansion arrays
    // and the small-DAG table; one workgroup per CU then, else two
    const size_t wide_lds = source_lds_bytes(L->n_max, ctx->wide_block, 0);
    const bool stage = ctx->wide_stage == 1 && wide_lds <= ctx->wide_lds_limit;
    L->wide_lds_cap = stage ? L->n_max : 0;
    const int per_cu = (stage && wide_lds * 2 > ctx->wide_lds_limit) || ctx->wide_block > 512 ? 1 : 2;
    L->wide_slots = std::min(sp.wide, ctx->wide_slots > 0 ? ctx->wide_slots : per_cu * ctx->cu_count);
    return BC_OK;
}

int n_bucket(int32_t n) {
    int b = 0;
    while (b < 31 && (int64_t(1) << b) < (int64_t)n) ++b;
    return b;
}

void put_schedule(bc_ctx *ctx, const bc_schedule &s) {
    ctx->block = s.block;
    ctx->run_slots = s.slots;
    ctx->big_b = s.big_b;
    ctx->wide_block = s.wide_block;
    ctx->wide_stage = s.wide_stage;
    ctx->wide_slots = s.wide_slots;
    ctx->table = s.table;
}

bc_schedule cur_schedule(const bc_ctx *ctx) {
    bc_schedule s;
    s.block = ctx->block;
    s.slots = ctx->run_slots;
    s.big_b = ctx->big_b;
    s.wide_block = ctx->wide_block;
    s.wide_stage = ctx->wide_stage;
    s.wide_slots = ctx->wide_slots;
    s.table = ctx->table;
    return s;
}

// The launch schedule of one step: the tuned one of its size bucket while
// the context uses tuned schedules, else the context's schedule.  Held for
// the step's shape and launches, then the context's schedule is back.
struct ScheduleScope {
    bc_ctx *ctx;
    bc_schedule saved{};
    bool active = false;
    ScheduleScope(bc_ctx *c, int32_t n_max) : ctx(c) {
        if (!ctx->use_tuned) return;
        auto it = ctx->tuned.find(n_bucket(n_max));
        if (it == ctx->tuned.end()) return;
        saved = cur_schedule(ctx);
        put_schedule(ctx, it->second);
        active = true;
    }
    ~ScheduleScope() {
        if (active) put_schedule(ctx, saved);
    }
};

bc_status check_step(bc_ctx *ctx, const std::vector<UpdateJob> &jobs);

bc_status run_step(bc_ctx *ctx, const std::vector<UpdateJob> &jobs, bool use_graph, StepEvents *se = nullptr) {
    int32_t n_max = 1;
    for (auto &j : jobs) n_max = std::max(n_max, j.g.n);
    ScheduleScope scope(ctx, n_max);
    LaunchShape L;
    bc_status st = shape_for(ctx, jobs, &L);
    if (st) return st;
    int r;
    if ((st = ring_acquire(ctx, &r))) return st;
    if (se) HIPCHK(hipEventRecord(se->begin, ctx->stream));
    if ((st = ring_stage(ctx, r, jobs))) return st;
    const bool timed = ctx->timing;
    // timing events sit on the stream between the parts (never inside a graph)
    for (int part = 0; part < 4; ++part) {
        if (timed) HIPCHK(hipEventRecord(ctx->tev[r][part], ctx->stream));
        if (!use_graph) {
            if ((st = launch_update_part(ctx, r, L, part))) return st;
        } else {
            hipGraphExec_t exec;
            if ((st = part_graph(ctx, r, L, part, &exec))) return st;
            HIPCHK(hipGraphLaunch(exec, ctx->stream));
        }
    }
    if (timed) HIPCHK(hipEventRecord(ctx->tev[r][4], ctx->stream));
    if (timed) ctx->tev_pending[r] = true;
    if (se) HIPCHK(hipEventRecord(se->end, ctx->stream));
    if ((st = ring_release(ctx, r))) return st;
    return ctx->check ? check_step(ctx, jobs) : BC_OK;
}

// Step events from the pool (timing-enabled events; created on first use).
bc_status take_step_events(bc_ctx *ctx, StepEvents **out) {
    StepEvents *se;
    if (!ctx->spare_steps.empty()) {
        se = ctx->spare_steps.back();
        ctx->spare_steps.pop_back();
    } else {
        se = new StepEvents();
        hipError_t e = hipEventCreate(&se->begin);
        if (e == hipSuccess) e = hipEventCreate(&se->end);
        if (e != hipSuccess) {
            if (se->begin) (void)hipEventDestroy(se->begin);
            delete se;
            return hip_fail(ctx, e, "hipEventCreate");
        }
    }
    se->refs = 0;
    *out = se;
    return BC_OK;
}

void unref_step(bc_ctx *ctx, StepEvents *se) {
    if (se && --se->refs == 0) ctx->spare_steps.push_back(se);
}

// The ticket's requests ran (in part) in step se: it starts at its first
// such step and ends at its last.
void attach_step(bc_ctx *ctx, Ticket &t, StepEvents *se) {
    if (!t.first) {
        t.first = se;
        se->refs++;
    }
    if (t.last != se) {
        StepEvents *prev = t.last;
        t.last = se;
        se->refs++;
        unref_step(ctx, prev);  // still held as t.first when it was the first step
    }
}

void release_ticket(bc_ctx *ctx, Ticket &t) {
    StepEvents *a = t.first, *b = t.last;
    t.first = t.last = nullptr;
    if (a) unref_step(ctx, a);
    if (b) unref_step(ctx, b);
}

// Maps the device clock to CLOCK_MONOTONIC: an event recorded on the idle
// clock stream completes between two host readings, whose midpoint is taken
// as its time (to within half their distance).  A try whose readings lie
// more than 50 us apart is repeated, up to four tries; the reference is
// always the last try's event and readings.
bc_status calibrate_clock(bc_ctx *ctx) {
    for (int i = 0; i < 4; ++i) {
        const int64_t t0 = monotonic_ns();
        HIPCHK(hipEventRecord(ctx->clock_ev, ctx->clock_stream));
        HIPCHK(hipEventSynchronize(ctx->clock_ev));
        const int64_t t1 = monotonic_ns();
        ctx->clock_ns = t0 + (t1 - t0) / 2;
        ctx->clock_span_ns = t1 - t0;
        if (t1 - t0 < 50000) break;
    }
    return BC_OK;
}

// CLOCK_MONOTONIC time of a completed timing event.
bc_status event_time_ns(bc_ctx *ctx, hipEvent_t ev, int64_t *out) {
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, ctx->clock_ev, ev));
    *out = ctx->clock_ns + (int64_t)((double)ms * 1e6);
    return BC_OK;
}

// Launches the next step of queued jobs: the head job of every graph whose
// FIFO is not empty, oldest head first, at most max_jobs of them.
bc_status launch_queued_step(bc_ctx *ctx, int32_t max_jobs, int32_t *launched, uint64_t *step_ticket) {
    *launched = 0;
    std::vector<std::pair<uint64_t, int32_t>> heads;
    for (auto &kv : ctx->queues)
        if (!kv.second.empty()) heads.push_back({kv.second.front().seq, kv.first});
    if (heads.empty()) return BC_OK;
    std::sort(heads.begin(), heads.end());
    const size_t take = std::min<size_t>(heads.size(), (size_t)std::max(1, std::min<int32_t>(max_jobs, JCAP)));
    std::vector<UpdateJob> jobs;
    std::vector<uint64_t> owners;
    Ticket st;
    for (size_t i = 0; i < take; ++i) {
        auto &q = ctx->queues[heads[i].second];
        jobs.push_back(q.front().job);
        owners.push_back(q.front().ticket);
        st.graphs.push_back(heads[i].second);
        q.pop_front();
    }
    ctx->queued_jobs -= (int64_t)jobs.size();
    StepEvents *se;
    bc_status rc = take_step_events(ctx, &se);
    if (rc) return rc;
    se->refs++;  // held while this function attaches it
    rc = run_step(ctx, jobs, true, se);
    if (!rc) {
        for (uint64_t id : owners) {
            auto it = ctx->tickets.find(id);
            if (it == ctx->tickets.end()) continue;
            attach_step(ctx, it->second, se);
            it->second.jobs_queued--;
        }
        if (step_ticket) {
            st.t_enqueue_ns = monotonic_ns();
            attach_step(ctx, st, se);
            *step_ticket = ctx->next_ticket++;
            ctx->tickets[*step_ticket] = st;
        }
        *launched = (int32_t)jobs.size();
    }
    unref_step(ctx, se);
    return rc;
}

// Launches every queued job (steps of heads until the FIFOs are empty): the
// calls that enqueue work directly, or act on a graph's state, keep the
// order in which requests were validated.
bc_status flush_queues(bc_ctx *ctx) {
    while (ctx->queued_jobs > 0) {
        int32_t launched = 0;
        bc_status st = launch_queued_step(ctx, JCAP, &launched, nullptr);
        if (st) return st;
        if (launched == 0) break;
    }
    return BC_OK;
}

UpdateJob job_template(const GraphRec *g) {
    UpdateJob j;
    memset(&j, 0, sizeof j);
    j.g = g->P;
    return j;
}

// Splits one validated update into jobs of at most KMAX arcs per direction.
// Each job is itself an incremental vertex update at v, so applying them in
// order reaches the same state.
void build_jobs(const GraphRec *g, int32_t v, const std::vector<std::pair<int32_t, int32_t>> &ein,
                const std::vector<std::pair<int32_t, int32_t>> &eout, std::vector<UpdateJob> &out) {
    size_t i = 0, o = 0;
    do {
        UpdateJob j = job_template(g);
        j.v = v;
        while (i < ein.size() && j.n_in < KMAX) {
            j.in_tail[j.n_in] = ein[i].first;
            j.in_w[j.n_in] = ein[i].second;
            j.u_tail[j.n_u] = ein[i].first;
            j.u_head[j.n_u] = v;
            j.u_w[j.n_u] = ein[i].second;
            ++j.n_in, ++j.n_u, ++i;
        }
        while (o < eout.size() && j.n_out < KMAX) {
            j.out_head[j.n_out] = eout[o].first;
            j.out_w[j.n_out] = eout[o].second;
            j.u_tail[j.n_u] = v;
            j.u_head[j.n_u] = eout[o].first;
            j.u_w[j.n_u] = eout[o].second;
            ++j.n_out, ++j.n_u, ++o;
        }
        if (j.n_out > 0) {
            j.row_v_D = g->P.rv_D;
            j.row_v_S = g->P.rv_S;
        } else {
            j.row_v_D = g->P.D + (size_t)v * g->n;
            j.row_v_S = g->P.S + (size_t)v * g->n;
        }
        out.push_back(j);
    } while (i < ein.size() || o < eout.size());
}

// Validates one request against the mirror plus the pending changes of
// earlier requests in the same call; on success appends its jobs and its
// arc changes.
struct Pending {
    std::map<std::pair<int32_t, int32_t>, int32_t> arcs;  // (a,b) -> new weight
    int64_t inserted = 0;
};

int64_t current_weight(const GraphRec *g, const Pending &p, int32_t a, int32_t b) {
    auto it = p.arcs.find({a, b});
    if (it != p.arcs.end()) return it->second;
    return g->mirror.find(a, b);
}

bc_status check_edge_arg(bc_ctx *ctx, const GraphRec *g, int32_t a, int32_t b, int64_t w) {
    if (a < 0 || b < 0 || a >= g->n || b >= g->n) return fail(ctx, BC_ERR_INVALID_ARG, "vertex id out of range");
    if (a == b) return fail(ctx, BC_ERR_SELF_LOOP, "self-loop");
    if (w <= 0 || w > W_MAX) return fail(ctx, BC_ERR_BAD_WEIGHT, "weight out of range");
    return BC_OK;
}

bc_status validate_vertex(bc_ctx *ctx, GraphRec *g, int32_t v, int32_t k, const bc_edge *e, Pending &p,
                          std::vector<UpdateJob> &jobs) {
    if (v < 0 || v >= g->n) return fail(ctx, BC_ERR_INVALID_ARG, "vertex id out of range");
    if (k < 0 || (k > 0 && !e)) return fail(ctx, BC_ERR_INVALID_ARG, "bad edge list");
    std::vector<std::pair<int32_t, int32_t>> ein, eout;
    std::vector<std::pair<std::pair<int32_t, int32_t>, int32_t>> changes;
    std::map<std::pair<int32_t, int32_t>, int> seen;
    for (int32_t i = 0; i < k; ++i) {
        const int32_t a = e[i].a, b = e[i].b;
        bc_status st = check_edge_arg(ctx, g, a, b, e[i].w);
        if (st) return st;
        if (a != v && b != v) return fail(ctx, BC_ERR_NOT_INCIDENT, "edge does not touch the updated vertex");
        const int32_t x = (a == v) ? b : a;
        const std::pair<int32_t, int32_t> key = g->directed ? std::make_pair(a, b) : std::make_pair(std::min(a, b), std::max(a, b));
        if (seen.count(key)) return fail(ctx, BC_ERR_DUPLICATE_EDGE, "edge repeated in one vertex update");
        seen[key] = 1;
        const int32_t w = (int32_t)e[i].w;
        if (g->directed) {
            const int64_t cw = current_weight(g, p, a, b);
            if (cw >= 0 && w >= cw) return fail(ctx, BC_ERR_NOT_INCREMENTAL, "new weight is not below the current one");
            if (b == v) ein.push_back({a, w});
            else eout.push_back({b, w});
            changes.push_back({{a, b}, w});
        } else {
            const int64_t cw = current_weight(g, p, x, v);
            if (cw >= 0 && w >= cw) return fail(ctx, BC_ERR_NOT_INCREMENTAL, "new weight is not below the current one");
            ein.push_back({x, w});
            eout.push_back({x, w});
            changes.push_back({{x, v}, w});
            changes.push_back({{v, x}, w});
        }
    }
    int64_t ins = 0;
    for (auto &c : changes)
        if (current_weight(g, p, c.first.first, c.first.second) < 0) ++ins;
    if (g->mirror.arcs + p.inserted + ins > g->arc_cap) return fail(ctx, BC_ERR_CAPACITY, "arc capacity exceeded");
    for (auto &c : changes) p.arcs[c.first] = c.second;
    p.inserted += ins;
    if (k > 0) build_jobs(g, v, ein, eout, jobs);
    return BC_OK;
}

// For a directed arc (u,v): the vertex form at v with E_i = {(u,v)}.  For an
// undirected edge {u,v}: the vertex form at u with E_i = {(v,u)} and
// E_o = {(u,v)}, equivalent to the two arc updates of G_D in sequence.
bc_status validate_edge(bc_ctx *ctx, GraphRec *g, int32_t u, int32_t v, int64_t w, Pending &p,
                        std::vector<UpdateJob> &jobs) {
    bc_status st = check_edge_arg(ctx, g, u, v, w);
    if (st) return st;
    bc_edge e{u, v, w};
    return validate_vertex(ctx, g, g->directed ? v : u, 1, &e, p, jobs);
}

void apply_pending(GraphRec *g, const Pending &p) {
    for (auto &kv : p.arcs) g->mirror.set(kv.first.first, kv.first.second, kv.second);
}

bc_status read_status(bc_ctx *ctx, GraphRec *g, int32_t *status) {
    HIPCHK(hipMemcpyAsync(status, &g->P.ctl->status, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return BC_OK;
}

bc_status sticky_to_status(int32_t st) {
    if (st & ST_SIGMA_OVF) return BC_ERR_SIGMA_OVERFLOW;
    if (st & ST_DIST_OVF) return BC_ERR_DIST_OVERFLOW;
    if (st & ST_ESTAR_CAP) return BC_ERR_ESTAR_CAPACITY;
    if (st & ST_CHECK) return BC_ERR_CHECK_FAILED;
    return BC_OK;
}

// Bitwise or of the sticky status words at the given device addresses:
// gathered by k_gather_status into the stream's staging area and copied into
// pinned host memory, one wait per STATUS_BATCH words.  clock: on the clock
// stream (polling results beside the work), else on the library stream
// (behind the work).
bc_status read_status(bc_ctx *ctx, const std::vector<const int32_t *> &words, bool clock, int32_t *acc) {
    hipStream_t st = clock ? ctx->clock_stream : ctx->stream;
    int32_t *dev = status_dev(ctx, clock);
    *acc = 0;
    for (size_t b = 0; b < words.size(); b += STATUS_BATCH) {
        const size_t e = std::min(words.size(), b + (size_t)STATUS_BATCH);
        for (size_t c = b; c < e; c += STATUS_GATHER) {
            StatusPtrs a{};
            const int cnt = (int)std::min<size_t>(STATUS_GATHER, e - c);
            for (int k = 0; k < cnt; ++k) a.p[k] = words[c + k];
            hipLaunchKernelGGL(k_gather_status, dim3(1), dim3(STATUS_GATHER), 0, st, a, cnt, dev + (c - b));
        }
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(ctx->h_status, dev, 4 * (e - b), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        for (size_t k = 0; k < e - b; ++k) *acc |= ctx->h_status[k];
    }
    return BC_OK;
}

// The maintained E* as an arc list grouped by tail (heads ascending within a
// tail), read from its by-head copy XC.  Refuses a graph with a sticky error:
// its E* may be incomplete then.
bc_status estar_by_tail(bc_ctx *ctx, GraphRec *g, std::vector<int32_t> &hp, std::vector<int32_t> &hd,
                        std::vector<int32_t> &hw) {
    const int32_t n = g->n;
    int32_t status = 0;
    bc_status st = read_status(ctx, g, &status);
    if (st) return st;
    if (status) return fail(ctx, sticky_to_status(status), "the graph carries a sticky error: use bc_recompute");
    int32_t m = 0;
    HIPCHK(hipMemcpyAsync(&m, &g->P.ctl->esc_m, 4, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    std::vector<int32_t> a((size_t)m), b((size_t)m), w((size_t)m);
    if (m) {
        HIPCHK(hipMemcpyAsync(a.data(), g->P.xc_src, 4 * (size_t)m, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipMemcpyAsync(b.data(), g->P.xc_dst, 4 * (size_t)m, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipMemcpyAsync(w.data(), g->P.xc_w, 4 * (size_t)m, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
    }
    // counting sort by tail; XC is grouped by ascending head, so heads stay
    // ascending within each tail
    hp.assign(n + 1, 0);
    for (int32_t e = 0; e < m; ++e) hp[a[e] + 1]++;
    for (int32_t i = 0; i < n; ++i) hp[i + 1] += hp[i];
    hd.resize((size_t)m);
    hw.resize((size_t)m);
    std::vector<int32_t> fill(hp.begin(), hp.end() - 1);
    for (int32_t e = 0; e < m; ++e) {
        const int32_t q = fill[a[e]]++;
        hd[q] = b[e];
        hw[q] = w[e];
    }
    return BC_OK;
}

// An arc set by tail (heads ascending within a tail).
struct ArcCsr {
    std::vector<int32_t> ptr, dst, w;
    int64_t size() const { return (int64_t)dst.size(); }
};

// The same arcs grouped by head (counting sort; tails stay ascending).
void by_head(int32_t n, const ArcCsr &t, ArcCsr &h) {
    const int64_t m = t.size();
    h.ptr.assign(n + 1, 0);
    h.dst.resize((size_t)m);
    h.w.resize((size_t)m);
    for (int64_t e = 0; e < m; ++e) h.ptr[t.dst[e] + 1]++;
    for (int32_t i = 0; i < n; ++i) h.ptr[i + 1] += h.ptr[i];
    std::vector<int32_t> fill(h.ptr.begin(), h.ptr.end() - 1);
    for (int32_t a = 0; a < n; ++a)
        for (int32_t e = t.ptr[a]; e < t.ptr[a + 1]; ++e) {
            const int32_t q = fill[t.dst[e]]++;
            h.dst[q] = a;
            h.w[q] = t.w[e];
        }
}

bc_status upload_csr(bc_ctx *ctx, int32_t n, const ArcCsr &c, int32_t *ptr, int32_t *other, int32_t *w) {
    HIPCHK(hipMemcpyAsync(ptr, c.ptr.data(), 4 * (size_t)(n + 1), hipMemcpyHostToDevice, ctx->stream));
    if (c.size()) {
        HIPCHK(hipMemcpyAsync(other, c.dst.data(), 4 * (size_t)c.size(), hipMemcpyHostToDevice, ctx->stream));
        HIPCHK(hipMemcpyAsync(w, c.w.data(), 4 * (size_t)c.size(), hipMemcpyHostToDevice, ctx->stream));
    }
    return BC_OK;
}

// The k lightest out-arcs of every vertex (all of them where there are at
// most k), heads ascending.
void lightest_arcs(int32_t n, const ArcCsr &full, int32_t k, ArcCsr &out) {
    out.ptr.assign(n + 1, 0);
    out.dst.clear();
    out.w.clear();
    std::vector<std::pair<int32_t, int32_t>> row;  // (w, head)
    for (int32_t a = 0; a < n; ++a) {
        row.clear();
        for (int32_t e = full.ptr[a]; e < full.ptr[a + 1]; ++e) row.push_back({full.w[e], full.dst[e]});
        if ((int32_t)row.size() > k) {
            std::nth_element(row.begin(), row.begin() + k, row.end());
            row.resize(k);
        }
        std::sort(row.begin(), row.end(), [](const std::pair<int32_t, int32_t> &x, const std::pair<int32_t, int32_t> &y) {
            return x.second < y.second;
        });
        for (auto &p : row) {
            out.dst.push_back(p.second);
            out.w.push_back(p.first);
        }
        out.ptr[a + 1] = (int32_t)out.dst.size();
    }
}

// Adds the listed arcs that the set lacks; returns how many were new.
int64_t add_missing(int32_t n, ArcCsr &set, const std::vector<int32_t> &a, const std::vector<int32_t> &b,
                    const std::vector<int32_t> &w) {
    std::vector<std::vector<std::pair<int32_t, int32_t>>> extra;
    int64_t added = 0;
    for (size_t i = 0; i < a.size(); ++i) {
        auto first = set.dst.begin() + set.ptr[a[i]], last = set.dst.begin() + set.ptr[a[i] + 1];
        if (std::binary_search(first, last, b[i])) continue;
        if (extra.empty()) extra.resize(n);
        extra[a[i]].push_back({b[i], w[i]});
        ++added;
    }
    if (!added) return 0;
    ArcCsr out;
    out.ptr.assign(n + 1, 0);
    std::vector<std::pair<int32_t, int32_t>> row;
    for (int32_t t = 0; t < n; ++t) {
        row.clear();
        for (int32_t e = set.ptr[t]; e < set.ptr[t + 1]; ++e) row.push_back({set.dst[e], set.w[e]});
        row.insert(row.end(), extra[t].begin(), extra[t].end());
        std::sort(row.begin(), row.end());
        for (auto &p : row) {
            out.dst.push_back(p.first);
            out.w.push_back(p.second);
        }
        out.ptr[t + 1] = (int32_t)out.dst.size();
    }
    set = std::move(out);
    return added;
}

// Out-arcs per vertex in the first searched set of a checked search, and
// the density from which the check pays (the set is at most a quarter of
// the arcs).
int32_t search_k(int32_t n) { return (int32_t)std::ceil(2.0 * std::log((double)std::max(n, 2))) + 4; }
bool use_checked_search(int32_t n, int64_t m) { return m >= 4 * (int64_t)search_k(n) * n; }

// Static pass: all-pairs distances, path counts, E* and BC from scratch
// (Alg 7 with the DAG taken from E*, Alg 6 steps 2-8).
//
const char *check_kind_name(int32_t k) {
    switch (k) {
        case CK_SOURCE: return "source entry";
        case CK_RELAX: return "shorter in-arc";
        case CK_NO_PATH: return "no tight in-arc";
        case CK_SIGMA: return "path count";
        case CK_PRED: return "stored predecessor";
        case CK_UNREACHED: return "unreachable pair";
        case CK_SYMMETRY: return "symmetry";
        case CK_ESTAR: return "E*";
        default: return "unknown";
    }
}

// State check (bc_check, BC_FLAG_CHECK) over the given arcs, which must be
// the arcs of the state on the device: they go by head into arcin_* (no
// update reads those), then the check kernels run on every source (all) or
// on the last update's affected ones, and on E*.  Synchronises.  Returns
// BC_ERR_CHECK_FAILED, with the first failure in the message, when a check
// fails; *status gets the graph's sticky bits (a graph that had some before
// is not checked).
bc_status run_check(bc_ctx *ctx, GraphRec *g, const Mirror &arcs, bool all, int32_t *status) {
    const int32_t n = g->n;
    Mirror m = arcs;
    m.compact();
    ArcCsr tail, head;
    tail.ptr.resize((size_t)n + 1);
    for (int32_t i = 0; i <= n; ++i) tail.ptr[i] = (int32_t)m.ptr[i];
    tail.dst = std::move(m.dst);
    tail.w = std::move(m.w);
    if (tail.size() > g->arc_cap) return fail(ctx, BC_ERR_CAPACITY, "arc capacity exceeded");
    by_head(n, tail, head);
    bc_status st = upload_csr(ctx, n, head, g->P.arcin_ptr, g->P.arcin_src, g->P.arcin_w);
    if (st) return st;
    hipLaunchKernelGGL(k_check_rows, dim3(2048), dim3(256), 0, ctx->stream, g->P, g->chk, all ? 1 : 0);
    hipLaunchKernelGGL(k_check_estar, dim3((int)std::min<int64_t>(((int64_t)n + 255) / 256, 1024)), dim3(256), 0,
                       ctx->stream, g->P, g->chk);
    HIPCHK(hipGetLastError());
    CheckRec rec{};
    *status = 0;
    HIPCHK(hipMemcpyAsync(&rec, g->chk, sizeof rec, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipMemcpyAsync(status, &g->P.ctl->status, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream));
    // the host arrays above are read by the copies: finish before they go
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (*status & ST_CHECK) {
        char msg[160];
        snprintf(msg, sizeof msg, "state check failed: %s at (%d, %d), %llu condition(s) false", check_kind_name(rec.kind),
                 rec.s, rec.t, rec.fails);
        return fail(ctx, BC_ERR_CHECK_FAILED, msg);
    }
    return BC_OK;
}

// Applies a step's arc changes to the check copies of its graphs' arcs, then
// checks each graph (BC_FLAG_CHECK).
bc_status check_step(bc_ctx *ctx, const std::vector<UpdateJob> &jobs) {
    for (const UpdateJob &j : jobs) {
        GraphRec *g = nullptr;
        for (GraphRec *r : ctx->graphs)
            if (r && r->live && r->P.ctl == j.g.ctl) g = r;
        if (!g) continue;
        for (int32_t k = 0; k < j.n_u; ++k) g->dev.set(j.u_tail[k], j.u_head[k], j.u_w[k]);
        int32_t status = 0;
        const bc_status st = run_check(ctx, g, g->dev, false, &status);
        if (st) return st;
    }
    return BC_OK;
}

// Static pass on the GPU from the mirror's arcs: distances, E*, counts,
// dependencies and BC (Alg 7 with the DAG taken from E*, Alg 6 steps 2-8).
// The distance search relaxes a set of arcs that contains E*; every
// shortest path lies in E* and any such set gives the same distances, DAGs,
// counts and BC (Section 6):
//   over_estar: the maintained E* (a graph without sticky errors);
//   a dense graph (checked search): the k lightest out-arcs of every vertex
//     first; then one pass over all arcs lists those with w(a,b) <= d_H(a,b)
//     for the distances d_H of the searched set H; the listed arcs H lacks
//     join it and the search runs again, until none is missing, when d_H is
//     the distance matrix and H contains E* (see k_search_check).  On
//     complete graphs with random weights E* has about n ln n arcs
//     (Section 1), so H stays a small fraction of the n^2 arcs;
//   otherwise (sparse graphs, or BC_FLAG_FULL_SEARCH): every arc.
bc_status static_pass(bc_ctx *ctx, GraphRec *g, bool over_estar = false) {
    const int32_t n = g->n;
    ArcCsr full;
    if (over_estar) {
        bc_status st = estar_by_tail(ctx, g, full.ptr, full.dst, full.w);
        if (st) return st;
    } else {
        g->mirror.compact();
        full.ptr.resize(n + 1);
        full.dst = g->mirror.dst;
        full.w = g->mirror.w;
        for (int32_t i = 0; i <= n; ++i) full.ptr[i] = (int32_t)g->mirror.ptr[i];
    }
    const int64_t m = full.size();
    if (m > g->arc_cap) return fail(ctx, BC_ERR_CAPACITY, "arc capacity exceeded");
    const bool checked = !over_estar && !ctx->full_search && use_checked_search(n, m);
    HIPCHK(hipMemsetAsync(g->P.ctl, 0, sizeof(GraphCtl), ctx->stream));
    HIPCHK(hipMemsetAsync(g->chk, 0, sizeof(CheckRec), ctx->stream));
    HIPCHK(hipMemsetAsync(g->P.bc_delta, 0, 8 * (size_t)n, ctx->stream));
    std::vector<UpdateJob> jobs(1, job_template(g));
    LaunchShape L;
    bc_status st = shape_for(ctx, jobs, &L);
    if (st) return st;
    int r;
    if ((st = ring_acquire(ctx, &r))) return st;
    if ((st = ring_stage(ctx, r, jobs))) return st;
    const UpdateJob *dj = ring_jobs_dev(ctx, r);
    const int32_t *nj = ring_njobs_dev(ctx, r);
    const int slots = std::min<int>(L.slots, n);
    // slots may still hold another layout's lists (n_layout can just have grown)
    const ScratchPlan sp = plan_scratch(ctx, ctx->n_layout);
    const size_t slot_region = (size_t)sp.src * sp.src_bytes + (size_t)sp.wide * sp.wide_bytes;
    HIPCHK(hipMemsetAsync(sp.src_base, 0, slot_region, ctx->stream));
    const int g_wave = (int)std::min<int64_t>(((int64_t)n * 64 + 255) / 256, 4096);
    hipStream_t s = ctx->stream;
    // the search stages the row in LDS when it fits beside its expansion
    // arrays (for n up to about 34 800), else works on the row in place
    const int32_t sssp_cap = source_lds_bytes(L.lds_cap, 1024, 0) <= ctx->sssp_lds_limit ? L.lds_cap : 0;
    ArcCsr search;  // the arcs the distance search relaxes
    bool have_dist = false;
    int32_t rounds = 0;
    if (checked) {
        // every arc by tail stays in arc_* for the check; the searched set
        // goes by tail into the by-head arrays, unused until the E* build
        if ((st = upload_csr(ctx, n, full, g->P.arc_ptr, g->P.arc_dst, g->P.arc_w))) return st;
        lightest_arcs(n, full, search_k(n), search);
        unsigned long long *cnt = (unsigned long long *)misc_dev(ctx);
        std::vector<int32_t> ca, cb, cw;
        for (;;) {
            ++rounds;
            if ((st = upload_csr(ctx, n, search, g->P.arcin_ptr, g->P.arcin_src, g->P.arcin_w))) return st;
            hipLaunchKernelGGL(k_reset_work, dim3(1), dim3(1), 0, s, g->P.ctl);
            hipLaunchKernelGGL(k_sssp, dim3(slots), dim3(1024), source_lds_bytes(sssp_cap, 1024, 0), s, dj,
                               L.src_base, L.slot_bytes, sssp_cap, L.n_layout, g->P.arcin_ptr, g->P.arcin_src,
                               g->P.arcin_w);
            HIPCHK(hipMemsetAsync(cnt, 0, 8, s));
            hipLaunchKernelGGL(k_search_check, dim3(std::max(1, std::min(g_wave, 4096))), dim3(256), 0, s, dj,
                               g->P.yc_src, g->P.yc_dst, g->P.yc_w, g->es_cap, cnt);
            HIPCHK(hipGetLastError());
            unsigned long long c = 0;
            int32_t status = 0;
            HIPCHK(hipMemcpyAsync(&c, cnt, 8, hipMemcpyDeviceToHost, s));
            HIPCHK(hipMemcpyAsync(&status, &g->P.ctl->status, 4, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            if (status) {
                have_dist = true;  // the sticky error is reported below
                break;
            }
            if ((int64_t)c > g->es_cap) {
                // more candidate arcs than E* may hold: search every arc
                search = full;
                break;
            }
            ca.resize((size_t)c);
            cb.resize((size_t)c);
            cw.resize((size_t)c);
            if (c) {
                HIPCHK(hipMemcpyAsync(ca.data(), g->P.yc_src, 4 * (size_t)c, hipMemcpyDeviceToHost, s));
                HIPCHK(hipMemcpyAsync(cb.data(), g->P.yc_dst, 4 * (size_t)c, hipMemcpyDeviceToHost, s));
                HIPCHK(hipMemcpyAsync(cw.data(), g->P.yc_w, 4 * (size_t)c, hipMemcpyDeviceToHost, s));
                HIPCHK(hipStreamSynchronize(s));
            }
            if (add_missing(n, search, ca, cb, cw) == 0) {
                have_dist = true;
                break;
            }
        }
    } else {
        search = std::move(full);
    }
    g->search_arcs = search.size();
    g->search_rounds = rounds;
    // the final arc set, by tail and by head, for the E* build
    ArcCsr head;
    by_head(n, search, head);
    if ((st = upload_csr(ctx, n, search, g->P.arc_ptr, g->P.arc_dst, g->P.arc_w))) return st;
    if ((st = upload_csr(ctx, n, head, g->P.arcin_ptr, g->P.arcin_src, g->P.arcin_w))) return st;
    g->P.arc_m = search.size();
    if (!have_dist) {
        hipLaunchKernelGGL(k_reset_work, dim3(1), dim3(1), 0, s, g->P.ctl);
        hipLaunchKernelGGL(k_sssp, dim3(slots), dim3(1024), source_lds_bytes(sssp_cap, 1024, 0), s, dj, L.src_base,
                           L.slot_bytes, sssp_cap, L.n_layout, g->P.arc_ptr, g->P.arc_dst, g->P.arc_w);
    }
    hipLaunchKernelGGL(k_es_count<ES_BUILD>, dim3(g_wave), dim3(256), 0, s, dj, nj);
    hipLaunchKernelGGL(k_es_scan<ES_BUILD>, dim3(1), dim3(1024), 0, s, dj, nj);
    hipLaunchKernelGGL(k_es_scatter<ES_BUILD>, dim3(g_wave), dim3(256), 0, s, dj, nj);
    hipLaunchKernelGGL(k_es_count<ES_BUILD_C>, dim3(g_wave), dim3(256), 0, s, dj, nj);
    hipLaunchKernelGGL(k_es_scan<ES_BUILD_C>, dim3(1), dim3(1024), 0, s, dj, nj);
    hipLaunchKernelGGL(k_es_scatter<ES_BUILD_C>, dim3(g_wave), dim3(256), 0, s, dj, nj);
    hipLaunchKernelGGL(k_reset_work, dim3(1), dim3(1), 0, s, g->P.ctl);
    hipLaunchKernelGGL(k_static, dim3(slots), dim3(1024), (size_t)L.lds_cap * 4, s, dj, L.src_base, L.slot_bytes,
                       L.lds_cap, L.n_layout);
    hipLaunchKernelGGL(k_commit, dim3((n + 255) / 256 < 2048 ? (n + 255) / 256 : 2048), dim3(256), 0, s, dj, nj, 1);
    HIPCHK(hipGetLastError());
    // the update kernels expect their per-workgroup flags and sums at zero
    HIPCHK(hipMemsetAsync(sp.src_base, 0, slot_region, s));
    st = ring_release(ctx, r);
    if (st) return st;
    // the host vectors above are read by the copies: finish before they go
    HIPCHK(hipStreamSynchronize(ctx->stream));
    int32_t status = 0;
    if ((st = read_status(ctx, g, &status))) return st;
    if (status) return fail(ctx, sticky_to_status(status), "static pass failed");
    if (ctx->check) {
        g->dev = g->mirror;
        return run_check(ctx, g, g->dev, true, &status);
    }
    return BC_OK;
}

bc_status set_lds_limit(bc_ctx *ctx, const void *fn, size_t *limit = nullptr) {
    hipFuncAttributes attr;
    HIPCHK(hipFuncGetAttributes(&attr, fn));
    // all of a gfx950 workgroup's 160 KiB of LDS, less what the kernel declares statically
    const int bytes = 160 * 1024 - (int)attr.sharedSizeBytes;
    HIPCHK(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
    if (limit) *limit = (size_t)bytes;
    return BC_OK;
}

// Resolves this device's address of the fixed scratch array, once per
// device (the context's device is current), and zeroes the array then: the
// dependency pass run in it keeps its counters at zero after every use.
bc_status fixed_scratch_setup(bc_ctx *ctx) {
    if (ctx->device < 0 || ctx->device >= FIXED_MAX_DEVICES)
        return fail(ctx, BC_ERR_NO_DEVICE, "device ordinal above the fixed scratch table");
    std::lock_guard<std::mutex> lock(fixed_mu);
    if (!fixed_addr[ctx->device]) {
        void *p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(bc_fixed_scratch)));
        if (!p) return fail(ctx, BC_ERR_HIP, "hipGetSymbolAddress returned no address");
        hipLaunchKernelGGL(k_zero_fill, dim3(256), dim3(256), 0, ctx->stream, (char *)p, FIXED_SCRATCH_BYTES);
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(ctx->stream));
        fixed_addr[ctx->device] = p;
    }
    ctx->fixed_scratch = (char *)fixed_addr[ctx->device];
    return BC_OK;
}

bc_status set_lds_limits(bc_ctx *ctx) {
    bc_status st;
    if ((st = set_lds_limit(ctx, (const void *)k_source<256>))) return st;
    if ((st = set_lds_limit(ctx, (const void *)k_source<128>))) return st;
    if ((st = set_lds_limit(ctx, (const void *)k_source_wide, &ctx->wide_lds_limit))) return st;
    if ((st = set_lds_limit(ctx, (const void *)k_sssp, &ctx->sssp_lds_limit))) return st;
    if ((st = set_lds_limit(ctx, (const void *)k_static))) return st;
    if ((st = set_lds_limit(ctx, (const void *)k_delta_row_byval))) return st;
    return set_lds_limit(ctx, (const void *)k_delta_row);
}

}  // namespace

namespace {

bool schedule_valid(const bc_ctx *ctx, const bc_schedule &s) {
    return !(s.block < 64 || s.block > 256 || s.block % 64 != 0 || s.slots < 0 || s.slots > ctx->slots || s.big_b < 1 ||
             s.big_b > LCAP || (s.wide_block != 256 && s.wide_block != 512 && s.wide_block != 1024) ||
             (s.table != 128 && s.table != 256) || (s.wide_stage != 1 && s.wide_stage != 2) || s.wide_slots < 0 ||
             s.wide_slots > ctx->slots);
}

// Tuning cache: a JSON object naming the device kind and listing one
// schedule per size bucket.  Written whole (to a temporary file, then
// renamed) after every tuning; read at bc_create.
bc_status write_tune_cache(bc_ctx *ctx) {
    if (ctx->tune_cache.empty()) return BC_OK;
    const std::string tmp = ctx->tune_cache + ".tmp";
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return fail(ctx, BC_ERR_INVALID_ARG, "cannot write the tuning cache " + tmp);
    fprintf(f, "{\"device\": \"%s\", \"schedules\": [", ctx->device_tag.c_str());
    bool first = true;
    for (auto &kv : ctx->tuned) {
        const bc_schedule &c = kv.second;
        fprintf(f,
                "%s\n  {\"n_bucket\": %d, \"block\": %d, \"slots\": %d, \"big_b\": %d, \"wide_block\": %d, "
                "\"wide_stage\": %d, \"wide_slots\": %d, \"table\": %d}",
                first ? "" : ",", kv.first, c.block, c.slots, c.big_b, c.wide_block, c.wide_stage, c.wide_slots,
                c.table);
        first = false;
    }
    fprintf(f, "\n]}\n");
    const bool ok = fclose(f) == 0;
    if (!ok || rename(tmp.c_str(), ctx->tune_cache.c_str()) != 0)
        return fail(ctx, BC_ERR_INVALID_ARG, "cannot write the tuning cache " + ctx->tune_cache);
    return BC_OK;
}

// Reads the integer after "key": inside [p, end); false when absent.
bool json_int(const char *p, const char *end, const char *key, int *out) {
    const std::string k = std::string("\"") + key + "\":";
    const std::string hay(p, end);
    const size_t at = hay.find(k);
    if (at == std::string::npos) return false;
    return sscanf(hay.c_str() + at + k.size(), " %d", out) == 1;
}

// Loads the cache's schedules when it names this device kind; entries out
// of range for this context are skipped.  A missing file is no error.
void read_tune_cache(bc_ctx *ctx) {
    if (ctx->tune_cache.empty()) return;
    FILE *f = fopen(ctx->tune_cache.c_str(), "r");
    if (!f) return;
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
    fclose(f);
    const std::string dev = "\"device\": \"" + ctx->device_tag + "\"";
    if (text.find(dev) == std::string::npos) return;
    size_t pos = text.find('[');
    while (pos != std::string::npos) {
        const size_t a = text.find('{', pos), b = text.find('}', a == std::string::npos ? pos : a);
        if (a == std::string::npos || b == std::string::npos) break;
        const char *p = text.c_str() + a, *e = text.c_str() + b;
        int bucket;
        bc_schedule c{};
        if (json_int(p, e, "n_bucket", &bucket) && json_int(p, e, "block", &c.block) && json_int(p, e, "slots", &c.slots) &&
            json_int(p, e, "big_b", &c.big_b) && json_int(p, e, "wide_block", &c.wide_block) &&
            json_int(p, e, "wide_stage", &c.wide_stage) && json_int(p, e, "wide_slots", &c.wide_slots) &&
            json_int(p, e, "table", &c.table) && schedule_valid(ctx, c))
            ctx->tuned[bucket] = c;
        pos = b + 1;
    }
    ctx->use_tuned = !ctx->tuned.empty();
}

}  // namespace

// ============================================================== C ABI ====

extern "C" {

uint64_t bc_graph_bytes(int32_t n, int64_t arc_capacity, int64_t estar_capacity) {
    if (n <= 0 || arc_capacity < 0) return 0;
    if (estar_capacity <= 0) estar_capacity = arc_capacity;
    size_t total = 0;
    carve(nullptr, n, std::max<int64_t>(arc_capacity, 1), std::max<int64_t>(estar_capacity, 1), &total);
    return total;
}

uint64_t bc_scratch_bytes(int32_t n_max, int32_t slots) {
    if (n_max <= 0) return 0;
    if (slots <= 0) slots = DEFAULT_SLOTS;
    return ring_bytes() + MISC_BYTES + pool_bytes(n_max) + (uint64_t)slots * slot_bytes_for(n_max) +
           (uint64_t)wide_slots_for(slots) * (wide_slot_bytes_for(n_max) + item_region_bytes(n_max));
}

const char *bc_status_string(bc_status s) {
    switch (s) {
        case BC_OK: return "ok";
        case BC_ERR_INVALID_ARG: return "invalid argument";
        case BC_ERR_SELF_LOOP: return "self-loop";
        case BC_ERR_BAD_WEIGHT: return "weight out of range";
        case BC_ERR_DUPLICATE_EDGE: return "duplicate edge";
        case BC_ERR_NOT_INCIDENT: return "edge not incident to the vertex";
        case BC_ERR_NOT_INCREMENTAL: return "update is not incremental";
        case BC_ERR_ADMISSION: return "memory budget exceeded";
        case BC_ERR_CAPACITY: return "capacity exceeded";
        case BC_ERR_SIGMA_OVERFLOW: return "path count overflow";
        case BC_ERR_DIST_OVERFLOW: return "distance overflow";
        case BC_ERR_HIP: return "HIP runtime error";
        case BC_ERR_NO_DEVICE: return "no gfx950 device";
        case BC_ERR_ESTAR_CAPACITY: return "E* capacity exceeded";
        case BC_ERR_CHECK_FAILED: return "state check failed";
        default: return "unknown status";
    }
}

const char *bc_last_error(bc_ctx *ctx) { return ctx ? ctx->last_error.c_str() : "no context"; }

bc_status bc_create(bc_ctx **out, const bc_config *cfg) {
    if (!out || !cfg) return BC_ERR_INVALID_ARG;
    *out = nullptr;
    int count = 0;
    hipError_t de = hipGetDeviceCount(&count);
    if (de != hipSuccess || cfg->device < 0 || cfg->device >= count) {
        fprintf(stderr, "bcinc: bc_create: device %d unavailable (%d devices, %s)\n", cfg->device, count,
                hipGetErrorString(de));
        return BC_ERR_NO_DEVICE;
    }
    hipDeviceProp_t prop;
    de = hipGetDeviceProperties(&prop, cfg->device);
    if (de != hipSuccess) {
        fprintf(stderr, "bcinc: bc_create: hipGetDeviceProperties: %s\n", hipGetErrorString(de));
        return BC_ERR_NO_DEVICE;
    }
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        fprintf(stderr, "bcinc: bc_create: device %d is %s, not gfx950\n", cfg->device, prop.gcnArchName);
        return BC_ERR_NO_DEVICE;
    }
    if (!cfg->scratch || cfg->scratch_bytes < ring_bytes() + MISC_BYTES) return BC_ERR_INVALID_ARG;
    if (((uintptr_t)cfg->scratch & 255) != 0) return BC_ERR_INVALID_ARG;
    bc_ctx *ctx = new bc_ctx();
    ctx->device = cfg->device;
    ctx->cu_count = prop.multiProcessorCount;
    ctx->scratch = (char *)cfg->scratch;
    ctx->scratch_bytes = cfg->scratch_bytes;
    ctx->budget = cfg->memory_budget;
    ctx->slots = cfg->slots > 0 ? cfg->slots : DEFAULT_SLOTS;
    ctx->block = cfg->block > 0 ? cfg->block : DEFAULT_BLOCK;
    if (ctx->block % 64 != 0 || ctx->block > 256) {
        delete ctx;
        return BC_ERR_INVALID_ARG;
    }
    auto bail = [&](hipError_t e, const char *what) {
        bc_status st = hip_fail(ctx, e, what);
        fprintf(stderr, "bcinc: %s\n", ctx->last_error.c_str());
        delete ctx;
        return st;
    };
    hipError_t e = hipSetDevice(cfg->device);
    if (e != hipSuccess) return bail(e, "hipSetDevice");
    if (cfg->stream) {
        ctx->stream = (hipStream_t)cfg->stream;
    } else {
        e = hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking);
        if (e != hipSuccess) return bail(e, "hipStreamCreate");
        ctx->own_stream = true;
    }
    e = hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking);
    if (e != hipSuccess) return bail(e, "hipStreamCreate");
    e = hipEventCreateWithFlags(&ctx->fork_ev, hipEventDisableTiming);
    if (e != hipSuccess) return bail(e, "hipEventCreate");
    e = hipEventCreateWithFlags(&ctx->join_ev, hipEventDisableTiming);
    if (e != hipSuccess) return bail(e, "hipEventCreate");
    e = hipStreamCreateWithFlags(&ctx->clock_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return bail(e, "hipStreamCreate");
    e = hipEventCreate(&ctx->clock_ev);
    if (e != hipSuccess) return bail(e, "hipEventCreate");
    e = hipHostMalloc((void **)&ctx->h_status, 4 * STATUS_BATCH, hipHostMallocDefault);
    if (e != hipSuccess) return bail(e, "hipHostMalloc");
    for (int r = 0; r < RING; ++r) {
        e = hipHostMalloc((void **)&ctx->h_ring[r], ring_slot_bytes(), hipHostMallocDefault);
        if (e != hipSuccess) return bail(e, "hipHostMalloc");
        ctx->h_njobs[r] = (int32_t *)ctx->h_ring[r];
        ctx->h_jobs[r] = (UpdateJob *)(ctx->h_ring[r] + 256);
        e = hipEventCreateWithFlags(&ctx->ring_ev[r], hipEventDisableTiming);
        if (e != hipSuccess) return bail(e, "hipEventCreate");
        for (int q = 0; q < 5; ++q) {
            e = hipEventCreate(&ctx->tev[r][q]);
            if (e != hipSuccess) return bail(e, "hipEventCreate");
        }
    }
    ctx->device_tag = std::string(prop.gcnArchName) + "/" + std::to_string(prop.multiProcessorCount) + "cu";
    if (cfg->tune_cache) ctx->tune_cache = cfg->tune_cache;
    read_tune_cache(ctx);
    ctx->timing = (cfg->flags & BC_FLAG_TIMING) != 0;
    ctx->full_search = (cfg->flags & BC_FLAG_FULL_SEARCH) != 0;
    ctx->check = (cfg->flags & BC_FLAG_CHECK) != 0;
    {
        // the row kernel is persistent: as many workgroups as stay resident
        int per_cu = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_rows, 256, 0);
        if (e != hipSuccess) return bail(e, "hipOccupancyMaxActiveBlocksPerMultiprocessor");
        ctx->rows_grid = std::max(1, per_cu) * ctx->cu_count;
    }
    if (set_lds_limits(ctx) != BC_OK) {
        fprintf(stderr, "bcinc: %s\n", ctx->last_error.c_str());
        delete ctx;
        return BC_ERR_HIP;
    }
    e = hipMemsetAsync(ctx->scratch, 0, ctx->scratch_bytes, ctx->stream);
    if (e != hipSuccess) return bail(e, "hipMemsetAsync");
    e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return bail(e, "hipStreamSynchronize");
    if (fixed_scratch_setup(ctx) != BC_OK || calibrate_clock(ctx) != BC_OK) {
        fprintf(stderr, "bcinc: %s\n", ctx->last_error.c_str());
        delete ctx;
        return BC_ERR_HIP;
    }
    *out = ctx;
    return BC_OK;
}

bc_status bc_set_schedule(bc_ctx *ctx, const bc_schedule *s) {
    if (!ctx || !s) return BC_ERR_INVALID_ARG;
    const int block = s->block ? s->block : ctx->block;
    const int slots = s->slots ? s->slots : ctx->run_slots;
    const int big_b = s->big_b ? s->big_b : ctx->big_b;
    const int wide_block = s->wide_block ? s->wide_block : ctx->wide_block;
    const int wide_stage = s->wide_stage ? s->wide_stage : ctx->wide_stage;
    const int wide_slots = s->wide_slots ? s->wide_slots : ctx->wide_slots;
    const int table = s->table ? s->table : ctx->table;
    const bc_schedule want{block, slots, big_b, wide_block, wide_stage, wide_slots, table};
    if (!schedule_valid(ctx, want)) return fail(ctx, BC_ERR_INVALID_ARG, "schedule value out of range");
    HIPCHK(hipSetDevice(ctx->device));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    // captured step graphs hold the old launch shapes
    for (auto &kv : ctx->graph_cache) {
        if (kv.second.exec) HIPCHK(hipGraphExecDestroy(kv.second.exec));
        if (kv.second.graph) HIPCHK(hipGraphDestroy(kv.second.graph));
    }
    ctx->graph_cache.clear();
    ctx->block = block;
    ctx->run_slots = slots;
    ctx->big_b = big_b;
    ctx->wide_block = wide_block;
    ctx->wide_stage = wide_stage;
    ctx->wide_slots = wide_slots;
    ctx->table = table;
    ctx->use_tuned = false;  // this schedule serves every step until the next tuning
    return BC_OK;
}

// Schedule autotuner.  Every candidate runs the caller's sample twice on
// fresh device clones of the sampled graphs (the first run also captures the
// candidate's step graphs); the second run's summed step time (HIP events
// around each step's kernels) ranks it.  Clones are dropped afterwards, so
// the resident graphs never see the sample.
bc_status bc_autotune(bc_ctx *ctx, int32_t cnt, const bc_request *reqs, void *workspace, uint64_t workspace_bytes,
                      bc_schedule *chosen) {
    if (!ctx || cnt <= 0 || !reqs || !workspace) return fail(ctx, BC_ERR_INVALID_ARG, "bad arguments to bc_autotune");
    if (((uintptr_t)workspace & 255) != 0) return fail(ctx, BC_ERR_INVALID_ARG, "workspace not 256-byte aligned");
    {
        const bc_status fq = flush_queues(ctx);
        if (fq) return fq;
    }
    std::vector<int32_t> gids;
    uint64_t need = 0;
    for (int32_t i = 0; i < cnt; ++i) {
        GraphRec *g = get_graph(ctx, reqs[i].graph);
        if (!g) return fail(ctx, BC_ERR_INVALID_ARG, "sample names no resident graph");
        if (std::find(gids.begin(), gids.end(), reqs[i].graph) == gids.end()) {
            gids.push_back(reqs[i].graph);
            need += align256(bc_graph_bytes(g->n, g->arc_cap, g->es_cap));
        }
    }
    if (workspace_bytes < need) return fail(ctx, BC_ERR_CAPACITY, "autotune workspace below the sampled graphs' bytes");
    bc_schedule start;
    bc_get_schedule(ctx, &start);
    // a step takes the schedule of its largest graph's size bucket, so
    // bucket B is tuned on steps like the ones it serves: the sample's
    // requests on graphs of bucket B and below, in sample order (a bucket
    // with a schedule from the cache or an earlier tuning is not tuned again)
    std::set<int> sampled;
    for (int32_t i = 0; i < cnt; ++i) sampled.insert(n_bucket(ctx->graphs[reqs[i].graph]->n));
    std::map<int, std::vector<bc_request>> by_bucket;
    for (const int b : sampled)
        for (int32_t i = 0; i < cnt; ++i)
            if (n_bucket(ctx->graphs[reqs[i].graph]->n) <= b) by_bucket[b].push_back(reqs[i]);
    const bool timing0 = ctx->timing;
    bc_status st = BC_OK;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if ((st = harvest_all(ctx))) return st;
    const double step0 = ctx->step_ms, src0 = ctx->source_ms, rows0 = ctx->rows_ms;
    const int64_t steps0 = ctx->timed_steps;
    const uint64_t budget0 = ctx->budget;
    ctx->budget = 0;  // the clones live in the caller's workspace, outside the admission budget
    // one run of a bucket's sample on fresh clones; returns the summed step time
    auto run = [&](const std::vector<bc_request> &sub, double *ms) -> bc_status {
        std::vector<int32_t> sg;
        for (auto &r : sub)
            if (std::find(sg.begin(), sg.end(), r.graph) == sg.end()) sg.push_back(r.graph);
        const size_t base_id = ctx->graphs.size();
        char *p = (char *)workspace;
        bc_status s2 = BC_OK;
        for (size_t k = 0; k < sg.size() && !s2; ++k) {
            GraphRec *g = ctx->graphs[sg[k]];
            const uint64_t b = align256(bc_graph_bytes(g->n, g->arc_cap, g->es_cap));
            bc_graph_id c;
            s2 = bc_clone_graph(ctx, sg[k], p, b, &c);
            p += b;
        }
        if (!s2) {
            std::vector<bc_request> mapped(sub);
            for (auto &r : mapped)
                r.graph = (bc_graph_id)(base_id + (std::find(sg.begin(), sg.end(), r.graph) - sg.begin()));
            ctx->step_ms = 0;
            uint64_t ticket = 0;
            s2 = bc_submit(ctx, (int32_t)mapped.size(), mapped.data(), &ticket, nullptr);
            if (!s2) s2 = bc_wait(ctx, ticket);
            if (!s2 && hipStreamSynchronize(ctx->stream) != hipSuccess) s2 = fail(ctx, BC_ERR_HIP, "autotune run");
            if (!s2) s2 = harvest_all(ctx);
            *ms = ctx->step_ms;
            for (size_t k = 0; k < sg.size() && !s2; ++k) {
                int32_t status = 0;
                s2 = read_status(ctx, ctx->graphs[base_id + k], &status);
                if (!s2 && status) s2 = fail(ctx, sticky_to_status(status), "sample failed on a clone");
            }
        }
        (void)hipStreamSynchronize(ctx->stream);
        while (ctx->graphs.size() > base_id) {
            GraphRec *g = ctx->graphs.back();
            if (g->live) ctx->in_use -= g->arena_bytes;
            delete g;
            ctx->graphs.pop_back();
        }
        return s2;
    };
    ctx->timing = true;
    bool tuned_any = false;
    for (auto &kv : by_bucket) {
        if (st) break;
        if (ctx->tuned.count(kv.first)) continue;  // reused (cache or earlier tuning)
        bc_schedule best = start;
        double best_ms = 1e300;
        // candidates: LDS table size, workgroup size of the DAG kernel (64 is
        // one wave per source, no workgroup barriers), wide-kernel workgroup
        // size and the deferral threshold
        for (int table : {256, 128})
            for (int block : {256, 128, 64})
                for (int wide_block : {512, 1024})
                    for (int big_b : {512, 1024}) {
                        if (st) break;
                        bc_schedule c = start;
                        c.block = block;
                        c.wide_block = wide_block;
                        c.big_b = big_b;
                        c.table = table;
                        if ((st = bc_set_schedule(ctx, &c))) break;
                        double ms = 0;
                        if ((st = run(kv.second, &ms))) break;
                        if ((st = run(kv.second, &ms))) break;
                        if (ms < best_ms) {
                            best_ms = ms;
                            best = c;
                        }
                    }
        if (!st) {
            ctx->tuned[kv.first] = best;
            tuned_any = true;
        }
    }
    ctx->timing = timing0;
    ctx->step_ms = step0;
    ctx->source_ms = src0;
    ctx->rows_ms = rows0;
    ctx->timed_steps = steps0;
    ctx->budget = budget0;
    // the context's schedule becomes the largest sampled bucket's, and
    // every step takes its own bucket's while one is known
    const bc_schedule pick = st ? start : ctx->tuned[by_bucket.rbegin()->first];
    bc_status st2 = bc_set_schedule(ctx, &pick);
    if (st) return st;
    if (st2) return st2;
    ctx->use_tuned = true;
    if (tuned_any && (st = write_tune_cache(ctx))) return st;
    if (chosen) *chosen = pick;
    return BC_OK;
}

bc_status bc_get_schedule(bc_ctx *ctx, bc_schedule *out) {
    if (!ctx || !out) return BC_ERR_INVALID_ARG;
    out->block = ctx->block;
    out->slots = ctx->run_slots;
    out->big_b = ctx->big_b;
    out->wide_block = ctx->wide_block;
    out->wide_stage = ctx->wide_stage;
    out->wide_slots = ctx->wide_slots;
    out->table = ctx->table;
    return BC_OK;
}

bc_status bc_destroy(bc_ctx *ctx) {
    if (!ctx) return BC_ERR_INVALID_ARG;
    (void)hipStreamSynchronize(ctx->stream);
    for (auto &kv : ctx->graph_cache) {
        if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
        if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
    }
    for (auto &kv : ctx->tickets) release_ticket(ctx, kv.second);
    ctx->tickets.clear();
    for (auto *se : ctx->spare_steps) {
        (void)hipEventDestroy(se->begin);
        (void)hipEventDestroy(se->end);
        delete se;
    }
    if (ctx->clock_ev) (void)hipEventDestroy(ctx->clock_ev);
    if (ctx->clock_stream) (void)hipStreamDestroy(ctx->clock_stream);
    if (ctx->h_status) (void)hipHostFree(ctx->h_status);
    for (int r = 0; r < RING; ++r) {
        if (ctx->h_ring[r]) (void)hipHostFree(ctx->h_ring[r]);
        if (ctx->ring_ev[r]) (void)hipEventDestroy(ctx->ring_ev[r]);
        for (int q = 0; q < 5; ++q)
            if (ctx->tev[r][q]) (void)hipEventDestroy(ctx->tev[r][q]);
    }
    for (auto *g : ctx->graphs) delete g;
    if (ctx->fork_ev) (void)hipEventDestroy(ctx->fork_ev);
    if (ctx->join_ev) (void)hipEventDestroy(ctx->join_ev);
    if (ctx->side) (void)hipStreamDestroy(ctx->side);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return BC_OK;
}

bc_status bc_load_graph(bc_ctx *ctx, int32_t n, int64_t m, const int32_t *src, const int32_t *dst, const int64_t *w,
                        int32_t directed, int64_t arc_capacity, int64_t estar_capacity, void *arena,
                        uint64_t arena_bytes, bc_graph_id *out) {
    if (!ctx || !out || n <= 0 || m < 0 || (m > 0 && (!src || !dst || !w)) || !arena)
        return fail(ctx, BC_ERR_INVALID_ARG, "bad arguments to bc_load_graph");
    if (((uintptr_t)arena & 255) != 0) return fail(ctx, BC_ERR_INVALID_ARG, "arena not 256-byte aligned");
    const int64_t arcs = directed ? m : 2 * m;
    if (arc_capacity < arcs) return fail(ctx, BC_ERR_CAPACITY, "arc capacity below the arc count");
    if (arc_capacity >= (int64_t)INT32_MAX) return fail(ctx, BC_ERR_CAPACITY, "arc capacity above 2^31-1");
    if (estar_capacity <= 0) estar_capacity = arc_capacity;
    estar_capacity = std::min(estar_capacity, arc_capacity);
    const uint64_t need = bc_graph_bytes(n, arc_capacity, estar_capacity);
    if (arena_bytes < need) return fail(ctx, BC_ERR_CAPACITY, "arena smaller than bc_graph_bytes");
    if (ctx->budget && ctx->in_use + arena_bytes > ctx->budget)
        return fail(ctx, BC_ERR_ADMISSION, "graph state would exceed the memory budget");
    if (plan_scratch(ctx, std::max(n, ctx->n_layout)).src < 1)
        return fail(ctx, BC_ERR_CAPACITY, "scratch too small for this n");
    // host mirror (validates ids, loops, weights, duplicates)
    GraphRec *g = new GraphRec();
    g->n = n;
    g->directed = directed ? 1 : 0;
    g->arc_cap = arc_capacity;
    g->es_cap = estar_capacity;
    g->arena = (char *)arena;
    g->arena_bytes = arena_bytes;
    Mirror &mr = g->mirror;
    mr.n = n;
    std::vector<std::pair<uint64_t, int32_t>> keyed;
    keyed.reserve(arcs);
    for (int64_t i = 0; i < m; ++i) {
        const int32_t a = src[i], b = dst[i];
        if (a < 0 || b < 0 || a >= n || b >= n) {
            delete g;
            return fail(ctx, BC_ERR_INVALID_ARG, "vertex id out of range");
        }
        if (a == b) {
            delete g;
            return fail(ctx, BC_ERR_SELF_LOOP, "self-loop");
        }
        if (w[i] <= 0 || w[i] > W_MAX) {
            delete g;
            return fail(ctx, BC_ERR_BAD_WEIGHT, "weight out of range");
        }
        keyed.push_back({(uint64_t)a * n + b, (int32_t)w[i]});
        if (!directed) keyed.push_back({(uint64_t)b * n + a, (int32_t)w[i]});
    }
    std::sort(keyed.begin(), keyed.end());
    for (size_t i = 1; i < keyed.size(); ++i)
        if (keyed[i].first == keyed[i - 1].first) {
            delete g;
            return fail(ctx, BC_ERR_DUPLICATE_EDGE, "duplicate edge");
        }
    mr.ptr.assign(n + 1, 0);
    mr.dst.resize(keyed.size());
    mr.w.resize(keyed.size());
    for (size_t i = 0; i < keyed.size(); ++i) {
        const int32_t a = (int32_t)(keyed[i].first / n);
        mr.dst[i] = (int32_t)(keyed[i].first % n);
        mr.w[i] = keyed[i].second;
        mr.ptr[a + 1]++;
    }
    for (int32_t a = 0; a < n; ++a) mr.ptr[a + 1] += mr.ptr[a];
    mr.arcs = (int64_t)keyed.size();
    size_t total = 0;
    g->P = carve((char *)arena, n, arc_capacity, estar_capacity, &total, &g->chk);
    g->P.directed = g->directed;
    g->live = true;
    ctx->n_layout = std::max(ctx->n_layout, n);  // the static pass below re-zeroes every slot
    ctx->graphs.push_back(g);
    ctx->in_use += arena_bytes;
    *out = (bc_graph_id)(ctx->graphs.size() - 1);
    bc_status st = static_pass(ctx, g);
    if (st) {
        g->live = false;
        ctx->in_use -= arena_bytes;
        return st;
    }
    return BC_OK;
}

bc_status bc_clone_graph(bc_ctx *ctx, bc_graph_id gid, void *arena, uint64_t arena_bytes, bc_graph_id *out) {
    GraphRec *src = get_graph(ctx, gid);
    if (!src) return fail(ctx, BC_ERR_INVALID_ARG, "no such graph");
    {
        const bc_status fq = flush_queues(ctx);
        if (fq) return fq;
    }
    if (!out || !arena) return fail(ctx, BC_ERR_INVALID_ARG, "bad arguments to bc_clone_graph");
    if (((uintptr_t)arena & 255) != 0) return fail(ctx, BC_ERR_INVALID_ARG, "arena not 256-byte aligned");
    const uint64_t need = bc_graph_bytes(src->n, src->arc_cap, src->es_cap);
    if (arena_bytes < need) return fail(ctx, BC_ERR_CAPACITY, "arena smaller than bc_graph_bytes");
    if (ctx->budget && ctx->in_use + arena_bytes > ctx->budget)
        return fail(ctx, BC_ERR_ADMISSION, "graph state would exceed the memory budget");
    HIPCHK(hipSetDevice(ctx->device));
    // stream-ordered: the copy sees every update enqueued on the source so far,
    // which the host mirror already holds
    HIPCHK(hipMemcpyAsync(arena, src->arena, need, hipMemcpyDeviceToDevice, ctx->stream));
    GraphRec *g = new GraphRec(*src);
    g->arena = (char *)arena;
    g->arena_bytes = arena_bytes;
    size_t total = 0;
    g->P = carve((char *)arena, g->n, g->arc_cap, g->es_cap, &total, &g->chk);
    g->P.directed = g->directed;
    ctx->graphs.push_back(g);
    ctx->in_use += arena_bytes;
    *out = (bc_graph_id)(ctx->graphs.size() - 1);
    return BC_OK;
}

bc_status bc_free_graph(bc_ctx *ctx, bc_graph_id gid) {
    GraphRec *g = get_graph(ctx, gid);
    if (!g) return fail(ctx, BC_ERR_INVALID_ARG, "no such graph");
    {
        const bc_status fq = flush_queues(ctx);
        if (fq) return fq;
    }
    HIPCHK(hipStreamSynchronize(ctx->stream));
    g->live = false;
    ctx->in_use -= g->arena_bytes;
    g->mirror = Mirror();
    g->dev = Mirror();
    return BC_OK;
}

bc_status bc_update_edge(bc_ctx *ctx, bc_graph_id gid, int32_t u, int32_t v, int64_t w) {
    GraphRec *g = get_graph(ctx, gid);
    if (!g) return fail(ctx, BC_ERR_INVALID_ARG, "no such graph");
    {
        const bc_status fq = flush_queues(ctx);
        if (fq) return fq;
    }
    Pending p;
    std::vector<UpdateJob> jobs;
    bc_status st = validate_edge(ctx, g, u, v, w, p, jobs);
    if (st) return st;
    apply_pending(g, p);
    for (auto &j : jobs) {
        std::vector<UpdateJob> one(1, j);
        if ((st = run_step(ctx, one, false))) return st;
    }
    g->updates += 1;
    return BC_OK;
}

bc_status bc_update_vertex(bc_ctx *ctx, bc_graph_id gid, int32_t v, int32_t k, const bc_edge *e) {
    GraphRec *g = get_graph(ctx, gid);
    if (!g) return fail(ctx, BC_ERR_INVALID_ARG, "no such graph");
    {
        const bc_status fq = flush_queues(ctx);
        if (fq) return fq;
    }
    Pending p;
    std::vector<UpdateJob> jobs;
    bc_status st = validate_vertex(ctx, g, v, k, e, p, jobs);
    if (st) return st;
    apply_pending(g, p);
    for (auto &j : jobs) {
        std::vector<UpdateJob> one(1, j);
        if ((st = run_step(ctx, one, false))) return st;
    }
    g->updates += 1;
    return BC_OK;
}

namespace {

// Validates requests as one call (none is taken if one fails): each request's
// jobs, in order, with the graphs' arc changes applied to their mirrors.
// req_jobs[i] holds request i's jobs.
static bc_status validate_requests(bc_ctx *ctx, int32_t cnt, const bc_request *reqs, int32_t *bad_index,
                            std::vector<std::vector<UpdateJob>> &req_jobs) {
    std::map<int32_t, Pending> pend;
    req_jobs.assign((size_t)cnt, {});
    for (int32_t i = 0; i < cnt; ++i) {
        const bc_request &r = reqs[i];
        GraphRec *g = get_graph(ctx, r.graph);
        bc_status st;
        if (!g) st = fail(ctx, BC_ERR_INVALID_ARG, "no such graph");
        else if (r.kind == 0) st = validate_edge(ctx, g, r.u, r.v, r.w, pend[r.graph], req_jobs[i]);
        else if (r.kind == 1) st = validate_vertex(ctx, g, r.v, r.k, r.edges, pend[r.graph], req_jobs[i]);
        else st = fail(ctx, BC_ERR_INVALID_ARG, "bad request kind");
        if (st) {
            if (bad_index) *bad_index = i;
            return st;
        }
    }
    for (auto &kv : pend) apply_pending(ctx->graphs[kv.first], kv.second);
    for (int32_t i = 0; i < cnt; ++i) ctx->graphs[reqs[i].graph]->updates += 1;
    return BC_OK;
}

}  // namespace

bc_status bc_submit(bc_ctx *ctx, int32_t cnt, const bc_request *reqs, uint64_t *ticket, int32_t *bad_index) {
    if (!ctx || cnt < 0 || (cnt > 0 && !reqs) || !ticket) return fail(ctx, BC_ERR_INVALID_ARG, "bad arguments to bc_submit");
    if (bad_index) *bad_index = -1;
    bc_status st = flush_queues(ctx);
    if (st) return st;
    std::vector<std::vector<UpdateJob>> req_jobs;
    if ((st = validate_requests(ctx, cnt, reqs, bad_index, req_jobs))) return st;
    Ticket t;
    t.t_enqueue_ns = monotonic_ns();
    std::vector<int32_t> order;
    std::map<int32_t, std::vector<UpdateJob>> per_graph;
    for (int32_t i = 0; i < cnt; ++i) {
        const int32_t gid = reqs[i].graph;
        if (std::find(order.begin(), order.end(), gid) == order.end()) order.push_back(gid);
        auto &v = per_graph[gid];
        v.insert(v.end(), req_jobs[i].begin(), req_jobs[i].end());
    }
    t.graphs = order;
    size_t steps = 0;
    for (auto &kv : per_graph) steps = std::max(steps, kv.second.size());
    std::vector<StepEvents *> used;
    auto step_once = [&](const std::vector<UpdateJob> &part) -> bc_status {
        StepEvents *se;
        bc_status rc = take_step_events(ctx, &se);
        if (rc) return rc;
        se->refs++;
        rc = run_step(ctx, part, true, se);
        if (!rc) attach_step(ctx, t, se);
        unref_step(ctx, se);
        return rc;
    };
    for (size_t k = 0; k < steps; ++k) {
        std::vector<UpdateJob> step;
        for (int32_t gid : order) {
            auto &v = per_graph[gid];
            if (k < v.size()) step.push_back(v[k]);
        }
        for (size_t off = 0; off < step.size(); off += JCAP) {
            std::vector<UpdateJob> part(step.begin() + off, step.begin() + std::min(step.size(), off + JCAP));
            if ((st = step_once(part))) {
                release_ticket(ctx, t);
                return st;
            }
        }
    }
    if (steps == 0) {
        // nothing to run: a marker step so the ticket still has device times
        StepEvents *se;
        if ((st = take_step_events(ctx, &se))) return st;
        se->refs++;
        HIPCHK(hipEventRecord(se->begin, ctx->stream));
        HIPCHK(hipEventRecord(se->end, ctx->stream));
        attach_step(ctx, t, se);
        unref_step(ctx, se);
    }
    *ticket = ctx->next_ticket++;
    ctx->tickets[*ticket] = t;
    return BC_OK;
}

bc_status bc_enqueue(bc_ctx *ctx, int32_t cnt, const bc_request *reqs, uint64_t *tickets, int32_t *bad_index) {
    if (!ctx || cnt < 0 || (cnt > 0 && (!reqs || !tickets))) return fail(ctx, BC_ERR_INVALID_ARG, "bad arguments to bc_enqueue");
    if (bad_index) *bad_index = -1;
    std::vector<std::vector<UpdateJob>> req_jobs;
    bc_status st = validate_requests(ctx, cnt, reqs, bad_index, req_jobs);
    if (st) return st;
    const int64_t now = monotonic_ns();
    for (int32_t i = 0; i < cnt; ++i) {
        const uint64_t id = ctx->next_ticket++;
        Ticket t;
        t.t_enqueue_ns = now;
        t.graphs.push_back(reqs[i].graph);
        t.jobs_queued = (int32_t)req_jobs[i].size();
        ctx->tickets[id] = t;
        auto &q = ctx->queues[reqs[i].graph];
        for (auto &j : req_jobs[i]) q.push_back(QueuedJob{j, id, ctx->queue_seq++});
        ctx->queued_jobs += (int64_t)req_jobs[i].size();
        tickets[i] = id;
    }
    return BC_OK;
}

bc_status bc_step(bc_ctx *ctx, int32_t max_jobs, int32_t *launched, uint64_t *step_ticket) {
    if (!ctx || !launched) return fail(ctx, BC_ERR_INVALID_ARG, "bad arguments to bc_step");
    if (step_ticket) *step_ticket = 0;
    return launch_queued_step(ctx, max_jobs > 0 ? max_jobs : JCAP, launched, step_ticket);
}

bc_status bc_poll(bc_ctx *ctx, uint64_t ticket, bc_result *out) {
    if (!ctx || !out) return BC_ERR_INVALID_ARG;
    memset(out, 0, sizeof *out);
    auto it = ctx->tickets.find(ticket);
    if (it == ctx->tickets.end()) {
        if (ticket > 0 && ticket < ctx->next_ticket) {
            out->done = 1;  // collected before: no times left to report
            return BC_OK;
        }
        return fail(ctx, BC_ERR_INVALID_ARG, "unknown ticket");
    }
    Ticket &t = it->second;
    out->t_enqueue_ns = t.t_enqueue_ns;
    if (t.jobs_queued > 0 || !t.last) return BC_OK;  // not launched (all of it) yet
    hipError_t e = hipEventQuery(t.last->end);
    if (e == hipErrorNotReady) return BC_OK;
    if (e != hipSuccess) return hip_fail(ctx, e, "hipEventQuery");
    // keep the clock mapping fresh (the clock stream is idle; no update work
    // is waited for)
    if (monotonic_ns() - ctx->clock_ns > CLOCK_REFRESH_NS) {
        bc_status cs = calibrate_clock(ctx);
        if (cs) return cs;
    }
    bc_status st = event_time_ns(ctx, t.first->begin, &out->t_start_ns);
    if (!st) st = event_time_ns(ctx, t.last->end, &out->t_finish_ns);
    if (st) return st;
    // the sticky status of the ticket's graphs, read on the clock stream
    std::vector<const int32_t *> words;
    for (int32_t gid : t.graphs) {
        GraphRec *g = get_graph(ctx, gid);
        if (g) words.push_back(&g->P.ctl->status);
    }
    int32_t acc = 0;
    bc_status rs = read_status(ctx, words, true, &acc);
    if (rs) return rs;
    out->status = sticky_to_status(acc);
    out->done = 1;
    release_ticket(ctx, t);
    ctx->tickets.erase(it);
    return BC_OK;
}

bc_status bc_wait(bc_ctx *ctx, uint64_t ticket) {
    if (!ctx) return BC_ERR_INVALID_ARG;
    auto it = ctx->tickets.find(ticket);
    if (it == ctx->tickets.end()) return (ticket > 0 && ticket < ctx->next_ticket) ? BC_OK : fail(ctx, BC_ERR_INVALID_ARG, "unknown ticket");
    // queued requests of the ticket are launched first (steps of heads)
    while (it->second.jobs_queued > 0) {
        int32_t launched = 0;
        bc_status st = launch_queued_step(ctx, JCAP, &launched, nullptr);
        if (st) return st;
        if (!launched) return fail(ctx, BC_ERR_INVALID_ARG, "ticket has queued jobs but no queue holds them");
    }
    if (it->second.last) HIPCHK(hipEventSynchronize(it->second.last->end));
    // the sticky status of the ticket's graphs, read on the clock stream (the
    // library stream may hold later steps)
    std::vector<const int32_t *> words;
    for (int32_t gid : it->second.graphs) {
        GraphRec *g = get_graph(ctx, gid);
        if (g) words.push_back(&g->P.ctl->status);
    }
    int32_t acc = 0;
    bc_status rs = read_status(ctx, words, true, &acc);
    release_ticket(ctx, it->second);
    ctx->tickets.erase(it);
    if (rs) return rs;
    return sticky_to_status(acc);
}

bc_status bc_sync(bc_ctx *ctx) {
    if (!ctx) return BC_ERR_INVALID_ARG;
    bc_status fs = flush_queues(ctx);
    if (fs) return fs;
    // every live graph's status word, gathered behind the work and copied
    // into pinned memory, then one wait
    std::vector<const int32_t *> words;
    for (GraphRec *g : ctx->graphs)
        if (g && g->live) words.push_back(&g->P.ctl->status);
    int32_t acc = 0;
    bc_status rs = read_status(ctx, words, false, &acc);
    if (rs) return rs;
    return sticky_to_status(acc);
}

bc_status bc_scores(bc_ctx *ctx, bc_graph_id gid, double *out) {
    GraphRec *g = get_graph(ctx, gid);
    if (!g || !out) return fail(ctx, BC_ERR_INVALID_ARG, "no such graph or null output");
    std::vector<double> hi(g->n), lo(g->n);
    HIPCHK(hipMemcpyAsync(hi.data(), g->P.bc_hi, 8 * (size_t)g->n, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipMemcpyAsync(lo.data(), g->P.bc_lo, 8 * (size_t)g->n, hipMemcpyDeviceToHost, ctx->stream));
    int32_t st = 0;
    bc_status s = read_status(ctx, g, &st);
    if (s) return s;
    if (st) return sticky_to_status(st);
    for (int32_t i = 0; i < g->n; ++i) out[i] = hi[i] + lo[i];
    return BC_OK;
}

bc_status bc_recompute(bc_ctx *ctx, bc_graph_id gid) {
    GraphRec *g = get_graph(ctx, gid);
    if (!g) return fail(ctx, BC_ERR_INVALID_ARG, "no such graph");
    {
        const bc_status fq = flush_queues(ctx);
        if (fq) return fq;
    }
    return static_pass(ctx, g);
}

bc_status bc_recompute_estar(bc_ctx *ctx, bc_graph_id gid) {
    GraphRec *g = get_graph(ctx, gid);
    if (!g) return fail(ctx, BC_ERR_INVALID_ARG, "no such graph");
    {
        const bc_status fq = flush_queues(ctx);
        if (fq) return fq;
    }
    return static_pass(ctx, g, true);
}

bc_status bc_check(bc_ctx *ctx, bc_graph_id gid) {
    GraphRec *g = get_graph(ctx, gid);
    if (!g) return fail(ctx, BC_ERR_INVALID_ARG, "no such graph");
    {
        const bc_status fq = flush_queues(ctx);
        if (fq) return fq;
    }
    // every request validated so far is launched: the mirror is the device's arc set
    int32_t status = 0;
    const bc_status st = run_check(ctx, g, g->mirror, true, &status);
    if (st) return st;
    return status ? fail(ctx, sticky_to_status(status), "graph carries a sticky error") : BC_OK;
}

bc_status bc_get_rows(bc_ctx *ctx, bc_graph_id gid, int32_t s0, int32_t cnt, int64_t *D, uint64_t *sigma) {
    GraphRec *g = get_graph(ctx, gid);
    if (!g || s0 < 0 || cnt < 0 || s0 + (int64_t)cnt > g->n) return fail(ctx, BC_ERR_INVALID_ARG, "bad row range");
    const size_t cells = (size_t)cnt * g->n;
    std::vector<int32_t> d32(D ? cells : 0);
    if (D) HIPCHK(hipMemcpyAsync(d32.data(), g->P.D + (size_t)s0 * g->n, 4 * cells, hipMemcpyDeviceToHost, ctx->stream));
    if (sigma) HIPCHK(hipMemcpyAsync(sigma, g->P.S + (size_t)s0 * g->n, 8 * cells, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (D)
        for (size_t i = 0; i < cells; ++i) D[i] = d32[i] == INF32 ? INT64_MAX : (int64_t)d32[i];
    return BC_OK;
}

bc_status bc_get_arcs(bc_ctx *ctx, bc_graph_id gid, int32_t *src, int32_t *dst, int64_t *w, int64_t cap,
                      int64_t *cnt) {
    GraphRec *g = get_graph(ctx, gid);
    if (!g || !cnt || cap < 0) return fail(ctx, BC_ERR_INVALID_ARG, "bad arguments");
    const Mirror &M = g->mirror;
    // the CSR in tail order, then the arcs inserted since its last rebuild
    // (sorted); an undirected edge once, from its smaller endpoint
    std::vector<std::pair<uint64_t, int32_t>> extra(M.extra.begin(), M.extra.end());
    std::sort(extra.begin(), extra.end());
    int64_t k = 0;
    auto emit = [&](int32_t a, int32_t b, int32_t wt) {
        if (!g->directed && b < a) return;
        if (k < cap) {
            if (src) src[k] = a;
            if (dst) dst[k] = b;
            if (w) w[k] = wt;
        }
        ++k;
    };
    for (int32_t a = 0; a < g->n; ++a)
        for (int64_t i = M.ptr[a]; i < M.ptr[a + 1]; ++i) emit(a, M.dst[i], M.w[i]);
    for (auto &e : extra) emit((int32_t)(e.first / (uint64_t)g->n), (int32_t)(e.first % (uint64_t)g->n), e.second);
    *cnt = k;
    return BC_OK;
}

bc_status bc_get_estar(bc_ctx *ctx, bc_graph_id gid, int32_t *a, int32_t *b, int64_t *w, int64_t cap, int64_t *cnt) {
    GraphRec *g = get_graph(ctx, gid);
    if (!g || !cnt || cap < 0) return fail(ctx, BC_ERR_INVALID_ARG, "bad arguments");
    int32_t m = 0;
    HIPCHK(hipMemcpyAsync(&m, &g->P.ctl->esc_m, 4, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    *cnt = m;
    const size_t k = (size_t)std::min<int64_t>(cap, m);
    std::vector<int32_t> ww(k);
    if (k) {
        if (a) HIPCHK(hipMemcpyAsync(a, g->P.xc_src, 4 * k, hipMemcpyDeviceToHost, ctx->stream));
        if (b) HIPCHK(hipMemcpyAsync(b, g->P.xc_dst, 4 * k, hipMemcpyDeviceToHost, ctx->stream));
        if (w) HIPCHK(hipMemcpyAsync(ww.data(), g->P.xc_w, 4 * k, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        if (w)
            for (size_t i = 0; i < k; ++i) w[i] = ww[i];
    }
    return BC_OK;
}

bc_status bc_get_dag(bc_ctx *ctx, bc_graph_id gid, int32_t s, int32_t *a, int32_t *b, int64_t cap, int64_t *cnt) {
    GraphRec *g = get_graph(ctx, gid);
    if (!g || s < 0 || s >= g->n || !cnt || cap < 0) return fail(ctx, BC_ERR_INVALID_ARG, "bad arguments");
    std::vector<UpdateJob> jobs(1, job_template(g));
    int r;
    bc_status st;
    if ((st = ring_acquire(ctx, &r))) return st;
    if ((st = ring_stage(ctx, r, jobs))) return st;
    unsigned long long *dcnt = (unsigned long long *)misc_dev(ctx);
    HIPCHK(hipMemsetAsync(dcnt, 0, 8, ctx->stream));
    // DAG(s) is a subset of E*, so the spare E* buffer YC holds it
    hipLaunchKernelGGL(k_dag_arcs, dim3(1024), dim3(256), 0, ctx->stream, ring_jobs_dev(ctx, r), s, g->P.yc_src,
                       g->P.yc_dst, g->es_cap, dcnt);
    HIPCHK(hipGetLastError());
    if ((st = ring_release(ctx, r))) return st;
    unsigned long long c = 0;
    HIPCHK(hipMemcpyAsync(&c, dcnt, 8, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    *cnt = (int64_t)c;
    const size_t k = (size_t)std::min<int64_t>(cap, (int64_t)c);
    if (k) {
        if (a) HIPCHK(hipMemcpyAsync(a, g->P.yc_src, 4 * k, hipMemcpyDeviceToHost, ctx->stream));
        if (b) HIPCHK(hipMemcpyAsync(b, g->P.yc_dst, 4 * k, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
    }
    return BC_OK;
}

bc_status bc_get_affected(bc_ctx *ctx, bc_graph_id gid, int32_t *out, int64_t cap, int64_t *cnt) {
    GraphRec *g = get_graph(ctx, gid);
    if (!g || !cnt || cap < 0 || (cap > 0 && !out)) return fail(ctx, BC_ERR_INVALID_ARG, "bad arguments");
    unsigned long long a = 0;
    HIPCHK(hipMemcpyAsync(&a, &g->P.ctl->affected_last, sizeof a, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    *cnt = (int64_t)a;
    const size_t k = (size_t)std::min<int64_t>(cap, (int64_t)a);
    if (k) {
        HIPCHK(hipMemcpyAsync(out, g->P.alist, 4 * k, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
    }
    return BC_OK;
}

bc_status bc_get_preds(bc_ctx *ctx, bc_graph_id gid, int32_t s, int32_t *out) {
    GraphRec *g = get_graph(ctx, gid);
    if (!g || s < 0 || s >= g->n || !out) return fail(ctx, BC_ERR_INVALID_ARG, "bad arguments");
    HIPCHK(hipMemcpyAsync(out, g->P.pred + (size_t)s * g->n, 4 * (size_t)g->n, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return BC_OK;
}

bc_status bc_get_delta(bc_ctx *ctx, bc_graph_id gid, int32_t s, double *out) {
    GraphRec *g = get_graph(ctx, gid);
    if (!g || s < 0 || s >= g->n || !out) return fail(ctx, BC_ERR_INVALID_ARG, "bad arguments");
    const ScratchPlan sp = plan_scratch(ctx, ctx->n_layout);
    if (sp.src < 1) return fail(ctx, BC_ERR_CAPACITY, "scratch too small");
    std::vector<UpdateJob> jobs(1, job_template(g));
    int r;
    bc_status st;
    if ((st = ring_acquire(ctx, &r))) return st;
    if ((st = ring_stage(ctx, r, jobs))) return st;
    const int lds = std::min<int32_t>(g->n, 28672);  // row, expansion arrays and small-DAG table fit in 160 KiB
    // the pass runs in wide slot 0; the row lands in its B-list value area,
    // which the pass does not use
    double *row = (double *)(sp.wide_base + wide_layout(ctx->n_layout).bl_s);
    hipLaunchKernelGGL(k_delta_row, dim3(1), dim3(1024), source_lds_bytes(lds, 1024, 0), ctx->stream,
                       ring_jobs_dev(ctx, r), s, sp.wide_base, lds, ctx->n_layout, row);
    HIPCHK(hipGetLastError());
    if ((st = ring_release(ctx, r))) return st;
    HIPCHK(hipMemcpyAsync(out, row, 8 * (size_t)g->n, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return BC_OK;
}

bc_status bc_get_delta_noalloc(bc_ctx *ctx, bc_graph_id gid, int32_t s, double *out) {
    GraphRec *g = get_graph(ctx, gid);
    if (!g || s < 0 || s >= g->n || !out) return fail(ctx, BC_ERR_INVALID_ARG, "bad arguments");
    if (g->n > FIXED_N_MAX)
        return fail(ctx, BC_ERR_CAPACITY, "graph has more vertices than the fixed scratch serves (32768)");
    if (!ctx->fixed_scratch) return fail(ctx, BC_ERR_HIP, "fixed scratch not resolved on this device");
    // the same pass as bc_get_delta, in the fixed slot laid out for the
    // largest n it serves (its zero-kept arrays then sit at fixed offsets for
    // every graph), the graph's pointers passed by value
    const int lds = std::min<int32_t>(g->n, 28672);
    hipLaunchKernelGGL(k_delta_row_byval, dim3(1), dim3(1024), source_lds_bytes(lds, 1024, 0), ctx->stream, g->P, s,
                       ctx->fixed_scratch, lds, FIXED_N_MAX, out);
    HIPCHK(hipGetLastError());
    return BC_OK;
}

bc_status bc_state_hash(bc_ctx *ctx, bc_graph_id gid, uint64_t out[2]) {
    GraphRec *g = get_graph(ctx, gid);
    if (!g || !out) return fail(ctx, BC_ERR_INVALID_ARG, "bad arguments");
    std::vector<UpdateJob> jobs(1, job_template(g));
    int r;
    bc_status st;
    if ((st = ring_acquire(ctx, &r))) return st;
    if ((st = ring_stage(ctx, r, jobs))) return st;
    unsigned long long *dh = (unsigned long long *)misc_dev(ctx) + 2;
    HIPCHK(hipMemsetAsync(dh, 0, 16, ctx->stream));
    hipLaunchKernelGGL(k_hash, dim3(1024), dim3(256), 0, ctx->stream, ring_jobs_dev(ctx, r), dh);
    HIPCHK(hipGetLastError());
    if ((st = ring_release(ctx, r))) return st;
    HIPCHK(hipMemcpyAsync(out, dh, 16, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return BC_OK;
}

bc_status bc_get_stats(bc_ctx *ctx, bc_graph_id gid, bc_update_stats *out) {
    GraphRec *g = get_graph(ctx, gid);
    if (!g || !out) return fail(ctx, BC_ERR_INVALID_ARG, "bad arguments");
    GraphCtl c;
    HIPCHK(hipMemcpyAsync(&c, g->P.ctl, sizeof c, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    out->affected_sources = (int64_t)c.affected_last;
    out->changed_pairs = (int64_t)c.changed_pairs;
    out->estar_arcs = c.esc_m;
    out->max_levels = c.max_levels;
    out->updates_applied = (int64_t)g->updates;
    out->total_affected = (int64_t)c.affected_total;
    out->total_changed = (int64_t)c.changed_total;
    out->deferred_sources = c.big_last;
    out->scan_bytes = (int64_t)c.scan_bytes_last;
    out->total_scan_bytes = (int64_t)c.scan_bytes_total;
    out->search_arcs = g->search_arcs;
    out->search_rounds = g->search_rounds;
    CheckRec r{};
    HIPCHK(hipMemcpyAsync(&r, g->chk, sizeof r, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    out->check_rows = (int64_t)r.rows;
    out->check_failures = (int64_t)r.fails;
    out->check_source = r.fails ? r.s : -1;
    out->check_target = r.fails ? r.t : -1;
    out->check_kind = r.fails ? r.kind : 0;
    return BC_OK;
}

bc_status bc_get_timing(bc_ctx *ctx, bc_timing *out) {
    if (!ctx || !out) return BC_ERR_INVALID_ARG;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    bc_status st = harvest_all(ctx);
    if (st) return st;
    out->step_ms = ctx->step_ms;
    out->source_ms = ctx->source_ms;
    out->rows_ms = ctx->rows_ms;
    out->steps = ctx->timed_steps;
    return BC_OK;
}

bc_status bc_reset_timing(bc_ctx *ctx) {
    if (!ctx) return BC_ERR_INVALID_ARG;
    HIPCHK(hipStreamSynchronize(ctx->stream));
    bc_status st = harvest_all(ctx);
    if (st) return st;
    ctx->step_ms = ctx->source_ms = ctx->rows_ms = 0;
    ctx->timed_steps = 0;
    return BC_OK;
}

}  // extern "C"
