// Device-side data structures of libbcinc (shared by its kernels and its host
// code; nothing here is shared with anything outside the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bcinc {

// Unreachable marker of the int32 distance matrix.  Finite distances stay
// strictly below it; a finite result that would reach it is an overflow.
constexpr int32_t INF32 = 0x7fffffff;
// Stored DAG predecessor of a pair (s, x): the tail of its only DAG(s) in-arc,
// or one of these.
constexpr int32_t PRED_NONE = -1;   // x == s or x unreachable from s
constexpr int32_t PRED_MULTI = -2;  // two or more DAG(s) in-arcs

// Arcs per direction carried inline by one update job (E_i and E_o of
// Section 4).  Larger vertex updates are split on the host into consecutive
// vertex updates at the same vertex.
constexpr int KMAX = 64;

// Most vertices whose distance row fits in LDS (4 bytes each) next to the
// per-workgroup bookkeeping: 36864 * 4 = 144 KiB of the 160 KiB of gfx950.
constexpr int32_t LDS_ROW_MAX = 36864;

// E* rebuild modes (see the k_es_* kernels).
//   ES_BUILD   all arcs (CSR by tail)  -> X  (arcs with w == d)
//   ES_BUILD_C all arcs (CSR by head)  -> XC (arcs with w == d)
//   ES_MERGE   XC plus the updated arcs -> YC (k_es_merge, elementwise)
//   ES_FILTER  YC                       -> XC (arcs with w == d after the update;
//              k_es_keep, k_es_wscan, k_es_place, arc-parallel)
enum { ES_BUILD = 0, ES_BUILD_C = 1, ES_MERGE = 2, ES_FILTER = 3 };

// Flags of the restricted dependency pass.  The LDS table keeps them apart;
// the global-memory pass packs them with the successor count in one word.
enum : int32_t { F_VIS = 1, F_B = 2 };
constexpr int32_t W_COUNT = 0x0fffffff, W_B = 1 << 29, W_VIS = 1 << 30;

// Sources whose changed-target set exceeds this many targets are deferred by
// the per-source kernel to its wide-workgroup companion.
constexpr int32_t BIG_B = 512;

// Sticky status bits of a graph.
enum : int32_t { ST_SIGMA_OVF = 1, ST_DIST_OVF = 2, ST_ESTAR_CAP = 4 };

// Control words of one graph, resident in device memory.  The counters that
// many workgroups bump with atomics during a step sit on 256-byte lines of
// their own: atomics on one line are serialized where the line lives, so
// counters sharing a line would queue behind each other.
struct GraphCtl {
    int32_t status;     // sticky ST_* bits
    int32_t a_count;    // |A| of the update in flight (written by the scan)
    int32_t max_levels; // deepest Kahn level count seen (statistic)
    int32_t es_m;       // arcs in X (E* by tail, built by the static pass)
    int32_t esc_m;      // arcs in XC (E* by head, kept current)
    int32_t esc_m_tmp;  // arcs in YC (E* by head plus the updated arcs)
    int32_t t_count;    // candidate targets of the update in flight
    int32_t big_last;   // deferred sources of the last update (statistic)
    unsigned long long affected_last;  // |A| of the last update
    unsigned long long updates;        // updates applied since load
    unsigned long long affected_total; // sums over all updates since load
    unsigned long long changed_total;
    unsigned long long scan_bytes_last;  // row-scan bytes of the last update (see k_commit)
    unsigned long long scan_bytes_total;
    alignas(256) int32_t work_next;    // next item of the persistent per-source kernel
    alignas(256) int32_t dag_count;    // listed sources with many changed targets: dlist[0 .. dag_count)
    alignas(256) int32_t dag_back;     // listed sources with few: dlist[n - dag_back .. n)
    alignas(256) int32_t dag_next;     // next listed source with many changed targets (DAG kernel)
    alignas(256) int32_t dag_next_light;  // next listed source with few
    alignas(256) int32_t big_count;    // deferred (large) sources of the update in flight
    alignas(256) int32_t big_next;     // next deferred source to process
    alignas(256) unsigned long long changed_pairs;  // statistic of the last update
};

// Per-source scalars of the update in flight (Alg 4 output).
//   dv = d'(s,v), sv = sigma'_sv, hv = sigma-hat'_sv (new paths through E_i);
//   flag bit 0: d'(s,v) == d(s,v) ("same"), bit 1: s is affected.
struct SrcScal {
    int32_t dv;
    int32_t flags;
    uint64_t sv;
    uint64_t hv;
};

// A source whose changed targets the row kernel listed: entries
// [off, off + nb) of the step's target pool.
struct DItem {
    int32_t s;
    int32_t nb;
    int64_t off;
};

// Target pool of one update step: the changed targets (with their new d and
// sigma) of every listed source of every job, bump-allocated.
struct StepPool {
    int32_t *t;
    int32_t *d;
    uint64_t *s;
    unsigned long long *next;
    int64_t cap;
};

// Most changed targets the row kernel lists for one source (in LDS).
constexpr int32_t LCAP = 1024;
// Listed sources with at least this many changed targets go first to the DAG
// kernel (their sub-DAGs take longest; starting them first shortens the tail).
constexpr int32_t HEAVY_NB = 32;

// Device pointers and sizes of one graph.  A copy rides in every job.
struct GraphPtrs {
    int32_t n;
    int32_t directed;
    int64_t es_cap;  // capacity of each E* buffer (arcs)
    int32_t *D;      // n x n distances, INF32 = unreachable
    int32_t *pred;   // n x n: pred[s*n + x] = the DAG(s) predecessor of x, PRED_NONE or PRED_MULTI
    uint64_t *S;     // n x n path counts
    double *bc_hi, *bc_lo;  // BC as an unevaluated sum hi + lo
    double *bc_delta;       // per-update difference, folded into (hi, lo) at commit
    // E* three ways: X by tail (static pass), XC by head (current), YC by
    // head with the updated arcs merged in (during an update).
    int32_t *x_ptr, *x_src, *x_dst, *x_w;
    int32_t *xc_ptr, *xc_src, *xc_dst, *xc_w;
    int32_t *yc_ptr, *yc_src, *yc_dst, *yc_w;
    int32_t *es_cnt;  // n + 1 counts / offsets for rebuilding
    SrcScal *scal;    // n
    int32_t *alist;   // n, affected sources
    int32_t *biglist; // n, affected sources deferred to the wide kernel
    DItem *dlist;     // n, sources listed by the row kernel
    int32_t *rv_D;    // snapshot of row v before the update (n)
    uint64_t *rv_S;
    int32_t *rvv_D;   // row v'' after the Out phase (n)
    uint64_t *rvv_S, *rvv_H;
    int32_t *tlist;   // candidate targets of the update in flight (n)
    int32_t *tl_rvD;  // d(v,t) for each candidate (compact copy)
    int32_t *tl_rvvD; // d''(v,t) for each candidate (compact copy)
    int32_t *f_any;   // n: min of f_in and f_out, where f_in = d(v,t) if the In phase can
                      // change a pair (s,t), else INF32, and f_out likewise for the Out
                      // phase with d''(v,t)
    int32_t *f_out;
    GraphCtl *ctl;
    // Full arc set by tail and by head (static recompute and E* build).  No
    // update reads them; a state check puts the current arcs by head in
    // arcin_* before it runs.
    int32_t *arc_ptr, *arc_dst, *arc_w;
    int32_t *arcin_ptr, *arcin_src, *arcin_w;
    int64_t arc_m;
};

// One update on one graph: centre vertex v, in-arcs E_i = {(in_tail[j], v)}
// and out-arcs E_o = {(v, out_head[j])} with their new weights.  An arc
// update (u, v) is the vertex form at v with E_i = {(u, v)} and E_o empty.
// The merged arc list u_* (tail-sorted) is E_i and E_o together, the arcs
// that enter E* candidates.
struct UpdateJob {
    GraphPtrs g;
    int32_t v;
    int32_t n_in, n_out;
    int32_t n_u;
    const int32_t *row_v_D;   // row v to read during the update: live row, or the snapshot
    const uint64_t *row_v_S;  // when the Out phase rewrites row v
    int32_t in_tail[KMAX], in_w[KMAX];
    int32_t out_head[KMAX], out_w[KMAX];
    int32_t u_tail[2 * KMAX], u_head[2 * KMAX], u_w[2 * KMAX];
};

__host__ __device__ constexpr inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Per-workgroup scratch of the static pass (Kahn levels over a whole DAG).
struct StaticLayout {
    size_t indeg, order, lvl, coef, queue2, total;
};

__host__ __device__ inline StaticLayout static_layout(int32_t n) {
    StaticLayout L;
    size_t off = 0;
    L.indeg = off;  off += align256(sizeof(int32_t) * (size_t)n);
    L.order = off;  off += align256(sizeof(int32_t) * (size_t)n);
    L.lvl = off;    off += align256(sizeof(int32_t) * ((size_t)n + 1));
    L.coef = off;   off += align256(sizeof(double) * (size_t)n);
    L.queue2 = off; off += align256(sizeof(int32_t) * (size_t)n);
    L.total = off;
    return L;
}

// Per-workgroup scratch of the DAG kernel's global sub-DAG pass: outdeg /
// acc / kcnt are kept all-zero between sources (each pass clears exactly the
// entries it used); a record of up to n sub-DAG arcs (ka = tail, kb = head,
// kr = tails grouped by head, kend = range ends) spares the Kahn rounds the
// Eq.1 tests.
struct UpdateLayout {
    size_t outdeg, acc, sub, q1, q2, kcnt, kend, ka, kb, kr, total;
    int64_t kcap;
};

__host__ __device__ inline UpdateLayout update_layout(int32_t n) {
    UpdateLayout L;
    size_t off = 0;
    L.kcap = n;
    L.outdeg = off; off += align256(sizeof(int32_t) * (size_t)n);
    L.acc = off;    off += align256(sizeof(double) * (size_t)n);
    L.sub = off;    off += align256(sizeof(int32_t) * (size_t)n);
    L.q1 = off;     off += align256(sizeof(int32_t) * (size_t)n);
    L.q2 = off;     off += align256(sizeof(int32_t) * (size_t)n);
    L.kcnt = off;   off += align256(sizeof(int32_t) * (size_t)n);
    L.kend = off;   off += align256(sizeof(int32_t) * (size_t)n);
    L.ka = off;     off += align256(sizeof(int32_t) * (size_t)L.kcap);
    L.kb = off;     off += align256(sizeof(int32_t) * (size_t)L.kcap);
    L.kr = off;     off += align256(sizeof(int32_t) * (size_t)L.kcap);
    L.total = off;
    return L;
}

// Most DAG arcs a full pass records, per vertex of the largest graph.
constexpr int32_t KARC_PER_VERTEX = 4;

// Per-workgroup scratch of the wide kernel: the arrays of UpdateLayout, the
// full-length changed-target list (bl_*), for full passes the recorded DAG
// arcs (ka = tail, kb = head, kr = tails grouped by head) with per-head
// counts (kcnt, kept all-zero) and range ends (kend), and the new distance
// and path-count rows of a source whose new pass runs apart from its old one
// (dnew, snew).
struct WideLayout {
    size_t outdeg, acc, sub, q1, q2, bl_t, bl_d, bl_s, kcnt, kend, ka, kb, kr, dnew, snew, total;
    int64_t kcap;
};

__host__ __device__ constexpr inline WideLayout wide_layout(int32_t n) {
    WideLayout L{};
    size_t off = 0;
    L.kcap = (int64_t)KARC_PER_VERTEX * n;
    L.outdeg = off; off += align256(sizeof(int32_t) * (size_t)n);
    L.acc = off;    off += align256(sizeof(double) * (size_t)n);
    L.sub = off;    off += align256(sizeof(int32_t) * (size_t)n);
    L.q1 = off;     off += align256(sizeof(int32_t) * (size_t)n);
    L.q2 = off;     off += align256(sizeof(int32_t) * (size_t)n);
    L.bl_t = off;   off += align256(sizeof(int32_t) * (size_t)n);
    L.bl_d = off;   off += align256(sizeof(int32_t) * (size_t)n);
    L.bl_s = off;   off += align256(sizeof(uint64_t) * (size_t)n);
    L.kcnt = off;   off += align256(sizeof(int32_t) * (size_t)n);
    L.kend = off;   off += align256(sizeof(int32_t) * (size_t)n);
    L.ka = off;     off += align256(sizeof(int32_t) * (size_t)L.kcap);
    L.kb = off;     off += align256(sizeof(int32_t) * (size_t)L.kcap);
    L.kr = off;     off += align256(sizeof(int32_t) * (size_t)L.kcap);
    L.dnew = off;   off += align256(sizeof(int32_t) * (size_t)n);
    L.snew = off;   off += align256(sizeof(uint64_t) * (size_t)n);
    L.total = off;
    return L;
}

// Changed-pair list of one deferred source whose old and new passes run on
// two workgroups: written by the old-pass workgroup, applied to D and sigma
// by k_wide_apply after the wide kernel.  Header (count) then t, d, sigma.
__host__ __device__ inline size_t item_region_bytes(int32_t n) {
    return 256 + align256(4 * (size_t)n) * 2 + align256(8 * (size_t)n);
}
struct ItemRegion {
    int32_t *nb, *t, *d;
    uint64_t *s;
};
__host__ __device__ inline ItemRegion item_region_at(char *base, int32_t n) {
    ItemRegion r;
    r.nb = (int32_t *)base;
    r.t = (int32_t *)(base + 256);
    r.d = (int32_t *)(base + 256 + align256(4 * (size_t)n));
    r.s = (uint64_t *)(base + 256 + 2 * align256(4 * (size_t)n));
    return r;
}

// Workgroup slots: the DAG kernel and the static pass share one region, the
// wide kernel has its own.
__host__ __device__ inline size_t slot_bytes_for(int32_t n) {
    const size_t a = static_layout(n).total, b = update_layout(n).total;
    return a > b ? a : b;
}
__host__ __device__ inline size_t wide_slot_bytes_for(int32_t n) { return wide_layout(n).total; }

}  // namespace bcinc
