// HIP kernels of libbcinc for gfx950 (64-lane wavefronts).
//
// Update pipeline for a batch of jobs (one update on each of several graphs):
//   k_scan        affected sources A and Alg 4 scalars (Eq.6, Eq.7)
//   k_rowv        row v'' of the Out phase (Alg 4 on the reverse graph)
//   k_es_*        E* candidates: merge the updated arcs into E* (buffer Y)
//   k_source      per affected source: old DAG dependencies, row update by
//                 Lemma 2 / Lemma 4, new DAG dependencies, BC difference
//   k_es_*        E*' = arcs of Y whose weight equals their new distance
//   k_commit      BC += difference (compensated), reset counters
// Static pass (initial state and full recompute, Alg 7):
//   k_sssp        distances of every source (frontier Bellman-Ford in LDS)
//   k_es_*        E* = arcs with w(a,b) = d(a,b)
//   k_static      per source: path counts in DAG order, dependencies, BC
#include "bc_device.h"

namespace bcinc {

// ------------------------------------------------------------ arithmetic ---

__device__ __forceinline__ uint64_t mul_chk(uint64_t a, uint64_t b, bool &ovf) {
    ovf |= (__umul64hi(a, b) != 0);
    return a * b;
}

__device__ __forceinline__ uint64_t add_chk(uint64_t a, uint64_t b, bool &ovf) {
    uint64_t r = a + b;
    ovf |= (r < a);
    return r;
}

// Lemma 4 (In phase) for one pair (s,t), with D(s,t) = d'(s,v) + d(v,t):
// case 1 keeps (d, sigma); case 2 adds sigma-hat'_sv * sigma_vt when
// d'(s,v) = d(s,v); case 3 adds sigma'_sv * sigma_vt when d'(s,v) < d(s,v);
// case 4 replaces both.  The arc update is the special case E_i = {(u,v)}:
// it reproduces the three cases of Lemma 2.  For t = v it returns Alg 4's
// d'(s,v), sigma'_sv.
__device__ __forceinline__ bool in_rule(int32_t d0, int32_t dv, int32_t dvt, int64_t &c) {
    if (dv == INF32 || dvt == INF32) return false;
    c = (int64_t)dv + (int64_t)dvt;
    return c <= (int64_t)d0;
}

// A graph whose E* outgrew its buffers is dead until reloaded: every kernel
// that walks E* row pointers skips it, so no access can leave the buffers.
__device__ __forceinline__ bool job_dead(const UpdateJob &J) {
    return (*(volatile int32_t *)&J.g.ctl->status & ST_ESTAR_CAP) != 0;
}

// ------------------------------------------------------------ wave tools ---

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint32_t popc_below(uint64_t mask, int lane) {
    return (uint32_t)__popcll(mask & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
}

// Block-wide exclusive scan of one int per thread (blockDim.x <= 1024).
__device__ int32_t block_excl_scan(int32_t x, int32_t *sh /* >= 32 */, int32_t &total) {
    const int lane = lane_id(), wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    int32_t incl = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int32_t y = __shfl_up(incl, d, 64);
        if (lane >= d) incl += y;
    }
    if (lane == 63) sh[wid] = incl;
    __syncthreads();
    if (wid == 0) {
        int32_t v = (lane < nw) ? sh[lane] : 0;
        int32_t vi = v;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            int32_t y = __shfl_up(vi, d, 64);
            if (lane >= d) vi += y;
        }
        if (lane < nw) sh[lane] = vi - v;
        if (lane == nw - 1) sh[32] = vi;
    }
    __syncthreads();
    int32_t res = sh[wid] + incl - x;
    total = sh[32];
    __syncthreads();
    return res;
}

// ------------------------------------------------------------ k_scan -------

// Per source s: Alg 4 over E_i (Eq.6 d'(s,v), Eq.7 sigma-hat'_sv, sigma'_sv),
// then the affected test.  s changes in the In phase iff d'(s,v) < d(s,v) or
// sigma-hat'_sv > 0 (Lemma 4 cases 2-4 need one of them; for an arc update
// this is Lemma 2 case 1 failing at t = v).  s changes in the Out phase iff
// d'(s,v) + w'(v,x) <= d'(s,x) for some (v,x) in E_o.  Affected sources are
// compacted with a wave ballot and one atomic per wave.
__global__ void __launch_bounds__(256) k_scan(const UpdateJob *__restrict__ jobs, const int32_t *__restrict__ njobs_p) {
    const int njobs = *njobs_p;
    for (int j = 0; j < njobs; ++j) {
        const UpdateJob &J = jobs[j];
        const int32_t n = J.g.n, v = J.v, n_in = J.n_in, n_out = J.n_out;
        const int32_t *D = J.g.D;
        const uint64_t *S = J.g.S;
        const int32_t *Dv = D + (size_t)v * n;
        bool ovf_s = false, ovf_d = false;
        for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < n; base += (int64_t)gridDim.x * blockDim.x) {
            const int32_t s = (int32_t)(base + threadIdx.x);
            bool aff = false;
            if (s < n) {
                const int32_t *Ds = D + (size_t)s * n;
                const uint64_t *Ss = S + (size_t)s * n;
                const int32_t dsv = Ds[v];
                int64_t cur = dsv;
                uint64_t sig = Ss[v], hat = 0;
                for (int k = 0; k < n_in; ++k) {
                    const int32_t u = J.in_tail[k];
                    const int32_t du = Ds[u];
                    if (du == INF32) continue;
                    const int64_t c = (int64_t)du + J.in_w[k];
                    if (c >= INF32) { ovf_d = true; continue; }
                    if (c == cur) {
                        const uint64_t su = Ss[u];
                        sig = add_chk(sig, su, ovf_s);
                        hat = add_chk(hat, su, ovf_s);
                    } else if (c < cur) {
                        cur = c;
                        sig = Ss[u];
                        hat = 0;
                    }
                }
                const bool same = (cur == (int64_t)dsv);
                aff = (cur < (int64_t)dsv) || (hat != 0);
                if (!aff && cur != INF32) {
                    for (int k = 0; k < n_out; ++k) {
                        const int32_t x = J.out_head[k];
                        int64_t d1 = Ds[x];
                        const int32_t dvx = Dv[x];
                        if (dvx != INF32 && cur + dvx < d1) d1 = cur + dvx;
                        const int64_t c = cur + J.out_w[k];
                        if (c < INF32 && c <= d1) { aff = true; break; }
                    }
                }
                SrcScal sc;
                sc.dv = (int32_t)cur;
                sc.flags = (same ? 1 : 0) | (aff ? 2 : 0);
                sc.sv = sig;
                sc.hv = hat;
                J.g.scal[s] = sc;
            }
            const uint64_t mask = __ballot(aff);
            if (mask) {
                const int lane = lane_id();
                const int leader = __ffsll((unsigned long long)mask) - 1;
                int32_t b0 = 0;
                if (lane == leader) b0 = atomicAdd(&J.g.ctl->a_count, (int32_t)__popcll(mask));
                b0 = __shfl(b0, leader, 64);
                if (aff) J.g.alist[b0 + popc_below(mask, lane)] = s;
            }
        }
        if (ovf_s) atomicOr(&J.g.ctl->status, ST_SIGMA_OVF);
        if (ovf_d) atomicOr(&J.g.ctl->status, ST_DIST_OVF);
    }
}

// ------------------------------------------------------------ k_rowv -------

// Row v'' (Section 4, Out phase): with E_o = {(v, x_j)}, Alg 4 on G'_R gives
// d''(v,t) = min(d'(v,t), min_j w'(v,x_j) + d'(x_j,t)) and the counts
// sigma''_vt, sigma-hat''_vt.  The rows x_j of G' are formed on the fly by
// the In-phase rule from the old rows.  Also snapshots the old row v, which
// the source v itself rewrites during the update.
__global__ void __launch_bounds__(256) k_rowv(const UpdateJob *__restrict__ jobs, const int32_t *__restrict__ njobs_p) {
    const int njobs = *njobs_p;
    for (int j = 0; j < njobs; ++j) {
        const UpdateJob &J = jobs[j];
        if (J.n_out == 0) continue;
        const int32_t n = J.g.n, v = J.v;
        const int32_t *D = J.g.D;
        const uint64_t *S = J.g.S;
        bool ovf_s = false, ovf_d = false;
        for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
            const int32_t dvt = D[(size_t)v * n + t];
            const uint64_t svt = S[(size_t)v * n + t];
            J.g.rv_D[t] = dvt;
            J.g.rv_S[t] = svt;
            int64_t cur = dvt;
            uint64_t sig = svt, hat = 0;
            for (int k = 0; k < J.n_out; ++k) {
                const int32_t x = J.out_head[k];
                const SrcScal sc = J.g.scal[x];
                int32_t d1 = D[(size_t)x * n + t];
                uint64_t s1 = 0;
                bool s1_known = false;
                int64_t c;
                if (in_rule(d1, sc.dv, dvt, c)) {
                    if (c >= INF32) { ovf_d = true; }
                    else if (c < d1) { d1 = (int32_t)c; s1 = mul_chk(sc.sv, svt, ovf_s); s1_known = true; }
                    else {
                        s1 = add_chk(S[(size_t)x * n + t], mul_chk((sc.flags & 1) ? sc.hv : sc.sv, svt, ovf_s), ovf_s);
                        s1_known = true;
                    }
                }
                if (d1 == INF32) continue;
                const int64_t cc = (int64_t)J.out_w[k] + d1;
                if (cc >= INF32) { ovf_d = true; continue; }
                if (cc <= cur) {
                    if (!s1_known) s1 = S[(size_t)x * n + t];
                    if (cc == cur) {
                        sig = add_chk(sig, s1, ovf_s);
                        hat = add_chk(hat, s1, ovf_s);
                    } else {
                        cur = cc;
                        sig = s1;
                        hat = 0;
                    }
                }
            }
            J.g.rvv_D[t] = (int32_t)cur;
            J.g.rvv_S[t] = sig;
            J.g.rvv_H[t] = hat;
        }
        if (ovf_s) atomicOr(&J.g.ctl->status, ST_SIGMA_OVF);
        if (ovf_d) atomicOr(&J.g.ctl->status, ST_DIST_OVF);
    }
}

// ------------------------------------------------------------ E* rebuild ---
//
// E* is a CSR by tail.  Three modes share one wave-per-tail compaction:
//   ES_MERGE:  Y = X plus the updated arcs (appended to their tails' segments)
//   ES_FILTER: X = arcs of Y with w == d(a,b) (after the update)
//   ES_BUILD:  X = arcs of the full arc set with w == d(a,b) (static pass)
// Arcs whose weight exceeds their distance lie on no shortest path, so they
// can be dropped; distances only decrease under incremental updates, so E*'
// is contained in E* plus the updated arcs.

struct EsView {
    const int32_t *ptr, *dst, *w;
    int32_t *optr, *osrc, *odst, *ow;
    int32_t m_limit;  // capacity of the output
    int32_t *m_out;   // where the total goes
};

__device__ __forceinline__ EsView es_view(const UpdateJob &J, int mode) {
    EsView e;
    if (mode == ES_MERGE) {
        e.ptr = J.g.x_ptr; e.dst = J.g.x_dst; e.w = J.g.x_w;
        e.optr = J.g.y_ptr; e.osrc = J.g.y_src; e.odst = J.g.y_dst; e.ow = J.g.y_w;
        e.m_out = &J.g.ctl->es_m_tmp;
    } else if (mode == ES_FILTER) {
        e.ptr = J.g.y_ptr; e.dst = J.g.y_dst; e.w = J.g.y_w;
        e.optr = J.g.x_ptr; e.osrc = J.g.x_src; e.odst = J.g.x_dst; e.ow = J.g.x_w;
        e.m_out = &J.g.ctl->es_m;
    } else {
        e.ptr = J.g.arc_ptr; e.dst = J.g.arc_dst; e.w = J.g.arc_w;
        e.optr = J.g.x_ptr; e.osrc = J.g.x_src; e.odst = J.g.x_dst; e.ow = J.g.x_w;
        e.m_out = &J.g.ctl->es_m;
    }
    e.m_limit = (int32_t)J.g.es_cap;
    return e;
}

__device__ __forceinline__ bool es_keep(const UpdateJob &J, int mode, int32_t a, int32_t b, int32_t w) {
    if (mode == ES_MERGE) return true;
    return J.g.D[(size_t)a * J.g.n + b] == w;
}

template <int MODE>
__global__ void __launch_bounds__(256) k_es_count(const UpdateJob *__restrict__ jobs, const int32_t *__restrict__ njobs_p) {
    const int njobs = *njobs_p;
    const int lane = lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int j = 0; j < njobs; ++j) {
        const UpdateJob &J = jobs[j];
        if (MODE != ES_BUILD && job_dead(J)) continue;
        const EsView e = es_view(J, MODE);
        const int32_t n = J.g.n;
        for (int64_t a = wave; a < n; a += nwaves) {
            const int32_t p0 = e.ptr[a], p1 = e.ptr[a + 1];
            int32_t cnt = 0;
            for (int32_t base = p0; base < p1; base += 64) {
                const int32_t i = base + lane;
                bool keep = false;
                if (i < p1) keep = es_keep(J, MODE, (int32_t)a, e.dst[i], e.w[i]);
                cnt += (int32_t)__popcll(__ballot(keep));
            }
            if (MODE == ES_MERGE) {
                for (int32_t base = 0; base < J.n_u; base += 64) {
                    const int32_t k = base + lane;
                    cnt += (int32_t)__popcll(__ballot(k < J.n_u && J.u_tail[k] == a));
                }
            }
            if (lane == 0) J.g.es_cnt[a] = cnt;
        }
    }
}

// One workgroup per job: exclusive scan of the per-tail counts into the
// output row pointers; the total goes to the control block.  A total above
// the capacity sets the sticky E* capacity error and the scatter is skipped.
template <int MODE>
__global__ void __launch_bounds__(1024) k_es_scan(const UpdateJob *__restrict__ jobs, const int32_t *__restrict__ njobs_p) {
    __shared__ int32_t sh[40];
    const int j = blockIdx.x;
    if (j >= *njobs_p) return;
    const UpdateJob &J = jobs[j];
    if (MODE != ES_BUILD && job_dead(J)) return;
    const EsView e = es_view(J, MODE);
    const int32_t n = J.g.n;
    const int32_t per = (n + blockDim.x - 1) / blockDim.x;
    const int32_t i0 = min(n, (int32_t)threadIdx.x * per), i1 = min(n, i0 + per);
    int32_t local = 0;
    for (int32_t i = i0; i < i1; ++i) local += J.g.es_cnt[i];
    int32_t total;
    int32_t off = block_excl_scan(local, sh, total);
    for (int32_t i = i0; i < i1; ++i) {
        const int32_t c = J.g.es_cnt[i];
        e.optr[i] = off;
        off += c;
    }
    if (threadIdx.x == 0) {
        e.optr[n] = total;
        if (total > e.m_limit) {
            atomicOr(&J.g.ctl->status, ST_ESTAR_CAP);
        } else {
            *e.m_out = total;
        }
    }
}

template <int MODE>
__global__ void __launch_bounds__(256) k_es_scatter(const UpdateJob *__restrict__ jobs, const int32_t *__restrict__ njobs_p) {
    const int njobs = *njobs_p;
    const int lane = lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int j = 0; j < njobs; ++j) {
        const UpdateJob &J = jobs[j];
        if (MODE == ES_FILTER && job_dead(J)) continue;
        const EsView e = es_view(J, MODE);
        const int32_t n = J.g.n;
        if (e.optr[n] > e.m_limit) continue;
        for (int64_t a = wave; a < n; a += nwaves) {
            const int32_t p0 = e.ptr[a], p1 = e.ptr[a + 1];
            int32_t out = e.optr[a];
            for (int32_t base = p0; base < p1; base += 64) {
                const int32_t i = base + lane;
                bool keep = false;
                int32_t b = 0, w = 0;
                if (i < p1) {
                    b = e.dst[i];
                    w = e.w[i];
                    keep = es_keep(J, MODE, (int32_t)a, b, w);
                }
                const uint64_t mask = __ballot(keep);
                if (keep) {
                    const int32_t o = out + (int32_t)popc_below(mask, lane);
                    e.osrc[o] = (int32_t)a;
                    e.odst[o] = b;
                    e.ow[o] = w;
                }
                out += (int32_t)__popcll(mask);
            }
            if (MODE == ES_MERGE) {
                for (int32_t base = 0; base < J.n_u; base += 64) {
                    const int32_t k = base + lane;
                    const bool hit = (k < J.n_u) && (J.u_tail[k] == a);
                    const uint64_t mask = __ballot(hit);
                    if (hit) {
                        const int32_t o = out + (int32_t)popc_below(mask, lane);
                        e.osrc[o] = (int32_t)a;
                        e.odst[o] = J.u_head[k];
                        e.ow[o] = J.u_w[k];
                    }
                    out += (int32_t)__popcll(mask);
                }
            }
        }
    }
}

// ------------------------------------------------------------ DAG passes ---
//
// One workgroup handles one source s.  DAG(s) is never stored: an arc (a,b)
// of E* is in DAG(s) iff d(s,a) is finite and d(s,a) + w(a,b) = d(s,b)
// (Eq.1; Lemma 3 shows the paper's Update-DAG builds exactly this set).
//   1. in-degrees over the E* arcs (arc-parallel, atomics),
//   2. Kahn rounds from s: a vertex whose last DAG predecessor is consumed
//      joins the next frontier, so the frontiers in order form a topological
//      order with level offsets (any reverse topological order serves the
//      accumulation, Section 2.1),
//   3. levels in reverse: each vertex pulls Eq.4 over its successors,
//      delta(a) = sigma_sa * sum_b (1 + delta(b)) / sigma_sb, summed in the
//      fixed CSR order, so a recomputation is bit-identical.
// MODE_OLD keeps delta in dold; MODE_NEW adds delta' - delta to bc_delta;
// MODE_STATIC also counts paths (sigma_sb = sum of sigma_sa over DAG
// predecessors, pushed in Kahn order) and adds delta to bc_delta;
// MODE_ROW writes delta to dold only (introspection).

struct BlockShared {
    int32_t head, tail, next, nlev;
    int32_t item;
    int32_t flags;
    int32_t scan[40];
    unsigned long long counter;
};

struct Slot {
    int32_t *indeg, *order, *lvl, *queue2;
    double *coef, *dold;
};

__device__ __forceinline__ Slot slot_at(char *base, int32_t n) {
    const SlotLayout L = slot_layout(n);
    Slot s;
    s.indeg = (int32_t *)(base + L.indeg);
    s.order = (int32_t *)(base + L.order);
    s.lvl = (int32_t *)(base + L.lvl);
    s.queue2 = (int32_t *)(base + L.queue2);
    s.coef = (double *)(base + L.coef);
    s.dold = (double *)(base + L.dold);
    return s;
}

template <int MODE>
__device__ void dag_pass(const int32_t s, const int32_t n, const int32_t *Drow, uint64_t *Srow, const int32_t *ptr,
                         const int32_t *src, const int32_t *dst, const int32_t *wt, const int32_t m, const Slot &sl,
                         double *bc_delta, GraphCtl *ctl, BlockShared &sh) {
    const int tid = threadIdx.x, bs = blockDim.x;
    for (int32_t i = tid; i < n; i += bs) {
        sl.indeg[i] = 0;
        if (MODE == MODE_OLD || MODE == MODE_ROW) sl.dold[i] = 0.0;
        if (MODE == MODE_STATIC) Srow[i] = (i == s) ? 1ull : 0ull;
    }
    __syncthreads();
    for (int32_t i = tid; i < m; i += bs) {
        const int32_t a = src[i];
        const int32_t da = Drow[a];
        if (da == INF32) continue;
        const int32_t b = dst[i];
        const int32_t db = Drow[b];
        if (db != INF32 && (int64_t)da + wt[i] == (int64_t)db) atomicAdd(&sl.indeg[b], 1);
    }
    if (tid == 0) {
        sl.order[0] = s;
        sh.head = 0;
        sh.tail = 1;
        sh.next = 1;
        sh.nlev = 0;
    }
    __syncthreads();
    bool ovf = false;
    for (;;) {
        const int32_t lo = sh.head, hi = sh.tail;
        if (lo >= hi) break;
        if (tid == 0) sl.lvl[sh.nlev] = lo;
        for (int32_t idx = lo + tid; idx < hi; idx += bs) {
            const int32_t a = sl.order[idx];
            const int32_t da = Drow[a];
            const uint64_t sa = (MODE == MODE_STATIC) ? Srow[a] : 0ull;
            const int32_t e1 = ptr[a + 1];
            for (int32_t e = ptr[a]; e < e1; ++e) {
                const int32_t b = dst[e];
                const int32_t db = Drow[b];
                if (db != INF32 && (int64_t)da + wt[e] == (int64_t)db) {
                    if (MODE == MODE_STATIC) {
                        const uint64_t old = atomicAdd((unsigned long long *)&Srow[b], (unsigned long long)sa);
                        if (old + sa < old) ovf = true;
                    }
                    if (atomicSub(&sl.indeg[b], 1) == 1) {
                        const int32_t pos = atomicAdd(&sh.next, 1);
                        sl.order[pos] = b;
                    }
                }
            }
        }
        __syncthreads();
        if (tid == 0) {
            sh.head = hi;
            sh.tail = sh.next;
            sh.nlev += 1;
        }
        __syncthreads();
    }
    if (MODE == MODE_STATIC && ovf) atomicOr(&ctl->status, ST_SIGMA_OVF);
    const int32_t nlev = sh.nlev;
    if (tid == 0) {
        sl.lvl[nlev] = sh.tail;
        atomicMax(&ctl->max_levels, nlev);
    }
    __syncthreads();
    for (int32_t L = nlev - 1; L >= 0; --L) {
        const int32_t lo = sl.lvl[L], hi = sl.lvl[L + 1];
        for (int32_t idx = lo + tid; idx < hi; idx += bs) {
            const int32_t a = sl.order[idx];
            const int32_t da = Drow[a];
            double acc = 0.0;
            const int32_t e1 = ptr[a + 1];
            for (int32_t e = ptr[a]; e < e1; ++e) {
                const int32_t b = dst[e];
                const int32_t db = Drow[b];
                if (db != INF32 && (int64_t)da + wt[e] == (int64_t)db) acc += sl.coef[b];
            }
            const double sa = (double)Srow[a];
            const double dl = sa * acc;
            sl.coef[a] = (1.0 + dl) / sa;
            if (a == s) continue;
            if (MODE == MODE_OLD || MODE == MODE_ROW) {
                sl.dold[a] = dl;
            } else if (MODE == MODE_NEW) {
                const double diff = dl - sl.dold[a];
                if (diff != 0.0) atomicAdd(&bc_delta[a], diff);
            } else {
                if (dl != 0.0) atomicAdd(&bc_delta[a], dl);
            }
        }
        __syncthreads();
    }
}

// Row update of one affected source (the all-pairs step of Alg 3 restricted
// to row s).  In phase: Lemma 4 with the old row v.  Out phase (if E_o is not
// empty): Lemma 4 on G'_R, D = d'(s,v) + d''(v,t), with row v''.  sigma is
// read only where a distance test says the pair may change, and only changed
// elements are written.
__device__ void row_update(const UpdateJob &J, const int32_t s, int32_t *Drow_lds, const bool lds, BlockShared &sh) {
    const int tid = threadIdx.x, bs = blockDim.x;
    const int32_t n = J.g.n;
    int32_t *Dg = J.g.D + (size_t)s * n;
    uint64_t *Sg = J.g.S + (size_t)s * n;
    const int32_t *Drow = lds ? Drow_lds : Dg;
    const SrcScal sc = J.g.scal[s];
    const bool same = (sc.flags & 1) != 0;
    const bool has_out = J.n_out > 0;
    const int32_t *rvD = J.row_v_D;
    const uint64_t *rvS = J.row_v_S;
    bool ovf_s = false, ovf_d = false;
    uint32_t changed = 0;
    for (int32_t t = tid; t < n; t += bs) {
        const int32_t d0 = Drow[t];
        int32_t d = d0;
        uint64_t sg = 0;
        bool sg_known = false;
        int64_t c;
        if (in_rule(d0, sc.dv, rvD[t], c)) {
            if (c >= INF32) {
                ovf_d = true;
            } else if (c < d0) {
                d = (int32_t)c;
                sg = mul_chk(sc.sv, rvS[t], ovf_s);
                sg_known = true;
            } else {
                const uint64_t add = mul_chk(same ? sc.hv : sc.sv, rvS[t], ovf_s);
                if (add != 0) {
                    sg = add_chk(Sg[t], add, ovf_s);
                    sg_known = true;
                }
            }
        }
        if (has_out) {
            const int32_t dvv = J.g.rvv_D[t];
            int64_t c2;
            if (in_rule(d, sc.dv, dvv, c2)) {
                if (c2 >= INF32) {
                    ovf_d = true;
                } else if (c2 < d) {
                    d = (int32_t)c2;
                    sg = mul_chk(sc.sv, J.g.rvv_S[t], ovf_s);
                    sg_known = true;
                } else {
                    const uint64_t mult = (dvv == rvD[t]) ? J.g.rvv_H[t] : J.g.rvv_S[t];
                    const uint64_t add = mul_chk(sc.sv, mult, ovf_s);
                    if (add != 0) {
                        sg = add_chk(sg_known ? sg : Sg[t], add, ovf_s);
                        sg_known = true;
                    }
                }
            }
        }
        if (sg_known) {
            Sg[t] = sg;
            if (d != d0) {
                Dg[t] = d;
                if (lds) Drow_lds[t] = d;
            }
            ++changed;
        }
    }
    if (ovf_s) atomicOr(&J.g.ctl->status, ST_SIGMA_OVF);
    if (ovf_d) atomicOr(&J.g.ctl->status, ST_DIST_OVF);
    if (changed) atomicAdd(&sh.counter, (unsigned long long)changed);
}

// Persistent per-source kernel: workgroups pull (job, affected source)
// items from a device counter until every job's list is empty.  Each item:
// old dependencies on E* (buffer X) from the old row, row update, new
// dependencies on the merged E* (buffer Y) from the new row, BC difference.
__global__ void __launch_bounds__(1024) k_source(const UpdateJob *__restrict__ jobs, const int32_t *__restrict__ njobs_p,
                                                 char *__restrict__ scratch, size_t slot_bytes, int32_t lds_cap) {
    extern __shared__ int32_t lds_row[];
    __shared__ BlockShared sh;
    const int njobs = *njobs_p;
    char *slot_base = scratch + (size_t)blockIdx.x * slot_bytes;
    for (int j = 0; j < njobs; ++j) {
        const UpdateJob &J = jobs[j];
        const int32_t n = J.g.n;
        const bool lds = n <= lds_cap;
        const Slot sl = slot_at(slot_base, n);
        GraphCtl *ctl = J.g.ctl;
        if (job_dead(J)) continue;
        const int32_t count = *(volatile int32_t *)&ctl->a_count;
        if (threadIdx.x == 0) sh.counter = 0;
        for (;;) {
            __syncthreads();
            if (threadIdx.x == 0) sh.item = atomicAdd(&ctl->work_next, 1);
            __syncthreads();
            const int32_t item = sh.item;
            if (item >= count) break;
            const int32_t s = J.g.alist[item];
            int32_t *Dg = J.g.D + (size_t)s * n;
            uint64_t *Sg = J.g.S + (size_t)s * n;
            const int32_t *Drow = Dg;
            if (lds) {
                for (int32_t t = threadIdx.x; t < n; t += blockDim.x) lds_row[t] = Dg[t];
                __syncthreads();
                Drow = lds_row;
            }
            dag_pass<MODE_OLD>(s, n, Drow, Sg, J.g.x_ptr, J.g.x_src, J.g.x_dst, J.g.x_w, ctl->es_m, sl, J.g.bc_delta,
                               ctl, sh);
            row_update(J, s, lds_row, lds, sh);
            __syncthreads();
            dag_pass<MODE_NEW>(s, n, Drow, Sg, J.g.y_ptr, J.g.y_src, J.g.y_dst, J.g.y_w, ctl->es_m_tmp, sl,
                               J.g.bc_delta, ctl, sh);
        }
        __syncthreads();
        if (threadIdx.x == 0 && sh.counter) atomicAdd(&ctl->changed_pairs, sh.counter);
    }
}

// ------------------------------------------------------------ commit -------

// BC(x) += bc_delta(x) as a compensated (hi, lo) pair (Knuth's two-sum),
// then clears bc_delta and the per-update counters.
__global__ void __launch_bounds__(256) k_commit(const UpdateJob *__restrict__ jobs, const int32_t *__restrict__ njobs_p,
                                                int32_t replace) {
    const int njobs = *njobs_p;
    for (int j = 0; j < njobs; ++j) {
        const UpdateJob &J = jobs[j];
        const int32_t n = J.g.n;
        for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
            const double d = J.g.bc_delta[t];
            if (replace) {
                J.g.bc_hi[t] = d;
                J.g.bc_lo[t] = 0.0;
            } else if (d != 0.0) {
                const double hi = J.g.bc_hi[t];
                const double s = hi + d;
                const double bp = s - hi;
                double e = (hi - (s - bp)) + (d - bp);
                e += J.g.bc_lo[t];
                const double h2 = s + e;
                J.g.bc_hi[t] = h2;
                J.g.bc_lo[t] = e - (h2 - s);
            }
            J.g.bc_delta[t] = 0.0;
        }
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            GraphCtl *c = J.g.ctl;
            c->affected_last = (unsigned long long)c->a_count;
            c->a_count = 0;
            c->work_next = 0;
            if (!replace) c->updates += 1;
        }
    }
}

// Clears the statistics that accumulate during an update (before k_scan).
__global__ void k_begin(const UpdateJob *__restrict__ jobs, const int32_t *__restrict__ njobs_p) {
    const int njobs = *njobs_p;
    for (int j = threadIdx.x; j < njobs; j += blockDim.x) {
        GraphCtl *c = jobs[j].g.ctl;
        c->changed_pairs = 0;
        c->a_count = 0;
        c->work_next = 0;
    }
}

// ------------------------------------------------------------ static pass --

// Distances from every source: frontier Bellman-Ford with the row in LDS
// (atomicMin relaxations; a vertex improved in a round is queued once for
// the next round).  Positive weights make it converge to d(s,.).
__global__ void __launch_bounds__(1024) k_sssp(const UpdateJob *__restrict__ jobs, char *__restrict__ scratch,
                                               size_t slot_bytes, int32_t lds_cap) {
    extern __shared__ int32_t lds_row[];
    __shared__ BlockShared sh;
    const UpdateJob &J = jobs[0];
    const int32_t n = J.g.n;
    const bool lds = n <= lds_cap;
    const Slot sl = slot_at(scratch + (size_t)blockIdx.x * slot_bytes, n);
    GraphCtl *ctl = J.g.ctl;
    const int tid = threadIdx.x, bs = blockDim.x;
    bool ovf = false;
    for (;;) {
        __syncthreads();
        if (tid == 0) sh.item = atomicAdd(&ctl->work_next, 1);
        __syncthreads();
        const int32_t s = sh.item;
        if (s >= n) break;
        int32_t *Dg = J.g.D + (size_t)s * n;
        int32_t *row = lds ? lds_row : Dg;
        int32_t *flag = sl.indeg;
        for (int32_t i = tid; i < n; i += bs) {
            row[i] = (i == s) ? 0 : INF32;
            flag[i] = 0;
        }
        if (tid == 0) {
            sl.order[0] = s;
            sh.tail = 1;
            sh.next = 0;
        }
        __syncthreads();
        int32_t *cur = sl.order, *nxt = sl.queue2;
        for (;;) {
            const int32_t qlen = sh.tail;
            if (qlen == 0) break;
            for (int32_t idx = tid; idx < qlen; idx += bs) {
                const int32_t a = cur[idx];
                const int32_t da = __atomic_load_n(&row[a], __ATOMIC_RELAXED);
                const int32_t e1 = J.g.arc_ptr[a + 1];
                for (int32_t e = J.g.arc_ptr[a]; e < e1; ++e) {
                    const int32_t b = J.g.arc_dst[e];
                    const int64_t nd = (int64_t)da + J.g.arc_w[e];
                    if (nd >= INF32) { ovf = true; continue; }
                    if ((int32_t)nd < __atomic_load_n(&row[b], __ATOMIC_RELAXED)) {
                        const int32_t old = atomicMin(&row[b], (int32_t)nd);
                        if ((int32_t)nd < old && atomicExch(&flag[b], 1) == 0) {
                            const int32_t pos = atomicAdd(&sh.next, 1);
                            nxt[pos] = b;
                        }
                    }
                }
            }
            __syncthreads();
            const int32_t nl = sh.next;
            for (int32_t idx = tid; idx < nl; idx += bs) flag[nxt[idx]] = 0;
            __syncthreads();
            if (tid == 0) {
                sh.tail = nl;
                sh.next = 0;
            }
            int32_t *tmp = cur;
            cur = nxt;
            nxt = tmp;
            __syncthreads();
        }
        if (lds)
            for (int32_t i = tid; i < n; i += bs) Dg[i] = row[i];
    }
    if (ovf) atomicOr(&ctl->status, ST_DIST_OVF);
}

// Per source after the distances and E* exist: path counts pushed in Kahn
// order (sigma_sb = sum over DAG predecessors a of sigma_sa, Alg 6 step 7),
// then the dependency pull, BC += delta (Alg 1 line 5).
__global__ void __launch_bounds__(1024) k_static(const UpdateJob *__restrict__ jobs, char *__restrict__ scratch,
                                                 size_t slot_bytes, int32_t lds_cap) {
    extern __shared__ int32_t lds_row[];
    __shared__ BlockShared sh;
    const UpdateJob &J = jobs[0];
    const int32_t n = J.g.n;
    const bool lds = n <= lds_cap;
    const Slot sl = slot_at(scratch + (size_t)blockIdx.x * slot_bytes, n);
    GraphCtl *ctl = J.g.ctl;
    if (job_dead(J)) return;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) sh.item = atomicAdd(&ctl->work_next, 1);
        __syncthreads();
        const int32_t s = sh.item;
        if (s >= n) break;
        int32_t *Dg = J.g.D + (size_t)s * n;
        const int32_t *Drow = Dg;
        if (lds) {
            for (int32_t t = threadIdx.x; t < n; t += blockDim.x) lds_row[t] = Dg[t];
            __syncthreads();
            Drow = lds_row;
        }
        dag_pass<MODE_STATIC>(s, n, Drow, J.g.S + (size_t)s * n, J.g.x_ptr, J.g.x_src, J.g.x_dst, J.g.x_w,
                              ctl->es_m, sl, J.g.bc_delta, ctl, sh);
    }
}

__global__ void k_reset_work(GraphCtl *ctl) {
    ctl->work_next = 0;
    ctl->a_count = 0;
}

// ------------------------------------------------------------ introspection

// Dependency row of one source by the same level-ordered accumulation.
__global__ void __launch_bounds__(1024) k_delta_row(const UpdateJob *__restrict__ jobs, int32_t s, char *__restrict__ scratch,
                                                    int32_t lds_cap) {
    extern __shared__ int32_t lds_row[];
    __shared__ BlockShared sh;
    const UpdateJob &J = jobs[0];
    const int32_t n = J.g.n;
    const bool lds = n <= lds_cap;
    const Slot sl = slot_at(scratch, n);
    if (job_dead(J)) return;
    int32_t *Dg = J.g.D + (size_t)s * n;
    const int32_t *Drow = Dg;
    if (lds) {
        for (int32_t t = threadIdx.x; t < n; t += blockDim.x) lds_row[t] = Dg[t];
        __syncthreads();
        Drow = lds_row;
    }
    dag_pass<MODE_ROW>(s, n, Drow, J.g.S + (size_t)s * n, J.g.x_ptr, J.g.x_src, J.g.x_dst, J.g.x_w, J.g.ctl->es_m, sl,
                       nullptr, J.g.ctl, sh);
}

// Arcs of DAG(s): the predicate of Eq.1 over E*.
__global__ void k_dag_arcs(const UpdateJob *__restrict__ jobs, int32_t s, int32_t *out_a, int32_t *out_b, int64_t cap,
                           unsigned long long *cnt) {
    const UpdateJob &J = jobs[0];
    if (job_dead(J)) return;
    const int32_t n = J.g.n, m = J.g.ctl->es_m;
    const int32_t *Drow = J.g.D + (size_t)s * n;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t a = J.g.x_src[i], b = J.g.x_dst[i];
        const int32_t da = Drow[a], db = Drow[b];
        if (da != INF32 && db != INF32 && (int64_t)da + J.g.x_w[i] == (int64_t)db) {
            const unsigned long long k = atomicAdd(cnt, 1ull);
            if ((int64_t)k < cap) {
                out_a[k] = a;
                out_b[k] = b;
            }
        }
    }
}

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Order-independent 2 x 64-bit hash of (D, sigma): sums of mixed
// (index, value) words, which commute, so the result is bit-exact.
__global__ void k_hash(const UpdateJob *__restrict__ jobs, unsigned long long *out) {
    const UpdateJob &J = jobs[0];
    const int64_t nn = (int64_t)J.g.n * J.g.n;
    uint64_t h0 = 0, h1 = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nn; i += (int64_t)gridDim.x * blockDim.x) {
        h0 += mix64(((uint64_t)i << 32) ^ (uint32_t)J.g.D[i] ^ 0x5bd1e995ull);
        h1 += mix64((uint64_t)i * 0x9E3779B97F4A7C15ull + J.g.S[i]);
    }
    for (int d = 32; d >= 1; d >>= 1) {
        h0 += (uint64_t)__shfl_down((unsigned long long)h0, d, 64);
        h1 += (uint64_t)__shfl_down((unsigned long long)h1, d, 64);
    }
    if (lane_id() == 0) {
        atomicAdd(&out[0], (unsigned long long)h0);
        atomicAdd(&out[1], (unsigned long long)h1);
    }
}

}  // namespace bcinc
