// HIP kernels of libbcinc for gfx950 (64-lane wavefronts).
//
// Update pipeline for a batch of jobs (one update on each of several graphs):
//   k_scan        affected sources A and Alg 4 scalars (Eq.6, Eq.7)
//   k_targets     row v'' of the Out phase (Alg 4 on the reverse graph) and
//                 the candidate targets of the update
//   k_es_*        E* (by head) plus the updated arcs (buffer YC)
//   k_source      per affected source: changed targets by Lemma 2 / Lemma 4,
//                 old and new partial dependencies over them, BC difference
//   k_es_*        E*' = arcs of YC whose weight equals their new distance
//   k_commit      BC += difference (compensated), reset counters
// Static pass (initial state and full recompute, Alg 7):
//   k_sssp        distances of every source (frontier Bellman-Ford in LDS)
//   k_es_*        E* = arcs with w(a,b) = d(a,b), by tail (X) and by head (XC)
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
// d'(s,v), sigma'_sv.  An unreachable pair (d0 = INF32) with a finite c is
// always taken, so that a c of 2^31-1 or more reaches the caller's distance
// overflow check.
__device__ __forceinline__ bool in_rule(int32_t d0, int32_t dv, int32_t dvt, int64_t &c) {
    if (dv == INF32 || dvt == INF32) return false;
    c = (int64_t)dv + (int64_t)dvt;
    return c <= (int64_t)d0 || d0 == INF32;
}

// A graph whose E* outgrew its buffers is dead until reloaded: every kernel
// that walks E* row pointers skips it, so no access can leave the buffers.
__device__ __forceinline__ bool job_dead(const UpdateJob &J) {
    return (*(volatile int32_t *)&J.g.ctl->status & ST_ESTAR_CAP) != 0;
}

// A graph with any sticky error holds no valid state until it is recomputed:
// the update kernels after the scan skip it (the bits only ever get set
// during a step, so a kernel that skips a job is never followed by one that
// runs it).
__device__ __forceinline__ bool job_halted(const UpdateJob &J) {
    return *(volatile int32_t *)&J.g.ctl->status != 0;
}

// Unreachable in the 64-bit sums of the scan kernels: far above every sum of
// two finite 31-bit distances, so a finite candidate never equals it.
constexpr int64_t INF64 = INT64_MAX / 4;

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
    for (int j = blockIdx.y; j < njobs; j += gridDim.y) {  // a row of blocks per job
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
                // 64-bit sums with INF64 for unreachable: a candidate of 2^31-1
                // or more is compared like any other and is an overflow only
                // if it wins (it is then the new finite d'(s,v))
                const int64_t d0 = dsv == INF32 ? INF64 : (int64_t)dsv;
                int64_t cur = d0;
                uint64_t sig = Ss[v], hat = 0;
                for (int k = 0; k < n_in; ++k) {
                    const int32_t u = J.in_tail[k];
                    const int32_t du = Ds[u];
                    if (du == INF32) continue;
                    const int64_t c = (int64_t)du + J.in_w[k];
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
                if (cur != INF64 && cur >= INF32) {
                    // d'(s,v) does not fit the distance matrix: the graph is
                    // halted (sticky), s is left out
                    ovf_d = true;
                    cur = d0;
                    hat = 0;
                }
                const bool same = (cur == d0);
                aff = (cur < d0) || (hat != 0);
                if (!aff && cur != INF64) {
                    for (int k = 0; k < n_out; ++k) {
                        const int32_t x = J.out_head[k];
                        int64_t d1 = Ds[x] == INF32 ? INF64 : (int64_t)Ds[x];
                        const int32_t dvx = Dv[x];
                        if (dvx != INF32 && cur + dvx < d1) d1 = cur + dvx;
                        // a candidate of 2^31-1 or more also marks s: the row
                        // kernel's pair update decides with row v'' whether it
                        // wins, and only then raises the overflow
                        const int64_t c = cur + J.out_w[k];
                        if (c <= d1) { aff = true; break; }
                    }
                }
                SrcScal sc;
                sc.dv = cur == INF64 ? INF32 : (int32_t)cur;
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

// ------------------------------------------------------------ k_targets ----

// Row v'' and the candidate targets of an update, one thread per target t.
//
// Row v'' (Section 4, Out phase): with E_o = {(v, x_j)}, Alg 4 on G'_R gives
// d''(v,t) = min(d'(v,t), min_j w'(v,x_j) + d'(x_j,t)) and the counts
// sigma''_vt, sigma-hat''_vt.  The rows x_j of G' are formed on the fly by
// the In-phase rule from the old rows.  The old row v is snapshotted, since
// the source v itself rewrites it during the update.
//
// Candidates: a pair (s,t) can change in the In phase only if
// d'(s,v) + d(v,t) <= d(s,t) with d'(s,v) = d(s,u_j) + w'_j for some in-arc,
// and d(s,t) <= d(s,u_j) + d(u_j,t), hence only if w'_j + d(v,t) <= d(u_j,t)
// (for an arc update this is the target set of the tail u).  It can change in
// the Out phase only if row v'' changed at t (d''(v,t) < d'(v,t), or a tie
// with new paths).  The union T is listed once per update, with row v and
// row v'' at t copied next to it, so each affected source scans T instead of
// its whole row when T is short.  For whole-row scans the two tests are kept
// per target as filter rows: f_out = d''(v,t) on Out candidates, INF32
// elsewhere, and f_any = min(f_in, f_out) with f_in = d(v,t) on In
// candidates, INF32 elsewhere.
__global__ void __launch_bounds__(256) k_targets(const UpdateJob *__restrict__ jobs, const int32_t *__restrict__ njobs_p) {
    const int njobs = *njobs_p;
    for (int j = blockIdx.y; j < njobs; j += gridDim.y) {  // a row of blocks per job
        const UpdateJob &J = jobs[j];
        const int32_t n = J.g.n, v = J.v;
        const int32_t *D = J.g.D;
        const uint64_t *S = J.g.S;
        bool ovf_s = false, ovf_d = false;
        for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < n; base += (int64_t)gridDim.x * blockDim.x) {
            const int32_t t = (int32_t)(base + threadIdx.x);
            bool cand = false, cand_out = false;
            int32_t dvt = INF32, cur = INF32;
            if (t < n) {
                dvt = D[(size_t)v * n + t];
                if (dvt != INF32) {
                    for (int k = 0; k < J.n_in; ++k) {
                        const int32_t dut = D[(size_t)J.in_tail[k] * n + t];
                        if ((int64_t)J.in_w[k] + dvt <= (int64_t)dut) {
                            cand = true;
                            break;
                        }
                    }
                }
                const int32_t f_in = cand ? dvt : INF32;
                cur = dvt;
                if (J.n_out > 0) {
                    const uint64_t svt = S[(size_t)v * n + t];
                    J.g.rv_D[t] = dvt;
                    J.g.rv_S[t] = svt;
                    // 64-bit sums with INF64 for unreachable, as in k_scan:
                    // only a winning candidate of 2^31-1 or more overflows
                    int64_t c64 = dvt == INF32 ? INF64 : (int64_t)dvt;
                    uint64_t sig = svt, hat = 0;
                    for (int k = 0; k < J.n_out; ++k) {
                        const int32_t x = J.out_head[k];
                        const SrcScal sc = J.g.scal[x];
                        int32_t d1 = D[(size_t)x * n + t];
                        uint64_t s1 = 0;
                        bool s1_known = false;
                        int64_t c;
                        if (in_rule(d1, sc.dv, dvt, c)) {
                            // in_rule takes c only where it is shortest: a
                            // c of 2^31-1 or more is a real overflow of (x,t)
                            if (c >= INF32) { ovf_d = true; }
                            else if (c < d1) { d1 = (int32_t)c; s1 = mul_chk(sc.sv, svt, ovf_s); s1_known = true; }
                            else {
                                s1 = add_chk(S[(size_t)x * n + t], mul_chk((sc.flags & 1) ? sc.hv : sc.sv, svt, ovf_s),
                                             ovf_s);
                                s1_known = true;
                            }
                        }
                        if (d1 == INF32) continue;
                        const int64_t cc = (int64_t)J.out_w[k] + d1;
                        if (cc <= c64) {
                            if (!s1_known) s1 = S[(size_t)x * n + t];
                            if (cc == c64) {
                                sig = add_chk(sig, s1, ovf_s);
                                hat = add_chk(hat, s1, ovf_s);
                            } else {
                                c64 = cc;
                                sig = s1;
                                hat = 0;
                            }
                        }
                    }
                    if (c64 != INF64 && c64 >= INF32) {
                        // d''(v,t) does not fit: the graph is halted (sticky)
                        ovf_d = true;
                        c64 = INF64;
                        hat = 0;
                    }
                    cur = c64 == INF64 ? INF32 : (int32_t)c64;
                    J.g.rvv_D[t] = cur;
                    J.g.rvv_S[t] = sig;
                    J.g.rvv_H[t] = hat;
                    cand_out = cur < dvt || hat != 0;
                    cand = cand || cand_out;
                }
                const int32_t f_out = cand_out ? cur : INF32;
                J.g.f_out[t] = f_out;
                J.g.f_any[t] = min(f_in, f_out);
            }
            const uint64_t mask = __ballot(cand);
            if (mask) {
                const int lane = lane_id();
                const int leader = __ffsll((unsigned long long)mask) - 1;
                int32_t b0 = 0;
                if (lane == leader) b0 = atomicAdd(&J.g.ctl->t_count, (int32_t)__popcll(mask));
                b0 = __shfl(b0, leader, 64);
                if (cand) {
                    const int32_t pos = b0 + (int32_t)popc_below(mask, lane);
                    J.g.tlist[pos] = t;
                    J.g.tl_rvD[pos] = dvt;
                    J.g.tl_rvvD[pos] = cur;
                }
            }
        }
        if (ovf_s) atomicOr(&J.g.ctl->status, ST_SIGMA_OVF);
        if (ovf_d) atomicOr(&J.g.ctl->status, ST_DIST_OVF);
    }
}

// ------------------------------------------------------------ E* rebuild ---
//
// E* is kept as segments of arcs keyed by tail (X, built by the static pass
// for its forward Kahn order) or by head (XC, kept current; the update walks
// DAG predecessors).  A wave-per-segment compaction builds X and XC in the
// static pass (see the ES_* enum); an update's merge (k_es_merge) and filter
// (k_es_keep / k_es_wscan / k_es_place) are arc-parallel.  An arc whose
// weight exceeds its distance lies on no
// shortest path and is dropped; distances only decrease under incremental
// updates, so E*' is contained in E* plus the updated arcs (Section 1
// definition of E*; Alg 6 steps 2-4 use the same test w(u,v) = d(u,v)).

struct EsView {
    const int32_t *ptr, *other, *w;  // input segments; other = the non-key endpoint
    bool by_head;                    // key endpoint: head (true) or tail (false)
    int32_t *optr, *osrc, *odst, *ow;
    int32_t m_limit;
    int32_t *m_out;
};

__device__ __forceinline__ EsView es_view(const UpdateJob &J, int mode) {
    EsView e;
    e.m_limit = (int32_t)J.g.es_cap;
    if (mode == ES_BUILD) {
        e.ptr = J.g.arc_ptr; e.other = J.g.arc_dst; e.w = J.g.arc_w; e.by_head = false;
        e.optr = J.g.x_ptr; e.osrc = J.g.x_src; e.odst = J.g.x_dst; e.ow = J.g.x_w;
        e.m_out = &J.g.ctl->es_m;
    } else {
        e.ptr = J.g.arcin_ptr; e.other = J.g.arcin_src; e.w = J.g.arcin_w; e.by_head = true;
        e.optr = J.g.xc_ptr; e.osrc = J.g.xc_src; e.odst = J.g.xc_dst; e.ow = J.g.xc_w;
        e.m_out = &J.g.ctl->esc_m;
    }
    return e;
}

__device__ __forceinline__ bool es_keep(const UpdateJob &J, const EsView &e, int32_t a, int32_t b, int32_t w) {
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

        const EsView e = es_view(J, MODE);
        const int32_t n = J.g.n;
        for (int64_t key = wave; key < n; key += nwaves) {
            const int32_t p0 = e.ptr[key], p1 = e.ptr[key + 1];
            int32_t cnt = 0;
            for (int32_t base = p0; base < p1; base += 64) {
                const int32_t i = base + lane;
                bool keep = false;
                if (i < p1) {
                    const int32_t o = e.other[i];
                    keep = e.by_head ? es_keep(J, e, o, (int32_t)key, e.w[i]) : es_keep(J, e, (int32_t)key, o, e.w[i]);
                }
                cnt += (int32_t)__popcll(__ballot(keep));
            }
            if (lane == 0) J.g.es_cnt[key] = cnt;
        }
    }
}

// One workgroup per job: exclusive scan of the per-segment counts into the
// output segment pointers; the total goes to the control block.  A total
// above the capacity sets the sticky E* capacity error and the scatter is
// skipped.
template <int MODE>
__global__ void __launch_bounds__(1024) k_es_scan(const UpdateJob *__restrict__ jobs, const int32_t *__restrict__ njobs_p) {
    __shared__ int32_t sh[40];
    const int j = blockIdx.x;
    if (j >= *njobs_p) return;
    const UpdateJob &J = jobs[j];

    const EsView e = es_view(J, MODE);
    const int32_t n = J.g.n;
    const int32_t *cnt = J.g.es_cnt;
    // tiles of 8 consecutive counts per thread (two 16-byte loads), one block
    // scan per tile, a running carry between tiles
    int32_t carry = 0;
    for (int32_t base = 0; base < n; base += 8 * (int32_t)blockDim.x) {
        const int32_t i0 = base + 8 * (int32_t)threadIdx.x;
        int32_t v[8];
        const bool whole = i0 + 8 <= n;
        if (whole) {
            const int4 a = *(const int4 *)(cnt + i0), b = *(const int4 *)(cnt + i0 + 4);
            v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
            v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
        } else {
#pragma unroll
            for (int k = 0; k < 8; ++k) v[k] = (i0 + k < n) ? cnt[i0 + k] : 0;
        }
        int32_t local = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) local += v[k];
        int32_t total;
        int32_t off = block_excl_scan(local, sh, total) + carry;
        int32_t o[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            o[k] = off;
            off += v[k];
        }
        if (whole) {
            *(int4 *)(e.optr + i0) = make_int4(o[0], o[1], o[2], o[3]);
            *(int4 *)(e.optr + i0 + 4) = make_int4(o[4], o[5], o[6], o[7]);
        } else {
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (i0 + k < n) e.optr[i0 + k] = o[k];
        }
        carry += total;
    }
    if (threadIdx.x == 0) {
        const int32_t total = carry;
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

        const EsView e = es_view(J, MODE);
        const int32_t n = J.g.n;
        if (e.optr[n] > e.m_limit) continue;
        for (int64_t key = wave; key < n; key += nwaves) {
            const int32_t p0 = e.ptr[key], p1 = e.ptr[key + 1];
            int32_t out = e.optr[key];
            for (int32_t base = p0; base < p1; base += 64) {
                const int32_t i = base + lane;
                bool keep = false;
                int32_t a = 0, b = 0, w = 0;
                if (i < p1) {
                    const int32_t o = e.other[i];
                    a = e.by_head ? o : (int32_t)key;
                    b = e.by_head ? (int32_t)key : o;
                    w = e.w[i];
                    keep = es_keep(J, e, a, b, w);
                }
                const uint64_t mask = __ballot(keep);
                if (keep) {
                    const int32_t o = out + (int32_t)popc_below(mask, lane);
                    e.osrc[o] = a;
                    e.odst[o] = b;
                    e.ow[o] = w;
                }
                out += (int32_t)__popcll(mask);
            }
        }
    }
}

// E* merge in one elementwise pass: YC keeps every XC arc and adds the
// update's arcs behind their head's XC arcs, so head h's segment starts
// before(h) entries later than in XC, before(h) = the update arcs into heads
// below h.  Each XC arc and each update arc is placed directly (the same
// layout the count / scan / scatter passes produce in the other modes).  An
// XC arc that the update lowers stays beside its new copy: its old weight
// satisfies Eq.1 for no source, and the filter drops it.
__global__ void __launch_bounds__(256) k_es_merge(const UpdateJob *__restrict__ jobs, const int32_t *__restrict__ njobs_p) {
    const int njobs = *njobs_p;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
    for (int j = blockIdx.y; j < njobs; j += gridDim.y) {  // a row of blocks per job
        const UpdateJob &J = jobs[j];
        if (job_halted(J)) continue;
        const int32_t n = J.g.n, nu = J.n_u;
        const int32_t *__restrict__ ptr = J.g.xc_ptr;
        const int32_t m = ptr[n];
        const int64_t total = (int64_t)m + nu;
        if (total > J.g.es_cap) {
            if (gid == 0) atomicOr(&J.g.ctl->status, ST_ESTAR_CAP);
            continue;
        }
        if (gid == 0) J.g.ctl->esc_m_tmp = (int32_t)total;
        for (int64_t h = gid; h <= n; h += nthreads) {
            int32_t before = 0;
            for (int k = 0; k < nu; ++k) before += J.u_head[k] < h;
            J.g.yc_ptr[h] = ptr[h] + before;
        }
        for (int64_t i = gid; i < m; i += nthreads) {
            const int32_t h = J.g.xc_dst[i];
            int32_t before = 0;
            for (int k = 0; k < nu; ++k) before += J.u_head[k] < h;
            const int64_t o = i + before;
            J.g.yc_src[o] = J.g.xc_src[i];
            J.g.yc_dst[o] = h;
            J.g.yc_w[o] = J.g.xc_w[i];
        }
        for (int64_t k = gid; k < nu; k += nthreads) {
            const int32_t h = J.u_head[k];
            int32_t before = 0;
            for (int q = 0; q < nu; ++q) before += J.u_head[q] < h || (J.u_head[q] == h && q < k);
            const int64_t o = (int64_t)ptr[h + 1] + before;
            J.g.yc_src[o] = J.u_tail[k];
            J.g.yc_dst[o] = h;
            J.g.yc_w[o] = J.u_w[k];
        }
    }
}

// E* filter, arc-parallel: XC = the arcs of YC with w = d'(a,b), in YC
// order.  One gather per arc sets a bit of a 64-bit keep mask per 64 arcs;
// one workgroup per job scans the masks' popcounts; then every kept arc and
// every head's segment start is placed directly.  The masks and their
// prefix sit in the by-tail E* arrays (X), which only the static pass uses
// and rebuilds before use.
__device__ __forceinline__ uint64_t *es_mask(const UpdateJob &J) { return (uint64_t *)J.g.x_src; }
__device__ __forceinline__ int32_t *es_wpre(const UpdateJob &J) { return J.g.x_dst; }

__global__ void __launch_bounds__(256) k_es_keep(const UpdateJob *__restrict__ jobs, const int32_t *__restrict__ njobs_p) {
    const int njobs = *njobs_p;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
    for (int j = blockIdx.y; j < njobs; j += gridDim.y) {  // a row of blocks per job
        const UpdateJob &J = jobs[j];
        if (job_halted(J)) continue;
        const int32_t n = J.g.n;
        const int64_t m = J.g.yc_ptr[n];
        const int64_t m64 = (m + 63) & ~(int64_t)63;
        uint64_t *const mask = es_mask(J);
        // a wave covers 64 consecutive arcs (the stride is a multiple of 64).
        // A tail outside the affected sources kept its row, so an arc of XC
        // (the front of its head's YC segment: XC's pointers still hold the
        // previous E*) stays without a test; the update's arcs, and the old
        // copy of a lowered arc (whose tail's row did change), are tested.
        for (int64_t i = gid; i < m64; i += nthreads) {
            bool keep = false;
            if (i < m) {
                const int32_t a = J.g.yc_src[i], b = J.g.yc_dst[i];
                const bool affected = (J.g.scal[a].flags & 2) != 0;
                const bool from_xc = i - J.g.yc_ptr[b] < J.g.xc_ptr[b + 1] - J.g.xc_ptr[b];
                keep = (!affected && from_xc) || J.g.D[(size_t)a * n + b] == J.g.yc_w[i];
            }
            const uint64_t word = __ballot(keep);
            if (lane_id() == 0) mask[i >> 6] = word;
        }
    }
}

__global__ void __launch_bounds__(1024) k_es_wscan(const UpdateJob *__restrict__ jobs, const int32_t *__restrict__ njobs_p) {
    __shared__ int32_t sh[40];
    const int j = blockIdx.x;
    if (j >= *njobs_p) return;
    const UpdateJob &J = jobs[j];
    if (job_halted(J)) return;
    const int64_t m = J.g.yc_ptr[J.g.n];
    const int32_t words = (int32_t)((m + 63) >> 6);
    const uint64_t *const mask = es_mask(J);
    int32_t *const wpre = es_wpre(J);
    int32_t carry = 0;
    for (int32_t base = 0; base < words; base += 4 * (int32_t)blockDim.x) {
        const int32_t w0 = base + 4 * (int32_t)threadIdx.x;
        int32_t c[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) c[k] = w0 + k < words ? __popcll(mask[w0 + k]) : 0;
        int32_t total;
        int32_t off = block_excl_scan(c[0] + c[1] + c[2] + c[3], sh, total) + carry;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (w0 + k < words) wpre[w0 + k] = off;
            off += c[k];
        }
        carry += total;
    }
    if (threadIdx.x == 0) {
        wpre[words] = carry;
        J.g.ctl->esc_m = carry;
    }
}

// arcs of YC before position p that are kept
__device__ __forceinline__ int32_t es_kept_before(const uint64_t *mask, const int32_t *wpre, const int64_t p) {
    const int64_t w = p >> 6;
    const int r = (int)(p & 63);
    return wpre[w] + (r ? __popcll(mask[w] & ((1ull << r) - 1)) : 0);
}

__global__ void __launch_bounds__(256) k_es_place(const UpdateJob *__restrict__ jobs, const int32_t *__restrict__ njobs_p) {
    const int njobs = *njobs_p;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
    for (int j = blockIdx.y; j < njobs; j += gridDim.y) {  // a row of blocks per job
        const UpdateJob &J = jobs[j];
        if (job_halted(J)) continue;
        const int32_t n = J.g.n;
        const int64_t m = J.g.yc_ptr[n];
        const uint64_t *const mask = es_mask(J);
        const int32_t *const wpre = es_wpre(J);
        for (int64_t i = gid; i < m; i += nthreads) {
            if (!((mask[i >> 6] >> (i & 63)) & 1)) continue;
            const int32_t o = es_kept_before(mask, wpre, i);
            J.g.xc_src[o] = J.g.yc_src[i];
            J.g.xc_dst[o] = J.g.yc_dst[i];
            J.g.xc_w[o] = J.g.yc_w[i];
        }
        for (int64_t h = gid; h <= n; h += nthreads) J.g.xc_ptr[h] = es_kept_before(mask, wpre, J.g.yc_ptr[h]);
    }
}

// ------------------------------------------------------------ DAG passes ---

struct BlockShared {
    int32_t head, tail, next, nlev;
    int32_t item;
    int32_t nb, nf;
    int32_t ovf, progress;
    int32_t nk, kpos;
    int32_t scan[40];
    unsigned long long counter;
};

struct SSlot {
    int32_t *indeg, *order, *lvl, *queue2;
    double *coef;
};

__device__ __forceinline__ SSlot sslot_at(char *base, int32_t n) {
    const StaticLayout L = static_layout(n);
    SSlot s;
    s.indeg = (int32_t *)(base + L.indeg);
    s.order = (int32_t *)(base + L.order);
    s.lvl = (int32_t *)(base + L.lvl);
    s.queue2 = (int32_t *)(base + L.queue2);
    s.coef = (double *)(base + L.coef);
    return s;
}

// A workgroup's slot.  Slots of the DAG kernel have no B list and no new
// row (null pointers) and an arc record of n arcs; wide-kernel slots have
// all of them, with a record of KARC_PER_VERTEX * n arcs.
struct USlot {
    int32_t *outdeg, *sub, *q1, *q2, *bl_t, *bl_d;
    double *acc;
    uint64_t *bl_s;
    int32_t *kcnt, *kend, *ka, *kb, *kr, *dnew;
    uint64_t *snew;
    int64_t kcap;
};

__device__ __forceinline__ USlot uslot_at(char *base, int32_t n) {
    const UpdateLayout L = update_layout(n);
    USlot u;
    u.outdeg = (int32_t *)(base + L.outdeg);
    u.acc = (double *)(base + L.acc);
    u.sub = (int32_t *)(base + L.sub);
    u.q1 = (int32_t *)(base + L.q1);
    u.q2 = (int32_t *)(base + L.q2);
    u.bl_t = u.bl_d = nullptr;
    u.bl_s = nullptr;
    u.kcnt = (int32_t *)(base + L.kcnt);
    u.kend = (int32_t *)(base + L.kend);
    u.ka = (int32_t *)(base + L.ka);
    u.kb = (int32_t *)(base + L.kb);
    u.kr = (int32_t *)(base + L.kr);
    u.dnew = nullptr;
    u.snew = nullptr;
    u.kcap = L.kcap;
    return u;
}

__device__ __forceinline__ USlot wslot_at(char *base, int32_t n) {
    const WideLayout L = wide_layout(n);
    USlot u;
    u.outdeg = (int32_t *)(base + L.outdeg);
    u.acc = (double *)(base + L.acc);
    u.sub = (int32_t *)(base + L.sub);
    u.q1 = (int32_t *)(base + L.q1);
    u.q2 = (int32_t *)(base + L.q2);
    u.bl_t = (int32_t *)(base + L.bl_t);
    u.bl_d = (int32_t *)(base + L.bl_d);
    u.bl_s = (uint64_t *)(base + L.bl_s);
    u.kcnt = (int32_t *)(base + L.kcnt);
    u.kend = (int32_t *)(base + L.kend);
    u.ka = (int32_t *)(base + L.ka);
    u.kb = (int32_t *)(base + L.kb);
    u.kr = (int32_t *)(base + L.kr);
    u.dnew = (int32_t *)(base + L.dnew);
    u.snew = (uint64_t *)(base + L.snew);
    u.kcap = L.kcap;
    return u;
}

// Whole-DAG pass of the static computation for one source (one workgroup).
// An arc (a,b) of E* is in DAG(s) iff d(s,a) is finite and
// d(s,a) + w(a,b) = d(s,b) (Eq.1).
//   1. in-degrees over the E* arcs (arc-parallel, atomics),
//   2. Kahn rounds from s: a vertex whose last DAG predecessor is consumed
//      joins the next frontier, so the frontiers in order form a topological
//      order with level offsets (any topological order serves, Section 2.1);
//      path counts are pushed along the way, sigma_sb = sum of sigma_sa over
//      the DAG predecessors a (Alg 6, step 7),
//   3. levels in reverse: each vertex pulls Eq.4 over its successors,
//      delta(a) = sigma_sa * sum_b (1 + delta(b)) / sigma_sb, and BC(a) gets
//      delta(a) for a != s (Alg 1).
// Out-degree above which the static pass gives a vertex a whole wave.
constexpr int32_t HEAVY_DEG = 32;

__device__ void static_dag_pass(const int32_t s, const int32_t n, const int32_t *Drow, uint64_t *Srow,
                                int32_t *pred, const int32_t *ptr, const int32_t *src, const int32_t *dst,
                                const int32_t *wt, const int32_t m, const SSlot &sl, double *bc_delta, GraphCtl *ctl,
                                BlockShared &sh) {
    const int tid = threadIdx.x, bs = blockDim.x;
    for (int32_t i = tid; i < n; i += bs) {
        sl.indeg[i] = 0;
        Srow[i] = (i == s) ? 1ull : 0ull;
        pred[i] = PRED_NONE;
    }
    __syncthreads();
    // DAG(s) in-arcs of every vertex (Eq.1 over E*): their count, and the
    // stored predecessor (the first tail to claim the pair, MULTI after that)
    for (int32_t i = tid; i < m; i += bs) {
        const int32_t a = src[i];
        const int32_t da = Drow[a];
        if (da == INF32) continue;
        const int32_t b = dst[i];
        const int32_t db = Drow[b];
        if (db != INF32 && (int64_t)da + wt[i] == (int64_t)db) {
            atomicAdd(&sl.indeg[b], 1);
            if (atomicCAS(&pred[b], PRED_NONE, a) != PRED_NONE) pred[b] = PRED_MULTI;
        }
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
    // A vertex with more than HEAVY_DEG E* out-arcs (a hub of a power-law
    // graph has thousands) is handled by a whole wave, its lanes striding over
    // the arcs; the others by one lane each.  The heavy vertices of a level
    // are listed in queue2 (unused by this pass) as the lanes meet them.
    const int lane = lane_id(), wid = tid >> 6, nw = bs >> 6;
    int32_t *const heavy = sl.queue2;
    // one DAG-arc test of the forward pass: sigma_sb += sigma_sa, and b joins
    // the next level once its last DAG predecessor has pushed
    auto push = [&](const int32_t da, const uint64_t sa, const int32_t e) {
        const int32_t b = dst[e];
        const int32_t db = Drow[b];
        if (db != INF32 && (int64_t)da + wt[e] == (int64_t)db) {
            const uint64_t old = atomicAdd((unsigned long long *)&Srow[b], (unsigned long long)sa);
            if (old + sa < old) ovf = true;
            if (atomicSub(&sl.indeg[b], 1) == 1) sl.order[atomicAdd(&sh.next, 1)] = b;
        }
    };
    for (;;) {
        const int32_t lo = sh.head, hi = sh.tail;
        if (lo >= hi) break;
        if (tid == 0) {
            sl.lvl[sh.nlev] = lo;
            sh.kpos = 0;
        }
        __syncthreads();
        for (int32_t idx = lo + tid; idx < hi; idx += bs) {
            const int32_t a = sl.order[idx];
            const int32_t e0 = ptr[a], e1 = ptr[a + 1];
            if (e1 - e0 > HEAVY_DEG) {
                heavy[atomicAdd(&sh.kpos, 1)] = a;
                continue;
            }
            const int32_t da = Drow[a];
            const uint64_t sa = Srow[a];
            for (int32_t e = e0; e < e1; ++e) push(da, sa, e);
        }
        __syncthreads();
        const int32_t nh = sh.kpos;
        for (int32_t h = wid; h < nh; h += nw) {
            const int32_t a = heavy[h];
            const int32_t da = Drow[a];
            const uint64_t sa = Srow[a];
            const int32_t e1 = ptr[a + 1];
            for (int32_t e = ptr[a] + lane; e < e1; e += 64) push(da, sa, e);
        }
        __syncthreads();
        if (tid == 0) {
            sh.head = hi;
            sh.tail = sh.next;
            sh.nlev += 1;
        }
        __syncthreads();
    }
    if (ovf) atomicOr(&ctl->status, ST_SIGMA_OVF);
    const int32_t nlev = sh.nlev;
    if (tid == 0) {
        sl.lvl[nlev] = sh.tail;
        atomicMax(&ctl->max_levels, nlev);
    }
    __syncthreads();
    // delta(a) from its DAG successors' coefficients (all of a later level)
    auto finish = [&](const int32_t a, const double acc) {
        const double sa = (double)Srow[a];
        const double dl = sa * acc;
        sl.coef[a] = (1.0 + dl) / sa;
        if (a != s && dl != 0.0) atomicAdd(&bc_delta[a], dl);
    };
    for (int32_t L = nlev - 1; L >= 0; --L) {
        const int32_t lo = sl.lvl[L], hi = sl.lvl[L + 1];
        if (tid == 0) sh.kpos = 0;
        __syncthreads();
        for (int32_t idx = lo + tid; idx < hi; idx += bs) {
            const int32_t a = sl.order[idx];
            const int32_t e0 = ptr[a], e1 = ptr[a + 1];
            if (e1 - e0 > HEAVY_DEG) {
                heavy[atomicAdd(&sh.kpos, 1)] = a;
                continue;
            }
            const int32_t da = Drow[a];
            double acc = 0.0;
            for (int32_t e = e0; e < e1; ++e) {
                const int32_t b = dst[e];
                const int32_t db = Drow[b];
                if (db != INF32 && (int64_t)da + wt[e] == (int64_t)db) acc += sl.coef[b];
            }
            finish(a, acc);
        }
        __syncthreads();
        const int32_t nh = sh.kpos;
        for (int32_t h = wid; h < nh; h += nw) {
            const int32_t a = heavy[h];
            const int32_t da = Drow[a];
            double acc = 0.0;
            const int32_t e1 = ptr[a + 1];
            for (int32_t e = ptr[a] + lane; e < e1; e += 64) {
                const int32_t b = dst[e];
                const int32_t db = Drow[b];
                if (db != INF32 && (int64_t)da + wt[e] == (int64_t)db) acc += sl.coef[b];
            }
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
            if (lane == 0) finish(a, acc);
        }
        __syncthreads();
    }
}

// Arc-parallel expansion helpers: the in-arcs of a list of vertices are
// flattened with a block-wide scan of their in-degrees; each lane takes XU
// consecutive arcs and issues their loads together.  Two keep the DAG kernel
// within its 96 registers without spills (four cost six spilled registers
// and were slower).
constexpr int XU = 2;

struct ExpandShared {
    int32_t *off, *vtx, *beg, *dx;
    double *val;
};

// Bytes of expansion arrays per thread (val, off, vtx, beg, dx).
constexpr size_t XB = 24;

// Dynamic LDS of the per-source kernels: the staged row (4 * lds_cap bytes),
// the expansion arrays (XB bytes per thread), then the small-DAG table.
__device__ __forceinline__ ExpandShared expand_at(char *dyn, int32_t lds_cap) {
    ExpandShared es;
    char *p = dyn + align256((size_t)lds_cap * 4);
    es.val = (double *)p;
    es.off = (int32_t *)(p + 8 * blockDim.x);
    es.vtx = es.off + blockDim.x;
    es.beg = es.vtx + blockDim.x;
    es.dx = es.beg + blockDim.x;
    return es;
}

__device__ __forceinline__ int32_t find_owner(const ExpandShared &es, int32_t nv, int32_t j) {
    int32_t lo = 0, hi = nv - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (es.off[mid] <= j) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Arcs jb .. jb+XU-1 of an expansion chunk of nv vertices and total arcs:
// for each, the owning chunk entry iv and the arc id ev (ok false past the
// end).  One binary search, then a forward walk (the arcs are consecutive).
template <int U>
__device__ __forceinline__ void chunk_arcs(const ExpandShared &es, const int32_t nv, const int32_t total,
                                           const int32_t jb, int32_t (&iv)[U], int32_t (&ev)[U], bool (&ok)[U]) {
    int32_t i = find_owner(es, nv, jb);
#pragma unroll
    for (int k = 0; k < U; ++k) {
        const int32_t j = jb + k;
        ok[k] = j < total;
        iv[k] = 0;
        ev[k] = 0;
        if (ok[k]) {
            while (i + 1 < nv && es.off[i + 1] <= j) ++i;
            iv[k] = i;
            ev[k] = es.beg[i] + (j - es.off[i]);
        }
    }
}

// Stored predecessors of the changed pairs (s, t), t in Bt[0..nb), from the
// new row Dnew and the merged E* by head (cptr/csrc/cw): the tail of t's only
// DAG'(s) in-arc, else PRED_MULTI.  A pair whose distance and count did not
// change keeps its DAG in-arcs (a new in-arc, or a tail whose own distance or
// count changed, would change the pair), so these are the only stored
// predecessors an update changes.  One workgroup; arc-parallel, RU arcs per
// lane in flight.
template <int RU>
__device__ void refresh_preds(const int32_t *__restrict__ Dnew, const int32_t *__restrict__ cptr,
                              const int32_t *__restrict__ csrc, const int32_t *__restrict__ cw,
                              const int32_t *__restrict__ Bt, const int32_t nb, int32_t *pred, BlockShared &sh,
                              const ExpandShared &es) {
    const int tid = threadIdx.x, bs = blockDim.x;
    for (int32_t i = tid; i < nb; i += bs) pred[Bt[i]] = PRED_NONE;
    __syncthreads();
    for (int32_t c = 0; c < nb; c += bs) {
        const int32_t idx = c + tid;
        int32_t t = 0, b0 = 0, deg = 0, dt = INF32;
        if (idx < nb) {
            t = Bt[idx];
            b0 = cptr[t];
            deg = cptr[t + 1] - b0;
            dt = Dnew[t];
        }
        int32_t total;
        const int32_t off = block_excl_scan(deg, sh.scan, total);
        es.off[tid] = off;
        es.vtx[tid] = t;
        es.beg[tid] = b0;
        es.dx[tid] = dt;
        __syncthreads();
        const int32_t nv = min(bs, nb - c);
        for (int32_t j0 = tid; j0 < total; j0 += bs * RU) {
            int32_t iv[RU], av[RU], wv[RU];
            bool ok[RU];
#pragma unroll
            for (int k = 0; k < RU; ++k) {
                const int32_t j = j0 + k * bs;
                ok[k] = j < total;
                iv[k] = ok[k] ? find_owner(es, nv, j) : 0;
                const int32_t e = es.beg[iv[k]] + (j - es.off[iv[k]]);
                av[k] = ok[k] ? csrc[e] : 0;
                wv[k] = ok[k] ? cw[e] : 0;
            }
#pragma unroll
            for (int k = 0; k < RU; ++k) {
                if (!ok[k]) continue;
                const int32_t da = Dnew[av[k]];
                if (da != INF32 && (int64_t)da + wv[k] == (int64_t)es.dx[iv[k]]) {
                    int32_t *const p = &pred[es.vtx[iv[k]]];
                    if (atomicCAS(p, PRED_NONE, av[k]) != PRED_NONE) *p = PRED_MULTI;
                }
            }
        }
        __syncthreads();
    }
}

// Partial dependency of source s over a target set B (one workgroup):
//   delta_B(x) = sum_{t in B} delta_st(x)
//              = sum_{w : x in P_s(w)} sigma_sx / sigma_sw * ([w in B] + delta_B(w)),
// Eq.4 with the indicator of B in place of 1.  It is non-zero only on the
// ancestors of B in DAG(s):
//   1. the vertices to visit and their successor counts: either a backward
//      BFS from B over DAG predecessor arcs (E* by head, Eq.1), counting each
//      sub-DAG vertex's successors inside the sub-DAG, or (full) one sweep
//      over all of E* counting every reachable vertex's DAG successors, for
//      large B where the sub-DAG is most of DAG(s) (vertices outside it get
//      delta_B = 0 and change nothing); a full pass in a slot with an arc
//      record also keeps the DAG(s) arcs it finds, grouped by head,
//   2. Kahn from the sinks (a reverse topological order, which serves the
//      accumulation, Section 2.1): each vertex pushes its term to its
//      predecessors once all its successors have pushed to it, over the
//      recorded arcs when there are any, else over its E* in-arcs with the
//      Eq.1 test.
// Targets whose d(s,t) and sigma_st do not change keep the same set of
// shortest paths, so delta_st is unchanged for them and the BC difference of
// source s is delta'_B - delta_B with B the changed targets (Alg 3 re-runs
// the whole accumulation; both give the same BC).
// OUT_ROW: delta_B goes to out[x] (introspection); otherwise
// out[x] += sign * delta_B(x) for x != s (out = the BC difference).
// RU: arcs in flight per lane in the arc-parallel loops (the E* sweep
// included); LU: vertices or recorded arcs in flight per lane in the loops
// over the row, the changed targets and the arc record (each lane issues LU
// independent loads or atomics before it uses any).
template <bool OUT_ROW, int RU, int LU = 1>
__device__ bool restricted_pass(const int32_t s, const int32_t n, const int32_t *__restrict__ Drow,
                                const uint64_t *__restrict__ Srow, const int32_t *__restrict__ cptr,
                                const int32_t *__restrict__ csrc, const int32_t *__restrict__ cdst,
                                const int32_t *__restrict__ cw, const int32_t *__restrict__ Bt, const int32_t nB,
                                const bool full, const USlot &u, const double sign, double *out,
                                const int32_t *__restrict__ pred, int32_t *new_pred, const bool b_pred,
                                BlockShared &sh, const ExpandShared &es) {
    const int tid = threadIdx.x, bs = blockDim.x;
    const int32_t kcap = (int32_t)u.kcap;
    if (tid == 0) {
        sh.next = 0;
        sh.tail = 0;
        sh.nk = 0;
        sh.kpos = 0;
    }
    __syncthreads();
    for (int32_t i0 = tid; i0 < nB; i0 += LU * bs) {
        int32_t tv[LU];
#pragma unroll
        for (int k = 0; k < LU; ++k) tv[k] = i0 + k * bs < nB ? Bt[i0 + k * bs] : s;
        bool live[LU];
#pragma unroll
        for (int k = 0; k < LU; ++k) live[k] = tv[k] != s && Drow[tv[k]] != INF32;
#pragma unroll
        for (int k = 0; k < LU; ++k) {
            if (!live[k]) continue;
            if (full) {
                u.outdeg[tv[k]] = W_B;
            } else {
                u.outdeg[tv[k]] = W_VIS | W_B;
                u.sub[atomicAdd(&sh.next, 1)] = tv[k];
            }
        }
    }
    __syncthreads();
    int32_t nsub;
    bool rec = false;  // Kahn walks recorded arcs
    // a full pass over a B that covers much of the row tests most in-arcs
    // anyway: one coalesced sweep over E* serves it better than the list
    const bool sweep = full && (!pred || (int64_t)nB * 4 >= (int64_t)n);
    if (sweep) {
        // 1. every DAG(s) arc: one more successor of its tail, and (with an
        //    arc record) the arc itself with one more arc into its head
        const int32_t m = cptr[n];
        for (int32_t e0 = tid; e0 < m; e0 += RU * bs) {
            int32_t av[RU], bv[RU], wv[RU];
#pragma unroll
            for (int k = 0; k < RU; ++k) {
                const int32_t e = e0 + k * bs;
                av[k] = 0;
                bv[k] = 0;
                wv[k] = 0;
                if (e < m) {
                    av[k] = csrc[e];
                    bv[k] = cdst[e];
                    wv[k] = cw[e];
                }
            }
#pragma unroll
            for (int k = 0; k < RU; ++k) {
                if (e0 + k * bs >= m) continue;
                const int32_t da = Drow[av[k]];
                if (da != INF32 && (int64_t)da + wv[k] == (int64_t)Drow[bv[k]]) {
                    atomicAdd(&u.outdeg[av[k]], 1);
                    if (kcap > 0) {
                        const int32_t p = atomicAdd(&sh.nk, 1);
                        if (p < kcap) {
                            u.ka[p] = av[k];
                            u.kb[p] = bv[k];
                            atomicAdd(&u.kcnt[bv[k]], 1);
                        }
                    }
                }
            }
        }
    } else if (full) {
        // 1. every reachable vertex's DAG(s) in-arcs: its stored predecessor
        //    (an unchanged pair keeps its DAG in-arcs), else (a changed target,
        //    or two or more in-arcs) Eq.1 over its E* in-arcs, below
        for (int32_t x0 = tid; x0 < n; x0 += LU * bs) {
            int32_t pv[LU];
            bool live[LU];
#pragma unroll
            for (int k = 0; k < LU; ++k) {
                const int32_t x = x0 + k * bs;
                live[k] = false;
                pv[k] = PRED_MULTI;
                if (x < n) {
                    const int32_t dx = Drow[x], o = u.outdeg[x], pr = pred[x];
                    live[k] = x != s && dx != INF32;
                    pv[k] = ((o & W_B) && !b_pred) ? PRED_MULTI : pr;
                }
            }
#pragma unroll
            for (int k = 0; k < LU; ++k) {
                if (!live[k]) continue;
                const int32_t x = x0 + k * bs, p = pv[k];
                if (p >= 0) {
                    atomicAdd(&u.outdeg[p], 1);
                    if (kcap > 0) {
                        const int32_t q = atomicAdd(&sh.nk, 1);
                        if (q < kcap) {
                            u.ka[q] = p;
                            u.kb[q] = x;
                            atomicAdd(&u.kcnt[x], 1);
                        }
                    }
                } else {
                    u.sub[atomicAdd(&sh.next, 1)] = x;
                }
            }
        }
    }
    __syncthreads();
    if (!sweep && !full) {
        // 1. backward walk from B.  A lane follows a chain of stored
        //    predecessors itself (a vertex's one DAG in-arc, then its tail's,
        //    and so on) until it reaches a vertex already in the sub-DAG, or
        //    s, or a vertex with two or more DAG in-arcs.  Those vertices (and
        //    the B vertices whose stored predecessor may not be read) test
        //    their E* in-arcs by Eq.1 in a round of their own, arc-parallel,
        //    and the tails first found there start the next round's walks.
        //    So the rounds follow the vertices with two or more in-arcs along
        //    a path, not its levels.
        int32_t wlo = 0, whi = sh.next;
        bool first = true;
        for (;;) {
            if (tid == 0) sh.head = 0;
            __syncthreads();
            for (int32_t idx = wlo + tid; idx < whi; idx += bs) {
                int32_t x = u.sub[idx];
                int32_t p = PRED_MULTI;
                if (pred && (b_pred || !first || !(u.outdeg[x] & W_B))) p = pred[x];
                for (;;) {
                    if (p < 0) {
                        // s has no DAG in-arc; any other vertex tests E*
                        if (p == PRED_MULTI || x != s) u.q1[atomicAdd(&sh.head, 1)] = x;
                        break;
                    }
                    // p's own predecessor, loaded before the count returns (unused
                    // when p is already in the sub-DAG, as every B vertex is)
                    const int32_t pp = pred[p];
                    const int32_t old = atomicAdd(&u.outdeg[p], 1);
                    if (kcap > 0) {
                        const int32_t k = atomicAdd(&sh.nk, 1);
                        if (k < kcap) {
                            u.ka[k] = p;
                            u.kb[k] = x;
                            atomicAdd(&u.kcnt[x], 1);
                        }
                    }
                    if (old & (W_COUNT | W_VIS)) break;
                    u.sub[atomicAdd(&sh.next, 1)] = p;
                    x = p;
                    p = pp;
                }
            }
            first = false;
            __syncthreads();
            const int32_t nslow = sh.head;
            if (nslow == 0) break;
            wlo = sh.next;
            for (int32_t c = 0; c < nslow; c += bs) {
                const int32_t idx = c + tid;
                int32_t x = 0, b0 = 0, deg = 0, dx = 0;
                if (idx < nslow) {
                    x = u.q1[idx];
                    b0 = cptr[x];
                    deg = cptr[x + 1] - b0;
                    dx = Drow[x];
                }
                int32_t total;
                const int32_t off = block_excl_scan(deg, sh.scan, total);
                es.off[tid] = off;
                es.vtx[tid] = x;
                es.beg[tid] = b0;
                es.dx[tid] = dx;
                __syncthreads();
                const int32_t nv = min(bs, nslow - c);
                for (int32_t jb = tid * RU; jb < total; jb += bs * RU) {
                    int32_t iv[RU], ev[RU], av[RU], wv[RU];
                    bool ok[RU];
                    chunk_arcs(es, nv, total, jb, iv, ev, ok);
#pragma unroll
                    for (int k = 0; k < RU; ++k) {
                        av[k] = ok[k] ? csrc[ev[k]] : 0;
                        wv[k] = ok[k] ? cw[ev[k]] : 0;
                    }
#pragma unroll
                    for (int k = 0; k < RU; ++k) {
                        if (!ok[k]) continue;
                        const int32_t a = av[k];
                        const int32_t da = Drow[a];
                        if (da == INF32 || (int64_t)da + wv[k] != (int64_t)es.dx[iv[k]]) continue;
                        if ((atomicAdd(&u.outdeg[a], 1) & (W_COUNT | W_VIS)) == 0)
                            u.sub[atomicAdd(&sh.next, 1)] = a;
                        if (kcap > 0) {
                            const int32_t p = atomicAdd(&sh.nk, 1);
                            if (p < kcap) {
                                const int32_t x = es.vtx[iv[k]];
                                u.ka[p] = a;
                                u.kb[p] = x;
                                atomicAdd(&u.kcnt[x], 1);
                            }
                        }
                    }
                }
                __syncthreads();
            }
            whi = sh.next;
        }
    } else if (!sweep) {
        // 1. one round over the vertices to test (a full pass: the others
        //    took their stored predecessor above), arc-parallel.  B vertices
        //    (always) and vertices with two or more DAG in-arcs test their E*
        //    in-arcs by Eq.1.
        int32_t lo = 0, hi = sh.next;
        __syncthreads();
        while (lo < hi) {
            if (tid == 0) sh.head = 0;
            __syncthreads();
            // the stored arcs first, one lane per vertex; the vertices that
            // test E* in-arcs go to the level's general list (the Kahn queue,
            // idle until the walk ends)
            for (int32_t idx = lo + tid; idx < hi; idx += bs) {
                const int32_t x = u.sub[idx];
                const int32_t p = (pred && (b_pred || !(u.outdeg[x] & W_B))) ? pred[x] : PRED_MULTI;
                if (p < 0) {
                    u.q1[atomicAdd(&sh.head, 1)] = x;
                    continue;
                }
                if ((atomicAdd(&u.outdeg[p], 1) & (W_COUNT | W_VIS)) == 0 && !full)
                    u.sub[atomicAdd(&sh.next, 1)] = p;
                if (kcap > 0) {
                    const int32_t k = atomicAdd(&sh.nk, 1);
                    if (k < kcap) {
                        u.ka[k] = p;
                        u.kb[k] = x;
                        atomicAdd(&u.kcnt[x], 1);
                    }
                }
            }
            __syncthreads();
            const int32_t nslow = sh.head;
            for (int32_t c = 0; c < nslow; c += bs) {
                const int32_t idx = c + tid;
                int32_t x = 0, b0 = 0, deg = 0, dx = 0;
                if (idx < nslow) {
                    x = u.q1[idx];
                    b0 = cptr[x];
                    deg = cptr[x + 1] - b0;
                    dx = Drow[x];
                }
                int32_t total;
                const int32_t off = block_excl_scan(deg, sh.scan, total);
                es.off[tid] = off;
                es.vtx[tid] = x;
                es.beg[tid] = b0;
                es.dx[tid] = dx;
                __syncthreads();
                const int32_t nv = min(bs, nslow - c);
                for (int32_t jb = tid * RU; jb < total; jb += bs * RU) {
                    int32_t iv[RU], ev[RU], av[RU], wv[RU];
                    bool ok[RU];
                    chunk_arcs(es, nv, total, jb, iv, ev, ok);
#pragma unroll
                    for (int k = 0; k < RU; ++k) {
                        av[k] = ok[k] ? csrc[ev[k]] : 0;
                        wv[k] = ok[k] ? cw[ev[k]] : 0;
                    }
#pragma unroll
                    for (int k = 0; k < RU; ++k) {
                        if (!ok[k]) continue;
                        const int32_t a = av[k];
                        const int32_t da = Drow[a];
                        if (da == INF32 || (int64_t)da + wv[k] != (int64_t)es.dx[iv[k]]) continue;
                        // one more successor inside the sub-DAG; the first arc
                        // found into a vertex not yet seen adds it to the list
                        // (a full pass has every vertex already)
                        if ((atomicAdd(&u.outdeg[a], 1) & (W_COUNT | W_VIS)) == 0 && !full)
                            u.sub[atomicAdd(&sh.next, 1)] = a;
                        if (kcap > 0) {
                            const int32_t p = atomicAdd(&sh.nk, 1);
                            if (p < kcap) {
                                const int32_t x = es.vtx[iv[k]];
                                u.ka[p] = a;
                                u.kb[p] = x;
                                atomicAdd(&u.kcnt[x], 1);
                            }
                        }
                    }
                }
                __syncthreads();
            }
            lo = hi;
            hi = full ? hi : sh.next;
            __syncthreads();
        }
    }
    if (full) {
        const int32_t nk = sh.nk;
        rec = kcap > 0 && nk <= kcap;
        if (rec) {
            // group the arcs by head: each head with arcs gets a range
            // [kend - kcnt, kend); the scatter advances kend from its start
            for (int32_t x0 = tid; x0 < n; x0 += LU * bs) {
                int32_t cv[LU];
#pragma unroll
                for (int k = 0; k < LU; ++k) cv[k] = x0 + k * bs < n ? u.kcnt[x0 + k * bs] : 0;
#pragma unroll
                for (int k = 0; k < LU; ++k)
                    if (cv[k]) u.kend[x0 + k * bs] = atomicAdd(&sh.kpos, cv[k]);
            }
            __syncthreads();
            for (int32_t p0 = tid; p0 < nk; p0 += LU * bs) {
                int32_t hv[LU], tv[LU], pos[LU];
#pragma unroll
                for (int k = 0; k < LU; ++k) {
                    const int32_t q = p0 + k * bs;
                    hv[k] = q < nk ? u.kb[q] : -1;
                    tv[k] = q < nk ? u.ka[q] : 0;
                }
#pragma unroll
                for (int k = 0; k < LU; ++k) pos[k] = hv[k] >= 0 ? atomicAdd(&u.kend[hv[k]], 1) : 0;
#pragma unroll
                for (int k = 0; k < LU; ++k)
                    if (hv[k] >= 0) u.kr[pos[k]] = tv[k];
            }
        } else if (kcap > 0) {
            // too many arcs to record: Kahn tests E*; undo the counts
            for (int32_t p = tid; p < kcap; p += bs) u.kcnt[u.kb[p]] = 0;
        }
        __syncthreads();
        if (tid == 0) sh.tail = 0;
        __syncthreads();
        for (int32_t x0 = tid; x0 < n; x0 += LU * bs) {
            bool sink[LU];
#pragma unroll
            for (int k = 0; k < LU; ++k) {
                const int32_t x = x0 + k * bs;
                sink[k] = false;
                if (x < n) {
                    const int32_t dx = Drow[x], o = u.outdeg[x];
                    sink[k] = dx != INF32 && (o & W_COUNT) == 0;
                }
            }
#pragma unroll
            for (int k = 0; k < LU; ++k)
                if (sink[k]) u.q1[atomicAdd(&sh.tail, 1)] = x0 + k * bs;
        }
        nsub = n;
    } else {
        nsub = sh.next;
        const int32_t nk = sh.nk;
        rec = kcap > 0 && nk <= kcap;
        if (rec) {
            // group the recorded arcs by head (the sub-DAG vertices)
            for (int32_t i = tid; i < nsub; i += bs) {
                const int32_t x = u.sub[i];
                const int32_t c = u.kcnt[x];
                if (c) u.kend[x] = atomicAdd(&sh.kpos, c);
            }
            __syncthreads();
            for (int32_t p = tid; p < nk; p += bs) u.kr[atomicAdd(&u.kend[u.kb[p]], 1)] = u.ka[p];
        } else if (kcap > 0) {
            for (int32_t p = tid; p < kcap; p += bs) u.kcnt[u.kb[p]] = 0;
        }
        __syncthreads();
        if (tid == 0) sh.tail = 0;
        __syncthreads();
        for (int32_t i = tid; i < nsub; i += bs) {
            const int32_t x = u.sub[i];
            if ((u.outdeg[x] & W_COUNT) == 0) u.q1[atomicAdd(&sh.tail, 1)] = x;
        }
    }
    __syncthreads();
    // 2. Kahn from the sinks
    int32_t qn = sh.tail;
    int32_t *qa = u.q1, *qb = u.q2;
    __syncthreads();
    while (qn > 0) {
        if (tid == 0) {
            sh.tail = 0;
            sh.kpos = 0;
        }
        __syncthreads();
        int32_t nslow = qn;
        const int32_t *slow = qa;
        if (pred || rec) {
            // a vertex with one DAG in-arc (a, x): sigma_sx = sigma_sa, so a
            // receives [x in B] + acc(x) itself (no count, no scan).  Its
            // tail is the stored predecessor for a vertex outside B, else
            // the one recorded arc.  The others go to the back of the next
            // round's queue (the two never meet: a vertex queued for the
            // next round is not in this one) for the general step.
            for (int32_t idx = tid; idx < qn; idx += bs) {
                const int32_t x = qa[idx];
                const bool in_b = (u.outdeg[x] & W_B) != 0;
                int32_t p = (pred && (b_pred || !in_b)) ? pred[x] : PRED_MULTI;
                if (p < 0 && rec && u.kcnt[x] == 1) p = u.kr[u.kend[x] - 1];
                if (p < 0) {
                    qb[n - 1 - atomicAdd(&sh.kpos, 1)] = x;
                    continue;
                }
                const double ax = u.acc[x];
                if (x != s && ax != 0.0) {
                    if (OUT_ROW) out[x] = ax;
                    else atomicAdd(&out[x], sign * ax);
                }
                const double push = (in_b ? 1.0 : 0.0) + ax;
                if (push != 0.0) atomicAdd(&u.acc[p], push);
                if ((atomicSub(&u.outdeg[p], 1) & W_COUNT) == 1) qb[atomicAdd(&sh.tail, 1)] = p;
            }
            __syncthreads();
            nslow = sh.kpos;
            slow = qb + n - nslow;
        }
        for (int32_t c = 0; c < nslow; c += bs) {
            const int32_t idx = c + tid;
            int32_t x = 0, b0 = 0, deg = 0, dx = 0;
            double coef = 0.0;
            if (idx < nslow) {
                x = slow[idx];
                const double ax = u.acc[x];
                if (x != s && ax != 0.0) {
                    if (OUT_ROW) out[x] = ax;
                    else atomicAdd(&out[x], sign * ax);
                }
                // each predecessor a receives sigma_sa * coef
                coef = (((u.outdeg[x] & W_B) ? 1.0 : 0.0) + ax) / (double)Srow[x];
                if (rec) {
                    deg = u.kcnt[x];
                    b0 = deg ? u.kend[x] - deg : 0;
                } else {
                    b0 = cptr[x];
                    deg = cptr[x + 1] - b0;
                }
                dx = Drow[x];
            }
            int32_t total;
            const int32_t off = block_excl_scan(deg, sh.scan, total);
            es.off[tid] = off;
            es.vtx[tid] = x;
            es.beg[tid] = b0;
            es.dx[tid] = dx;
            es.val[tid] = coef;
            __syncthreads();
            const int32_t nv = min(bs, nslow - c);
            for (int32_t jb = tid * RU; jb < total; jb += bs * RU) {
                int32_t iv[RU], ev[RU], av[RU], wv[RU];
                bool ok[RU];
                chunk_arcs(es, nv, total, jb, iv, ev, ok);
#pragma unroll
                for (int k = 0; k < RU; ++k) {
                    av[k] = ok[k] ? (rec ? u.kr[ev[k]] : csrc[ev[k]]) : 0;
                    wv[k] = (ok[k] && !rec) ? cw[ev[k]] : 0;
                }
                double cf[RU];
#pragma unroll
                for (int k = 0; k < RU; ++k) {
                    cf[k] = 0.0;
                    if (!ok[k]) continue;
                    if (!rec) {
                        const int32_t da = Drow[av[k]];
                        ok[k] = da != INF32 && (int64_t)da + wv[k] == (int64_t)es.dx[iv[k]];
                    }
                    if (ok[k]) cf[k] = es.val[iv[k]];
                }
                uint64_t sa[RU];
#pragma unroll
                for (int k = 0; k < RU; ++k) sa[k] = (ok[k] && cf[k] != 0.0) ? Srow[av[k]] : 0;
#pragma unroll
                for (int k = 0; k < RU; ++k) {
                    if (!ok[k]) continue;
                    const int32_t a = av[k];
                    if (cf[k] != 0.0) atomicAdd(&u.acc[a], (double)sa[k] * cf[k]);
                    if ((atomicSub(&u.outdeg[a], 1) & W_COUNT) == 1) qb[atomicAdd(&sh.tail, 1)] = a;
                }
            }
            __syncthreads();
        }
        qn = sh.tail;
        int32_t *tmp = qa;
        qa = qb;
        qb = tmp;
        __syncthreads();
    }
    // the new stored predecessors of the changed targets: every E* in-arc of
    // a B vertex was tested, so its recorded in-arcs are all its DAG in-arcs
    const bool preds_done = rec && new_pred != nullptr;
    if (preds_done) {
        for (int32_t i0 = tid; i0 < nB; i0 += LU * bs) {
            int32_t tv[LU], cv[LU], ev[LU];
            bool live[LU];
#pragma unroll
            for (int k = 0; k < LU; ++k) tv[k] = i0 + k * bs < nB ? Bt[i0 + k * bs] : s;
#pragma unroll
            for (int k = 0; k < LU; ++k) {
                live[k] = false;
                cv[k] = 0;
                ev[k] = 0;
                if (tv[k] != s) {
                    const int32_t dt = Drow[tv[k]];
                    cv[k] = u.kcnt[tv[k]];
                    ev[k] = u.kend[tv[k]];
                    live[k] = dt != INF32;
                }
            }
#pragma unroll
            for (int k = 0; k < LU; ++k) {
                if (!live[k]) continue;
                new_pred[tv[k]] = cv[k] == 1 ? u.kr[ev[k] - 1] : cv[k] == 0 ? PRED_NONE : PRED_MULTI;
            }
        }
        __syncthreads();
    }
    if (full) {
        for (int32_t x = tid; x < n; x += bs) {
            u.outdeg[x] = 0;
            u.acc[x] = 0.0;
            if (rec) u.kcnt[x] = 0;
        }
    } else {
        for (int32_t i = tid; i < nsub; i += bs) {
            const int32_t x = u.sub[i];
            u.outdeg[x] = 0;
            u.acc[x] = 0.0;
            if (rec) u.kcnt[x] = 0;
        }
    }
    __syncthreads();
    return preds_done;
}

// Small sub-DAGs in LDS.  Most sources' sub-DAGs hold a few dozen vertices,
// so the partial-dependency pass keeps their per-vertex state in an
// open-addressing hash table in LDS (with d(s,x) and sigma_sx cached), records
// the sub-DAG's arcs while discovering it, and runs the Kahn rounds over that
// arc list without touching global memory.  Only the E* in-arcs and the
// predecessors' distances are read from global memory.  A sub-DAG that
// outgrows the table is redone by restricted_pass (nothing global has been
// written by then).
// Table sizes of the LDS passes are a template parameter TS (a power of two
// of at most 256, so a slot fits a byte): TS hash slots, 3/4 of them admitted
// as vertices (load factor 3/4), 2 TS sub-DAG arcs.  Smaller tables let more
// workgroups share a CU; larger ones fall back to global memory less often.
#define SD_CONSTS                          \
    constexpr int SD_SLOTS = TS;           \
    constexpr int SD_CAP = TS * 3 / 4;     \
    constexpr int SD_ARCS = 2 * TS;

struct SmallDag {
    int32_t *key, *flags, *outdeg, *dval, *round;
    double *acc, *coef;
    uint64_t *sval;
    int16_t *sub, *arc_a, *arc_x;
};

template <int TS>
__host__ __device__ constexpr size_t small_dag_bytes() {
    SD_CONSTS
    return (size_t)SD_SLOTS * (5 * 4 + 3 * 8 + 2) + (size_t)SD_ARCS * 4 + 256;
}

template <int TS>
__device__ __forceinline__ SmallDag small_dag_at(char *p) {
    SD_CONSTS
    SmallDag d;
    d.acc = (double *)p;             p += 8 * SD_SLOTS;
    d.coef = (double *)p;            p += 8 * SD_SLOTS;
    d.sval = (uint64_t *)p;          p += 8 * SD_SLOTS;
    d.key = (int32_t *)p;            p += 4 * SD_SLOTS;
    d.flags = (int32_t *)p;          p += 4 * SD_SLOTS;
    d.outdeg = (int32_t *)p;         p += 4 * SD_SLOTS;
    d.dval = (int32_t *)p;           p += 4 * SD_SLOTS;
    d.round = (int32_t *)p;          p += 4 * SD_SLOTS;
    d.sub = (int16_t *)p;            p += 2 * SD_SLOTS;
    d.arc_a = (int16_t *)p;          p += 2 * SD_ARCS;
    d.arc_x = (int16_t *)p;
    return d;
}

// Slot of vertex x, inserting it if absent; -1 if the table is full.
template <int TS>
__device__ __forceinline__ int32_t sd_slot(const SmallDag &d, int32_t x, bool &inserted) {
    SD_CONSTS
    uint32_t h = ((uint32_t)x * 2654435761u) >> 24;
    inserted = false;
    for (int p = 0; p < SD_SLOTS; ++p) {
        const int32_t slot = (int32_t)((h + (uint32_t)p) & (SD_SLOTS - 1));
        const int32_t prev = atomicCAS(&d.key[slot], -1, x);
        if (prev == -1) {
            inserted = true;
            return slot;
        }
        if (prev == x) return slot;
    }
    return -1;
}

// The partial dependency of restricted_pass with all per-vertex state in
// LDS.  Returns false (and leaves global memory untouched) if the sub-DAG
// does not fit.
// One arc (a, x) of the LDS walk (x in slot sxv, da = d(s,a)): recorded,
// a's successor count raised, and a queued at its first sight.
template <int TS>
__device__ __forceinline__ void sd_add_arc(const SmallDag &d, BlockShared &sh, const int32_t a, const int32_t sxv,
                                           const int32_t da, const uint64_t *__restrict__ Srow) {
    SD_CONSTS
    bool ins;
    const int32_t sa = sd_slot<TS>(d, a, ins);
    const int32_t k = atomicAdd(&sh.tail, 1);
    if (sa < 0 || k >= SD_ARCS) {
        sh.ovf = 1;
        return;
    }
    d.arc_a[k] = (int16_t)sa;
    d.arc_x[k] = (int16_t)sxv;
    atomicAdd(&d.outdeg[sa], 1);
    if ((atomicOr(&d.flags[sa], F_VIS) & F_VIS) == 0) {
        d.dval[sa] = da;
        d.sval[sa] = Srow[a];
        const int32_t pos = atomicAdd(&sh.next, 1);
        if (pos >= SD_CAP) sh.ovf = 1;
        else d.sub[pos] = (int16_t)sa;
    }
}

template <int TS>
__device__ bool small_pass(const int32_t s, const int32_t *__restrict__ Drow, const uint64_t *__restrict__ Srow,
                           const int32_t *__restrict__ cptr, const int32_t *__restrict__ csrc,
                           const int32_t *__restrict__ cw, const int32_t *__restrict__ Bt, const int32_t nB,
                           const double sign, double *out, const int32_t *__restrict__ pred, const bool b_pred,
                           BlockShared &sh, const ExpandShared &es, const SmallDag &d) {
    SD_CONSTS
    const int tid = threadIdx.x, bs = blockDim.x;
    for (int32_t i = tid; i < SD_SLOTS; i += bs) {
        d.key[i] = -1;
        d.flags[i] = 0;
        d.outdeg[i] = 0;
        d.acc[i] = 0.0;
        d.round[i] = -1;
    }
    if (tid == 0) {
        sh.next = 0;
        sh.tail = 0;  // arcs
        sh.ovf = 0; // overflow
    }
    __syncthreads();
    for (int32_t i = tid; i < nB; i += bs) {
        const int32_t t = Bt[i];
        const int32_t dt = Drow[t];
        if (t == s || dt == INF32) continue;
        bool ins;
        const int32_t slot = sd_slot<TS>(d, t, ins);
        const int32_t pos = atomicAdd(&sh.next, 1);
        if (slot < 0 || pos >= SD_CAP) {
            sh.ovf = 1;
            continue;
        }
        d.flags[slot] = F_VIS | F_B;
        d.dval[slot] = dt;
        d.sval[slot] = Srow[t];
        d.sub[pos] = (int16_t)slot;
    }
    __syncthreads();
    if (sh.ovf) return false;
    int32_t lo = 0, hi = sh.next;
    __syncthreads();
    while (lo < hi) {
        if (tid == 0) sh.head = 0;
        __syncthreads();
        // a vertex with one stored predecessor (outside B, or any with
        // b_pred): that arc, at once; the others (their E* in-arcs tested)
        // listed in d.round, idle until the accumulation
        for (int32_t idx = lo + tid; idx < hi; idx += bs) {
            const int32_t sx = d.sub[idx];
            const int32_t x = d.key[sx];
            const int32_t p = (pred && (b_pred || !(d.flags[sx] & F_B))) ? pred[x] : PRED_MULTI;
            if (p < 0) {
                d.round[atomicAdd(&sh.head, 1)] = sx;
                continue;
            }
            sd_add_arc<TS>(d, sh, p, sx, Drow[p], Srow);
        }
        __syncthreads();
        const int32_t nslow = sh.head;
        for (int32_t c = 0; c < nslow; c += bs) {
            const int32_t idx = c + tid;
            int32_t sx = 0, b0 = 0, deg = 0;
            if (idx < nslow) {
                sx = d.round[idx];
                const int32_t x = d.key[sx];
                b0 = cptr[x];
                deg = cptr[x + 1] - b0;
            }
            int32_t total;
            const int32_t off = block_excl_scan(deg, sh.scan, total);
            es.off[tid] = off;
            es.vtx[tid] = sx;
            es.beg[tid] = b0;
            __syncthreads();
            const int32_t nv = min(bs, nslow - c);
            for (int32_t j = tid; j < total; j += bs) {
                const int32_t i = find_owner(es, nv, j);
                const int32_t sxv = es.vtx[i];
                const int32_t e = es.beg[i] + (j - es.off[i]);
                const int32_t a = csrc[e];
                const int32_t da = Drow[a];
                if (da != INF32 && (int64_t)da + cw[e] == (int64_t)d.dval[sxv]) sd_add_arc<TS>(d, sh, a, sxv, da, Srow);
            }
            __syncthreads();
        }
        const bool ovf = sh.ovf != 0;
        lo = hi;
        hi = sh.next;
        __syncthreads();
        if (ovf) return false;
    }
    const int32_t nsub = hi, narcs = sh.tail;
    for (int32_t i = tid; i < SD_SLOTS; i += bs) d.round[i] = -1;
    __syncthreads();
    // Kahn from the sinks over the recorded arcs, all in LDS.  Round r makes
    // final the vertices whose successors all became final before r.
    for (int32_t i = tid; i < nsub; i += bs) {
        const int32_t sx = d.sub[i];
        if (d.outdeg[sx] == 0) d.round[sx] = 0;
    }
    __syncthreads();
    for (int32_t r = 0;; ++r) {
        if (tid == 0) sh.progress = 0;
        __syncthreads();
        // the vertices final in round r publish their coefficient and BC term
        for (int32_t i = tid; i < nsub; i += bs) {
            const int32_t sx = d.sub[i];
            if (d.round[sx] != r) continue;
            const double ax = d.acc[sx];
            const int32_t x = d.key[sx];
            if (x != s && ax != 0.0) atomicAdd(&out[x], sign * ax);
            d.coef[sx] = (((d.flags[sx] & F_B) ? 1.0 : 0.0) + ax) / (double)d.sval[sx];
            sh.progress = 1;
        }
        __syncthreads();
        if (sh.progress == 0) break;
        // and push to their predecessors
        for (int32_t k = tid; k < narcs; k += bs) {
            const int32_t sx = d.arc_x[k];
            if (d.round[sx] != r) continue;
            const int32_t sa = d.arc_a[k];
            atomicAdd(&d.acc[sa], (double)d.sval[sa] * d.coef[sx]);
            if (atomicSub(&d.outdeg[sa], 1) == 1) d.round[sa] = r + 1;
        }
        __syncthreads();
    }
    return true;
}

// Old and new partial dependency of one source in one traversal (LDS only).
// The vertices to visit are the union of the old sub-DAG (ancestors of B in
// DAG(s)) and the new one (ancestors of B in DAG'(s)); both are walked back
// from B level by level at once, so the dependent gathers of a level serve
// both.  The new distances and path counts are those of the B list for
// targets in B and the old ones elsewhere, so D and sigma are not written
// before the new pass.  Over the merged E* segment of a head x (E* by head,
// with the update's arcs appended), the first |E*(x)| arcs are the old E*
// arcs with their old weights: the old Eq.1 test looks at those only, the new
// test at all of them (an old-weight copy of a lowered arc cannot pass it).
// The two Kahn accumulations then run over the recorded arcs, and BC gets the
// difference delta'_B - delta_B once per vertex.  Returns false, before
// anything global is written, when the union does not fit.
#define DD_CONSTS                          \
    constexpr int DD_SLOTS = TS;           \
    constexpr int DD_CAP = TS * 3 / 4;     \
    constexpr int DD_ARCS = 2 * TS;        \
    constexpr int DD_FRONT = 2 * DD_CAP;
enum : int32_t { DF_O = 1, DF_N = 2, DF_B = 4 };

struct DualDag {
    int32_t *key, *flags, *cnt, *dold, *dnew, *round, *pr, *ybeg, *ydeg, *xdeg, *front, *slow, *arcs;
    double *acc_o, *acc_n, *coef;
    uint64_t *sold, *snew;
    // after the walk: the recorded arcs grouped by head (harc over ybeg and
    // ydeg, 2 * TS entries), each head's range end (hend over slow) and
    // in-arc count (hdeg over xdeg), and the Kahn work list (over coef)
    int32_t *harc, *hend, *hdeg, *klist;
};

template <int TS>
__host__ __device__ constexpr size_t dual_dag_bytes() {
    DD_CONSTS
    return (size_t)DD_SLOTS * (10 * 4 + 5 * 8) + (size_t)DD_FRONT * 8 + (size_t)DD_ARCS * 4 + 256;
}

template <int TS>
__device__ __forceinline__ DualDag dual_dag_at(char *p) {
    DD_CONSTS
    DualDag d;
    d.acc_o = (double *)p;    p += 8 * DD_SLOTS;
    d.acc_n = (double *)p;    p += 8 * DD_SLOTS;
    d.coef = (double *)p;     p += 8 * DD_SLOTS;
    d.sold = (uint64_t *)p;   p += 8 * DD_SLOTS;
    d.snew = (uint64_t *)p;   p += 8 * DD_SLOTS;
    d.key = (int32_t *)p;     p += 4 * DD_SLOTS;
    d.flags = (int32_t *)p;   p += 4 * DD_SLOTS;
    d.cnt = (int32_t *)p;     p += 4 * DD_SLOTS;  // successors: old in bits 0-15, new in 16-31
    d.dold = (int32_t *)p;    p += 4 * DD_SLOTS;
    d.dnew = (int32_t *)p;    p += 4 * DD_SLOTS;
    d.round = (int32_t *)p;   p += 4 * DD_SLOTS;
    d.pr = (int32_t *)p;      p += 4 * DD_SLOTS;  // stored (old) predecessor
    d.ybeg = (int32_t *)p;    p += 4 * DD_SLOTS;  // changed targets: merged E* in-arcs (start,
    d.ydeg = (int32_t *)p;    p += 4 * DD_SLOTS;  // count,
    d.xdeg = (int32_t *)p;    p += 4 * DD_SLOTS;  // and how many are old E* arcs)
    d.front = (int32_t *)p;   p += 4 * DD_FRONT;  // slot | memberships to expand << 16; after the walk
                                                  // the new stored predecessor of each changed target
    d.slow = (int32_t *)p;    p += 4 * DD_FRONT;  // a level's entries for the general expansion
    d.arcs = (int32_t *)p;                        // tail slot | head slot << 8 | kinds << 16
    d.harc = d.ybeg;
    d.hend = d.slow;
    d.hdeg = d.xdeg;
    d.klist = (int32_t *)d.coef;
    return d;
}

template <int TS>
__device__ __forceinline__ int32_t dd_find(const DualDag &d, int32_t x) {
    DD_CONSTS
    uint32_t h = ((uint32_t)x * 2654435761u) >> 24;
    for (int p = 0; p < DD_SLOTS; ++p) {
        const int32_t slot = (int32_t)((h + (uint32_t)p) & (DD_SLOTS - 1));
        const int32_t k = d.key[slot];
        if (k == x) return slot;
        if (k == -1) return -1;
    }
    return -1;
}

template <int TS>
__device__ __forceinline__ int32_t dd_slot(const DualDag &d, int32_t x) {
    DD_CONSTS
    uint32_t h = ((uint32_t)x * 2654435761u) >> 24;
    for (int p = 0; p < DD_SLOTS; ++p) {
        const int32_t slot = (int32_t)((h + (uint32_t)p) & (DD_SLOTS - 1));
        const int32_t prev = atomicCAS(&d.key[slot], -1, x);
        if (prev == -1 || prev == x) return slot;
    }
    return -1;
}

// One arc (a, x) of the union walk (x in slot sx; kinds: the sub-DAGs it is
// in; sa: a's slot or -1): recorded, a's successor counts and memberships
// raised, and a queued for the next level with any membership it gains.
// da_o, sg, pa: d(s,a), sigma_sa and a's stored predecessor, kept at a's
// first sight (a not in B: its new values are its old ones).
template <int TS>
__device__ __forceinline__ void dd_add_arc(const DualDag &d, BlockShared &sh, const int32_t a, int32_t sa,
                                           const int32_t sx, const int32_t kinds, const int32_t da_o, const uint64_t sg,
                                           const int32_t pa) {
    DD_CONSTS
    if (sa < 0) sa = dd_slot<TS>(d, a);
    const int32_t k = atomicAdd(&sh.tail, 1);
    if (sa < 0 || k >= DD_ARCS) {
        sh.ovf = 1;
        return;
    }
    d.arcs[k] = sa | (sx << 8) | (kinds << 16);
    atomicAdd(&d.cnt[sa], ((kinds & DF_O) ? 1 : 0) + ((kinds & DF_N) ? 1 << 16 : 0));
    const int32_t old = atomicOr(&d.flags[sa], kinds);
    const int32_t gained = kinds & ~old;
    if (!gained) return;
    if (!(old & (DF_O | DF_N | DF_B))) {
        if (atomicAdd(&sh.nk, 1) >= DD_CAP) {
            sh.ovf = 1;
            return;
        }
        d.dold[sa] = da_o;
        d.dnew[sa] = da_o;
        d.sold[sa] = sg;
        d.snew[sa] = sg;
        d.pr[sa] = pa;
    }
    const int32_t pos = atomicAdd(&sh.next, 1);
    if (pos >= DD_FRONT) sh.ovf = 1;
    else d.front[pos] = sa | (gained << 16);
}

// The recorded arcs grouped by head (a counting sort in LDS), for the Kahn
// walks of both sub-DAGs.
template <int TS>
__device__ __forceinline__ void dual_group_arcs(const DualDag &d, const int32_t narcs, BlockShared &sh) {
    DD_CONSTS
    const int tid = threadIdx.x, bs = blockDim.x;
    for (int32_t i = tid; i < DD_SLOTS; i += bs) d.hdeg[i] = 0;
    __syncthreads();
    for (int32_t k = tid; k < narcs; k += bs) atomicAdd(&d.hdeg[(d.arcs[k] >> 8) & 0xff], 1);
    __syncthreads();
    // exclusive scan over the slots, a run of consecutive slots per thread
    const int32_t per = (DD_SLOTS + bs - 1) / bs, i0 = min(tid * per, DD_SLOTS), i1 = min(i0 + per, DD_SLOTS);
    int32_t run = 0;
    for (int32_t i = i0; i < i1; ++i) run += d.hdeg[i];
    int32_t total;
    int32_t off = block_excl_scan(run, sh.scan, total);
    for (int32_t i = i0; i < i1; ++i) {
        d.hend[i] = off;
        off += d.hdeg[i];
    }
    __syncthreads();
    // the scatter leaves hend[h] at the end of h's range
    for (int32_t k = tid; k < narcs; k += bs) {
        const int32_t e = d.arcs[k];
        d.harc[atomicAdd(&d.hend[(e >> 8) & 0xff], 1)] = e;
    }
    __syncthreads();
}

// Dependency accumulation over one of the two sub-DAGs (kind 1: old, 2: new)
// from its sinks: a member x, once every successor has pushed, gives each
// DAG predecessor a the share sigma_sa * ([x in B] + acc(x)) / sigma_sx.  The
// lane whose push completes a carries on with a at once, so a chain takes no
// rounds; a vertex completing two or more waits for the next round.
template <int TS>
__device__ __forceinline__ void dual_kahn(const DualDag &d, const int kind, BlockShared &sh) {
    DD_CONSTS
    const int tid = threadIdx.x, bs = blockDim.x;
    const int shift = kind == DF_O ? 0 : 16;
    double *const acc = kind == DF_O ? d.acc_o : d.acc_n;
    const uint64_t *const sv = kind == DF_O ? d.sold : d.snew;
    if (tid == 0) sh.kpos = 0;
    __syncthreads();
    for (int32_t i = tid; i < DD_SLOTS; i += bs)
        if (d.key[i] >= 0 && (d.flags[i] & kind) && ((d.cnt[i] >> shift) & 0xffff) == 0)
            d.klist[atomicAdd(&sh.kpos, 1)] = i;
    __syncthreads();
    int32_t lo = 0, hi = sh.kpos;
    while (lo < hi) {
        for (int32_t idx = lo + tid; idx < hi; idx += bs) {
            int32_t x = d.klist[idx];
            for (;;) {
                const double c = (((d.flags[x] & DF_B) ? 1.0 : 0.0) + acc[x]) / (double)sv[x];
                int32_t next = -1;
                const int32_t e1 = d.hend[x];
                for (int32_t e = e1 - d.hdeg[x]; e < e1; ++e) {
                    const int32_t arc = d.harc[e];
                    if (!((arc >> 16) & kind)) continue;
                    const int32_t a = arc & 0xff;
                    if (c != 0.0) atomicAdd(&acc[a], (double)sv[a] * c);
                    // release: the share lands before the count drops;
                    // acquire: the last pusher sees every other share
                    const int32_t left = __hip_atomic_fetch_sub(&d.cnt[a], 1 << shift, __ATOMIC_ACQ_REL,
                                                                 __HIP_MEMORY_SCOPE_WORKGROUP);
                    if (((left >> shift) & 0xffff) == 1) {
                        if (next < 0) next = a;
                        else d.klist[atomicAdd(&sh.kpos, 1)] = a;
                    }
                }
                if (next < 0) break;
                x = next;
            }
        }
        __syncthreads();
        lo = hi;
        hi = sh.kpos;
        __syncthreads();
    }
}

template <int TS>
__device__ bool dual_pass(const int32_t s, const int32_t *__restrict__ Dold, const uint64_t *__restrict__ Sold,
                          const int32_t *__restrict__ xcp, const int32_t *__restrict__ ycp,
                          const int32_t *__restrict__ ycs, const int32_t *__restrict__ ycw,
                          const int32_t *__restrict__ Bt, const int32_t *__restrict__ Bd,
                          const uint64_t *__restrict__ Bs, const int32_t *__restrict__ pred, const int32_t nb,
                          double *out, BlockShared &sh, const ExpandShared &es, const DualDag &d) {
    DD_CONSTS
    const int tid = threadIdx.x, bs = blockDim.x;
    for (int32_t i = tid; i < DD_SLOTS; i += bs) {
        d.key[i] = -1;
        d.flags[i] = 0;
        d.cnt[i] = 0;
        d.acc_o[i] = 0.0;
        d.acc_n[i] = 0.0;
    }
    if (tid == 0) {
        sh.next = 0;   // frontier entries
        sh.tail = 0;   // recorded arcs
        sh.nk = 0;     // vertices
        sh.ovf = 0;
    }
    __syncthreads();
    // B: roots of both sub-DAGs (of the old one only if t was reachable)
    for (int32_t i = tid; i < nb; i += bs) {
        const int32_t t = Bt[i];
        if (t == s) continue;
        const int32_t slot = dd_slot<TS>(d, t);
        const int32_t v = atomicAdd(&sh.nk, 1);
        const int32_t pos = atomicAdd(&sh.next, 1);
        if (slot < 0 || v >= DD_CAP || pos >= DD_FRONT) {
            sh.ovf = 1;
            continue;
        }
        // everything the walk reads of t, in one round trip
        const int32_t dt = Dold[t];
        const uint64_t st = Sold[t];
        const int32_t pt = pred[t];
        const int32_t yb = ycp[t], ye = ycp[t + 1], xb = xcp[t], xe = xcp[t + 1];
        const int32_t mem = DF_N | (dt != INF32 ? DF_O : 0);
        d.flags[slot] = DF_B | mem;
        d.dold[slot] = dt;
        d.dnew[slot] = Bd[i];
        d.sold[slot] = dt != INF32 ? st : 0;
        d.snew[slot] = Bs[i];
        d.pr[slot] = pt;
        d.ybeg[slot] = yb;
        d.ydeg[slot] = ye - yb;
        d.xdeg[slot] = xe - xb;
        d.front[pos] = slot | (mem << 16);
    }
    __syncthreads();
    if (sh.ovf) return false;
    int32_t lo = 0, hi = sh.next;
    __syncthreads();
    // per general entry: its stored old predecessor and how many of its
    // merged in-arcs are tested (the rest of its work items: the stored arc)
    int32_t *const ex_pred = (int32_t *)es.val, *const ex_test = ex_pred + bs;
    while (lo < hi) {
        if (tid == 0) sh.kpos = 0;
        __syncthreads();
        // an unchanged vertex with one stored predecessor: that arc, at
        // once, for both memberships (an unchanged pair keeps its DAG
        // in-arcs); the others to the level's general list
        for (int32_t idx = lo + tid; idx < hi; idx += bs) {
            const int32_t entry = d.front[idx];
            const int32_t sl = entry & 0xffff;
            if (d.key[sl] == s) continue;
            const int32_t pr = d.pr[sl];
            if ((d.flags[sl] & DF_B) || pr < 0) {
                d.slow[atomicAdd(&sh.kpos, 1)] = entry;
                continue;
            }
            // with the distance, what a first sight of the tail needs
            const int32_t da_o = Dold[pr];
            const uint64_t sg = Sold[pr];
            const int32_t pa = pred[pr];
            dd_add_arc<TS>(d, sh, pr, dd_find<TS>(d, pr), sl, (entry >> 16) & (DF_O | DF_N), da_o, sg, pa);
        }
        __syncthreads();
        const int32_t nslow = sh.kpos;
        for (int32_t c = 0; c < nslow; c += bs) {
            const int32_t idx = c + tid;
            int32_t entry = 0, b0 = 0, cnt = 0, ntest = 0, olen = 0, pr = PRED_NONE;
            if (idx < nslow) {
                entry = d.slow[idx];
                const int32_t sl = entry & 0xffff, mem = entry >> 16;
                const int32_t x = d.key[sl];
                pr = d.pr[sl];
                if (d.flags[sl] & DF_B) {
                    // a changed target: its new DAG in-arcs by Eq.1 over the
                    // merged E*; its old ones from the stored predecessor, or
                    // by Eq.1 over the old E* arcs where two or more
                    b0 = d.ybeg[sl];
                    ntest = d.ydeg[sl];
                    olen = ((mem & DF_O) && pr < 0) ? d.xdeg[sl] : 0;
                    cnt = ntest + (((mem & DF_O) && pr >= 0) ? 1 : 0);
                } else {
                    // two or more DAG in-arcs: Eq.1 over E*
                    b0 = ycp[x];
                    ntest = ycp[x + 1] - b0;
                    olen = (mem & DF_O) ? xcp[x + 1] - xcp[x] : 0;
                    cnt = ntest;
                }
            }
            int32_t total;
            const int32_t off = block_excl_scan(cnt, sh.scan, total);
            es.off[tid] = off;
            es.vtx[tid] = entry;
            es.beg[tid] = b0;
            es.dx[tid] = olen;
            ex_pred[tid] = pr;
            ex_test[tid] = ntest;
            __syncthreads();
            const int32_t nv = min(bs, nslow - c);
            for (int32_t j = tid; j < total; j += bs) {
                const int32_t i = find_owner(es, nv, j);
                const int32_t ent = es.vtx[i];
                const int32_t sx = ent & 0xffff, mem = ent >> 16;
                const int32_t rel = j - es.off[i];
                int32_t a, da_o, pa, sa, kinds;
                uint64_t sg;
                if (rel < ex_test[i]) {
                    const int32_t e = es.beg[i] + rel;
                    a = ycs[e];
                    const int32_t w = ycw[e];
                    // with the distance, what a first sight of a needs
                    da_o = Dold[a];
                    sg = Sold[a];
                    pa = pred[a];
                    sa = dd_find<TS>(d, a);
                    const int32_t da_n = (sa >= 0 && (d.flags[sa] & DF_B)) ? d.dnew[sa] : da_o;
                    const bool po = (mem & DF_O) && rel < es.dx[i] && da_o != INF32 &&
                                    (int64_t)da_o + w == (int64_t)d.dold[sx];
                    const bool pn = (mem & DF_N) && da_n != INF32 && (int64_t)da_n + w == (int64_t)d.dnew[sx];
                    if (!po && !pn) continue;
                    kinds = (po ? DF_O : 0) | (pn ? DF_N : 0);
                } else {
                    // the stored predecessor of a changed target: old
                    // membership only
                    a = ex_pred[i];
                    da_o = Dold[a];
                    sg = Sold[a];
                    pa = pred[a];
                    sa = dd_find<TS>(d, a);
                    kinds = DF_O;
                }
                dd_add_arc<TS>(d, sh, a, sa, sx, kinds, da_o, sg, pa);
            }
            __syncthreads();
        }
        const bool ovf = sh.ovf != 0;
        lo = hi;
        hi = sh.next;
        __syncthreads();
        if (ovf) return false;
    }
    const int32_t narcs = sh.tail;
    // the new stored predecessor of each changed target: its only recorded
    // new-DAG in-arc (every new in-arc of a changed target was tested and
    // recorded when it was expanded), else MULTI
    for (int32_t i = tid; i < DD_SLOTS; i += bs) d.round[i] = 0;
    __syncthreads();
    for (int32_t k = tid; k < narcs; k += bs) {
        const int32_t e = d.arcs[k];
        if (!((e >> 16) & DF_N)) continue;
        const int32_t sx = (e >> 8) & 0xff;
        if (!(d.flags[sx] & DF_B)) continue;
        if (atomicAdd(&d.round[sx], 1) == 0) d.front[sx] = d.key[e & 0xff];
    }
    __syncthreads();
    for (int32_t i = tid; i < DD_SLOTS; i += bs)
        if (d.key[i] >= 0 && (d.flags[i] & DF_B) && d.round[i] != 1)
            d.front[i] = d.round[i] == 0 ? PRED_NONE : PRED_MULTI;
    __syncthreads();
    dual_group_arcs<TS>(d, narcs, sh);
    dual_kahn<TS>(d, DF_O, sh);
    dual_kahn<TS>(d, DF_N, sh);
    for (int32_t i = tid; i < DD_SLOTS; i += bs) {
        const int32_t x = d.key[i];
        if (x < 0 || x == s) continue;
        const double diff = d.acc_n[i] - d.acc_o[i];
        if (diff != 0.0) atomicAdd(&out[x], diff);
    }
    __syncthreads();
    return true;
}

// Row-v data an update reads for every pair (s,t) of an affected row.
struct RowV {
    const int32_t *rvD;   // d(v,t)  (= d'(v,t))
    const uint64_t *rvS;  // sigma_vt
    const int32_t *rvvD;  // d''(v,t)           (Out phase only)
    const uint64_t *rvvS; // sigma''_vt
    const uint64_t *rvvH; // sigma-hat''_vt
    bool has_out;
};

// New (d, sigma) of pair (s,t) by Lemma 4 In phase (D = d'(s,v) + d(v,t)),
// then, if E_o is not empty, Lemma 4 on G'_R (D = d'(s,v) + d''(v,t)).  sigma
// is read only where a distance test says the pair may change.  Returns true
// if the pair changes.
__device__ __forceinline__ bool pair_update(const RowV &R, const SrcScal &sc, const bool same, const int32_t t,
                                            const int32_t d0, const int32_t rvd, const int32_t dvv,
                                            const uint64_t *Sg, int32_t &d_out, uint64_t &s_out, bool &ovf_s,
                                            bool &ovf_d) {
    int32_t d = d0;
    uint64_t sg = 0;
    bool sg_known = false;
    int64_t c;
    if (in_rule(d0, sc.dv, rvd, c)) {
        if (c >= INF32) {
            ovf_d = true;
        } else if (c < d0) {
            d = (int32_t)c;
            sg = mul_chk(sc.sv, R.rvS[t], ovf_s);
            sg_known = true;
        } else {
            const uint64_t add = mul_chk(same ? sc.hv : sc.sv, R.rvS[t], ovf_s);
            if (add != 0) {
                sg = add_chk(Sg[t], add, ovf_s);
                sg_known = true;
            }
        }
    }
    if (R.has_out) {
        int64_t c2;
        if (in_rule(d, sc.dv, dvv, c2)) {
            if (c2 >= INF32) {
                ovf_d = true;
            } else if (c2 < d) {
                d = (int32_t)c2;
                sg = mul_chk(sc.sv, R.rvvS[t], ovf_s);
                sg_known = true;
            } else {
                const uint64_t mult = (dvv == rvd) ? R.rvvH[t] : R.rvvS[t];
                const uint64_t add = mul_chk(sc.sv, mult, ovf_s);
                if (add != 0) {
                    sg = add_chk(sg_known ? sg : Sg[t], add, ovf_s);
                    sg_known = true;
                }
            }
        }
    }
    d_out = d;
    s_out = sg;
    return sg_known;
}

// Quick reject: neither phase can reach pair (s,t) unless d'(s,v) plus the
// row-v distance is at most the current d(s,t) (Lemma 4 case 1 otherwise).
// in_on is false for a source whose In phase is void: d'(s,v) = d(s,v) with
// no new paths into v (sigma-hat'_sv = 0), where a tie adds 0 paths and a
// strict gain would break the triangle inequality of the old distances.
__device__ __forceinline__ bool may_change(int32_t d0, int32_t dv, int32_t rvd, int32_t dvv, bool in_on) {
    if (dv == INF32) return false;
    const bool in = in_on && rvd != INF32 && ((int64_t)dv + rvd <= (int64_t)d0 || d0 == INF32);
    const bool out = dvv != INF32 && ((int64_t)dv + dvv <= (int64_t)d0 || d0 == INF32);
    return in || out;
}

// The same test against one filter row f (f_any, or f_out when the In phase
// is void) for a finite d'(s,v): d'(s,v) + f(t) <= d(s,t), or t unreachable.
// Finite distances are below 2^31-1, so the sum of two fits in 32 unsigned
// bits.
__device__ __forceinline__ bool may_change1(int32_t d0, int32_t dv, int32_t f) {
    return f != INF32 && ((uint32_t)dv + (uint32_t)f <= (uint32_t)d0 || d0 == INF32);
}

// Changed-target list a row scan fills: entries go to (t, d, s) up to cap;
// the count (BlockShared::nb) keeps going past cap, and then the list is
// incomplete.
struct BList {
    int32_t *t, *d;
    uint64_t *s;
    int32_t cap;
};

// A streamed row quad.  Each affected row is read once per update, so its
// loads are nontemporal: they do not displace the filter row, which every
// row of the update reads again, from the caches.
__device__ __forceinline__ int4 load_stream(const int4 *p) {
    typedef int v4i __attribute__((ext_vector_type(4)));
    const v4i t = __builtin_nontemporal_load((const v4i *)p);
    return make_int4(t.x, t.y, t.z, t.w);
}

// Bit mask of the pairs of one quad that may change (dv finite).
__device__ __forceinline__ uint32_t quad_mask(const int4 d, const int4 f, const int32_t dv) {
    return (may_change1(d.x, dv, f.x) ? 1u : 0u) | (may_change1(d.y, dv, f.y) ? 2u : 0u) |
           (may_change1(d.z, dv, f.z) ? 4u : 0u) | (may_change1(d.w, dv, f.w) ? 8u : 0u);
}

// Row scan of affected source s (the all-pairs step of Alg 3, restricted to
// row s), in two phases:
//   1. the distance filter (may_change) over the candidate targets when that
//      list is short, else over the whole row against the filter rows; the
//      targets that pass go to F (up to fcap; the count in sh.nf goes on),
//   2. after a barrier, all lanes share the flagged targets: the full
//      Lemma 4 update of each (from the rows themselves), and the pairs that
//      change go to the B list L with their new values (count in sh.nb).
// Keeping the second phase out of the streaming loop keeps that loop small
// and spreads the flagged pairs over the workgroup.  The caller zeroes sh.nf
// and sh.nb before; if sh.nf > fcap after the call, the B list is incomplete.
// QU quads per lane are in flight in the streaming loop.
template <int QU>
__device__ __forceinline__ void scan_row(const UpdateJob &J, const RowV &R, const SrcScal &sc, const bool same,
                                         const int32_t *__restrict__ Drow, const uint64_t *__restrict__ Sg,
                                         const bool use_tlist, const int32_t t_count, int32_t *F, const int32_t fcap,
                                         const BList &L, BlockShared &sh, bool &ovf_s, bool &ovf_d) {
    const int tid = threadIdx.x, bs = blockDim.x;
    const int32_t n = J.g.n;
    const bool in_on = !same || sc.hv != 0;
    auto flag = [&](int32_t t) {
        const int32_t pos = atomicAdd(&sh.nf, 1);
        if (pos < fcap) F[pos] = t;
    };
    if (use_tlist) {
        const int32_t *const tlist = J.g.tlist, *const tl_rvD = J.g.tl_rvD, *const tl_rvvD = J.g.tl_rvvD;
        for (int32_t i = tid; i < t_count; i += bs) {
            const int32_t t = tlist[i];
            if (may_change(Drow[t], sc.dv, tl_rvD[i], R.has_out ? tl_rvvD[i] : INF32, in_on)) flag(t);
        }
    } else if (sc.dv == INF32) {
        // v unreachable from s: no pair of the row can change
    } else if ((n & 3) == 0) {
        // QU quads (4 QU pairs) per lane in flight, tested against one
        // filter row
        const int32_t nq = n >> 2;
        const int4 *D4 = (const int4 *)Drow;
        const int4 *F4 = (const int4 *)(in_on ? J.g.f_any : J.g.f_out);
        for (int32_t q0 = tid; q0 < nq; q0 += QU * bs) {
            int4 dq[QU], fq[QU];
#pragma unroll
            for (int k = 0; k < QU; ++k) {
                const int32_t q = q0 + k * bs;
                dq[k] = (q < nq) ? load_stream(D4 + q) : make_int4(0, 0, 0, 0);
                fq[k] = (q < nq) ? F4[q] : make_int4(INF32, INF32, INF32, INF32);
            }
            uint32_t m = 0;
#pragma unroll
            for (int k = 0; k < QU; ++k) m |= quad_mask(dq[k], fq[k], sc.dv) << (4 * k);
            while (m) {
                const int b = __ffs(m) - 1;
                m &= m - 1;
                flag(((q0 + (b >> 2) * bs) << 2) + (b & 3));
            }
        }
    } else {
        const int32_t *f = in_on ? J.g.f_any : J.g.f_out;
        for (int32_t t = tid; t < n; t += bs)
            if (may_change1(Drow[t], sc.dv, f[t])) flag(t);
    }
    __syncthreads();
    const int32_t nf = min(sh.nf, fcap);
    for (int32_t i = tid; i < nf; i += bs) {
        const int32_t t = F[i];
        int32_t d;
        uint64_t sg;
        if (pair_update(R, sc, same, t, Drow[t], R.rvD[t], R.has_out ? R.rvvD[t] : INF32, Sg, d, sg, ovf_s, ovf_d)) {
            const int32_t pos = atomicAdd(&sh.nb, 1);
            if (pos < L.cap) {
                L.t[pos] = t;
                L.d[pos] = d;
                L.s[pos] = sg;
            }
        }
    }
}

__device__ __forceinline__ RowV row_v_of(const UpdateJob &J) {
    RowV R;
    R.rvD = J.row_v_D;
    R.rvS = J.row_v_S;
    R.rvvD = J.g.rvv_D;
    R.rvvS = J.g.rvv_S;
    R.rvvH = J.g.rvv_H;
    R.has_out = J.n_out > 0;
    return R;
}

// Rows of an update with at most 64 candidate targets (the candidate list is
// scanned instead of the rows): each wave takes 64 / lpr rows at once, a
// group of lpr lanes per row (lpr = the candidate count rounded up to a power
// of two), one candidate per lane, with no workgroup barriers.  The changed pairs of a
// row are compacted with a ballot and written to the step's target pool
// straight from the lanes; the listing rules are those of k_rows, with the
// pool and list reservations of a wave's rows taken in one atomic each.
__device__ void rows_few_targets(const UpdateJob &J, const RowV &R, const int32_t count, const int32_t t_count,
                                 const int32_t cap, const StepPool &pool) {
    GraphCtl *ctl = J.g.ctl;
    const int32_t n = J.g.n;
    const int lane = lane_id();
    int lpr = 1;
    while (lpr < t_count) lpr <<= 1;
    const int rpw = 64 / lpr;
    const int g = lane / lpr, r = lane - g * lpr;
    const uint64_t gmask = lpr == 64 ? ~0ull : ((1ull << lpr) - 1);
    // this lane's candidate and its row-v data, the same for every row
    const bool has_t = r < t_count;
    const int32_t t = has_t ? J.g.tlist[r] : 0;
    const int32_t f_rvd = has_t ? J.g.tl_rvD[r] : INF32;
    const int32_t f_rvvd = has_t && R.has_out ? J.g.tl_rvvD[r] : INF32;
    const int32_t rvd = has_t ? R.rvD[t] : INF32;
    const int32_t rvvd = has_t && R.has_out ? R.rvvD[t] : INF32;
    bool ovf_s = false, ovf_d = false;
    int32_t listed_pairs = 0;
    for (;;) {
        int32_t base = 0;
        if (lane == 0) base = atomicAdd(&ctl->work_next, rpw);
        base = __shfl(base, 0, 64);
        if (base >= count) break;
        const int32_t item = base + g;
        const bool row_ok = item < count;
        int32_t s = 0, d = 0;
        uint64_t sg = 0;
        bool chg = false;
        if (row_ok && has_t) {
            s = J.g.alist[item];
            const SrcScal sc = J.g.scal[s];
            const bool same = (sc.flags & 1) != 0;
            const int32_t *Drow = J.g.D + (size_t)s * n;
            const int32_t d0 = Drow[t];
            if (may_change(d0, sc.dv, f_rvd, f_rvvd, !same || sc.hv != 0))
                chg = pair_update(R, sc, same, t, d0, rvd, rvvd, J.g.S + (size_t)s * n, d, sg, ovf_s, ovf_d);
        }
        const uint64_t gm = (__ballot(chg) >> (g * lpr)) & gmask;
        const int32_t nb = (int32_t)__popcll(gm);
        // the groups' first lanes (each holds a candidate, so it read s) list
        // their sources, with one reservation per wave in the pool and in
        // each end of the list: a wave prefix sum of the pool entries wanted
        const bool lead = row_ok && r == 0 && nb > 0;
        const int32_t want = lead && nb <= cap ? nb : 0;
        int32_t incl = want;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int32_t v = __shfl_up(incl, o, 64);
            if (lane >= o) incl += v;
        }
        const int32_t total = __shfl(incl, 63, 64);
        int32_t pb_lo = 0, pb_hi = 0;
        if (lane == 0 && total > 0) {
            const unsigned long long o = atomicAdd(pool.next, (unsigned long long)total);
            pb_lo = (int32_t)(o & 0xffffffffull);
            pb_hi = (int32_t)(o >> 32);
        }
        pb_lo = __shfl(pb_lo, 0, 64);
        pb_hi = __shfl(pb_hi, 0, 64);
        const unsigned long long pbase = ((unsigned long long)(uint32_t)pb_hi << 32) | (uint32_t)pb_lo;
        const unsigned long long mine = pbase + (unsigned long long)(incl - want);
        const bool listed = want > 0 && mine + (unsigned long long)nb <= (unsigned long long)pool.cap;
        const uint64_t hm = __ballot(listed && nb >= HEAVY_NB), lm = __ballot(listed && nb < HEAVY_NB);
        const uint64_t dm = __ballot(lead && !listed);
        int32_t hb = 0, lb = 0, db = 0;
        if (lane == 0) {
            if (hm) hb = atomicAdd(&ctl->dag_count, (int32_t)__popcll(hm));
            if (lm) lb = atomicAdd(&ctl->dag_back, (int32_t)__popcll(lm));
            if (dm) db = atomicAdd(&ctl->big_count, (int32_t)__popcll(dm));
        }
        hb = __shfl(hb, 0, 64);
        lb = __shfl(lb, 0, 64);
        db = __shfl(db, 0, 64);
        if (listed) {
            DItem it;
            it.s = s;
            it.nb = nb;
            it.off = (int64_t)mine;
            if (nb >= HEAVY_NB) J.g.dlist[hb + (int32_t)popc_below(hm, lane)] = it;
            else J.g.dlist[n - 1 - (lb + (int32_t)popc_below(lm, lane))] = it;
            listed_pairs += nb;
        } else if (lead) {
            J.g.biglist[db + (int32_t)popc_below(dm, lane)] = s;
        }
        // the group's changed pairs go to its pool entries
        const int src_lane = g * lpr;
        const bool g_listed = __shfl((int32_t)listed, src_lane, 64) != 0;
        const int32_t off_lo = __shfl((int32_t)(mine & 0xffffffffull), src_lane, 64);
        const int32_t off_hi = __shfl((int32_t)(mine >> 32), src_lane, 64);
        if (chg && g_listed) {
            const unsigned long long p = (((unsigned long long)(uint32_t)off_hi << 32) | (uint32_t)off_lo) +
                                         (unsigned long long)__popcll(gm & ((1ull << r) - 1));
            pool.t[p] = t;
            pool.d[p] = d;
            pool.s[p] = sg;
        }
    }
    if (ovf_s) atomicOr(&ctl->status, ST_SIGMA_OVF);
    if (ovf_d) atomicOr(&ctl->status, ST_DIST_OVF);
    // one statistic update per wave
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) listed_pairs += __shfl_xor(listed_pairs, o, 64);
    if (lane == 0 && listed_pairs) atomicAdd(&ctl->changed_pairs, (unsigned long long)listed_pairs);
}

// Row kernel (persistent): workgroups pull affected sources from a device
// counter and scan their rows (scan_row).  A source's changed targets are
// collected in LDS; up to big_b of them are copied to the step's target pool
// and the source is listed for the DAG kernel, more (or a full pool) defer
// the source to the wide kernel, which scans the row again.  Nothing in D or
// sigma is written here: the old partial dependency still needs the old row.
__global__ void __launch_bounds__(256) k_rows(const UpdateJob *__restrict__ jobs, const int32_t *__restrict__ njobs_p,
                                              int32_t big_b, StepPool pool) {
    __shared__ int32_t lt[LCAP], ld[LCAP], lf[LCAP];
    __shared__ uint64_t ls[LCAP];
    __shared__ BlockShared sh;
    __shared__ long long sh_off;
    const int tid = threadIdx.x, bs = blockDim.x;
    const int njobs = *njobs_p;
    const BList L{lt, ld, ls, min(big_b, LCAP)};
    for (int j = 0; j < njobs; ++j) {
        const UpdateJob &J = jobs[j];
        if (job_halted(J)) continue;
        GraphCtl *ctl = J.g.ctl;
        const int32_t n = J.g.n;
        const int32_t count = *(volatile int32_t *)&ctl->a_count;
        const RowV R = row_v_of(J);
        const int32_t t_count = *(volatile int32_t *)&ctl->t_count;
        const bool use_tlist = (int64_t)t_count * 8 <= (int64_t)n;
        if (use_tlist && t_count <= 64) {
            // a row without candidates cannot change
            if (t_count > 0) rows_few_targets(J, R, count, t_count, L.cap, pool);
            continue;
        }
        if (tid == 0) sh.counter = 0;
        bool ovf_s = false, ovf_d = false;
        for (;;) {
            __syncthreads();
            if (tid == 0) {
                sh.item = atomicAdd(&ctl->work_next, 1);
                sh.nb = 0;
                sh.nf = 0;
            }
            __syncthreads();
            const int32_t item = sh.item;
            if (item >= count) break;
            const int32_t s = J.g.alist[item];
            const SrcScal sc = J.g.scal[s];
            const int32_t *Drow = J.g.D + (size_t)s * n;
            const uint64_t *Sg = J.g.S + (size_t)s * n;
            scan_row<8>(J, R, sc, (sc.flags & 1) != 0, Drow, Sg, use_tlist, t_count, lf, LCAP, L, sh, ovf_s, ovf_d);
            __syncthreads();
            const int32_t nb = sh.nb;
            if (nb == 0 && sh.nf <= LCAP) continue;
            if (tid == 0) {
                long long off = -1;
                if (nb <= L.cap && sh.nf <= LCAP) {
                    const unsigned long long o = atomicAdd(pool.next, (unsigned long long)nb);
                    if (o + (unsigned long long)nb <= (unsigned long long)pool.cap) off = (long long)o;
                }
                if (off >= 0) {
                    DItem it;
                    it.s = s;
                    it.nb = nb;
                    it.off = off;
                    if (nb >= HEAVY_NB) J.g.dlist[atomicAdd(&ctl->dag_count, 1)] = it;
                    else J.g.dlist[n - 1 - atomicAdd(&ctl->dag_back, 1)] = it;
                    sh.counter += (unsigned long long)nb;
                } else {
                    J.g.biglist[atomicAdd(&ctl->big_count, 1)] = s;
                }
                sh_off = off;
            }
            __syncthreads();
            const long long off = sh_off;
            if (off >= 0) {
                for (int32_t i = tid; i < nb; i += bs) {
                    pool.t[off + i] = lt[i];
                    pool.d[off + i] = ld[i];
                    pool.s[off + i] = ls[i];
                }
            }
        }
        if (ovf_s) atomicOr(&ctl->status, ST_SIGMA_OVF);
        if (ovf_d) atomicOr(&ctl->status, ST_DIST_OVF);
        __syncthreads();
        if (tid == 0 && sh.counter) atomicAdd(&ctl->changed_pairs, sh.counter);
    }
}

// Alg 2 (Update-DAG) on the stored predecessors, for a one-arc update (u, v)
// and a changed target t of source s.  A target whose distance fell
// (WT-changed) has exactly its DAG(v) in-arcs as DAG'(s) in-arcs, or the arc
// (u, v) alone when t = v; one whose distance stayed (NUM-changed) keeps its
// old in-arcs and gains those (at v: gains (u, v), so it has two or more).
// DAG(v) itself does not change (no shortest path from v enters v again), so
// row v of the predecessors is read as it stands while other rows change.
__device__ __forceinline__ bool one_arc_job(const UpdateJob &J) { return J.n_in == 1 && J.n_out == 0; }

__device__ __forceinline__ int32_t edge_pred(const UpdateJob &J, const int32_t t, const int32_t old_pred,
                                             const bool fell) {
    if (t == J.v) return fell ? J.in_tail[0] : PRED_MULTI;
    const int32_t pv = J.g.pred[(size_t)J.v * J.g.n + t];
    if (fell) return pv;
    return old_pred >= 0 && old_pred == pv ? pv : PRED_MULTI;
}

// One listed source with its changed targets B (Bt, Bd, Bs; nb of them):
// both partial dependencies in one traversal in LDS (dual_pass) and then the
// changed pairs written to D and sigma; or, when the two sub-DAGs do not fit
// together:
//   1. old partial dependency over B (E* by head, old row), sign -1,
//   2. write the changed pairs (only those) to D and sigma,
//   3. new partial dependency over B (merged E*, new row), sign +1,
// each in LDS (small_pass) when it fits, else in the workgroup's slot.
template <int TS>
__device__ __forceinline__ void update_source(const UpdateJob &J, const int32_t s, const int32_t *__restrict__ Bt,
                                              const int32_t *__restrict__ Bd, const uint64_t *__restrict__ Bs,
                                              const int32_t nb, const bool lds, int32_t *lds_row, const USlot &u,
                                              BlockShared &sh, const ExpandShared &es, const SmallDag &sd,
                                              const DualDag &dd) {
    const int tid = threadIdx.x, bs = blockDim.x;
    const int32_t n = J.g.n;
    int32_t *const Dg = J.g.D + (size_t)s * n;
    uint64_t *const Sg = J.g.S + (size_t)s * n;
    const int32_t *Drow = lds ? lds_row : Dg;
    double *const bc_delta = J.g.bc_delta;
    // an LDS table holds at most 3/4 of its slots in vertices: larger B sets
    // go straight to the slot passes.  The union of both sub-DAGs with a B of
    // half that many or more almost never fits (on the Chung-Lu headline
    // window, 120 of 20 600 such sources fit with the 128-slot table), so
    // those skip the union walk; the new sub-DAG alone often fits
    const bool fits = nb < TS * 3 / 4;
    const bool dual_fits = nb < TS * 3 / 8;
    int32_t *const pred_row = J.g.pred + (size_t)s * n;
    const bool dual = dual_fits && dual_pass<TS>(s, Drow, Sg, J.g.xc_ptr, J.g.yc_ptr, J.g.yc_src, J.g.yc_w, Bt, Bd, Bs,
                                            pred_row, nb, bc_delta, sh, es, dd);
    // when the union outgrew the table it is mostly the old sub-DAG that did:
    // the old pass goes straight to the slot (it follows stored
    // predecessors), the new one tries the LDS table first
    if (!dual)
        restricted_pass<false, XU>(s, n, Drow, Sg, J.g.xc_ptr, J.g.xc_src, J.g.xc_dst, J.g.xc_w, Bt, nb, false, u,
                                   -1.0, bc_delta, pred_row, nullptr, true, sh, es);
    // a one-arc update gives the changed targets' new predecessors by Alg 2
    // (before the old distances are overwritten); the new pass then follows
    // them like any stored predecessor and tests no E* in-arcs of B
    const bool edge = one_arc_job(J);
    for (int32_t i = tid; i < nb; i += bs) {
        const int32_t t = Bt[i];
        const int32_t d = Bd[i];
        if (edge && !dual) pred_row[t] = edge_pred(J, t, pred_row[t], d < Drow[t]);
        Sg[t] = Bs[i];
        Dg[t] = d;
        if (lds) lds_row[t] = d;
        if (dual) {
            // the union walk found the changed targets' new predecessors
            const int32_t sl = dd_find<TS>(dd, t);
            if (sl >= 0) pred_row[t] = dd.front[sl];
        }
    }
    __syncthreads();
    if (dual) return;
    // the new pass reads the stored predecessors of unchanged pairs only (and
    // of a one-arc update's changed targets, written above), so it may write
    // the changed targets' new ones from its arc record
    bool preds_done = false;
    if (!fits || !small_pass<TS>(s, Drow, Sg, J.g.yc_ptr, J.g.yc_src, J.g.yc_w, Bt, nb, 1.0, bc_delta, pred_row,
                                 edge, sh, es, sd))
        preds_done = restricted_pass<false, XU>(s, n, Drow, Sg, J.g.yc_ptr, J.g.yc_src, J.g.yc_dst, J.g.yc_w, Bt, nb,
                                                false, u, 1.0, bc_delta, pred_row, edge ? nullptr : pred_row, edge, sh,
                                                es);
    if (!preds_done && !edge) refresh_preds<4>(Drow, J.g.yc_ptr, J.g.yc_src, J.g.yc_w, Bt, nb, pred_row, sh, es);
}

// DAG kernel (persistent): workgroups pull the sources the row kernel listed
// and run update_source on each.  The row is staged in LDS when n <= lds_cap
// (dynamic LDS of 4*lds_cap bytes).  Every workgroup's slot is laid out for
// the context-wide n_layout (the largest graph), so the zero-kept arrays sit
// at the same place for every job.  The work is bound by dependent gathers, so
// the register budget is held to five waves per SIMD (ten 128-thread
// workgroups per CU), 96 registers with no spills.
template <int TS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5, 8))) k_source(const UpdateJob *__restrict__ jobs, const int32_t *__restrict__ njobs_p,
                                                char *__restrict__ scratch, size_t slot_bytes, int32_t lds_cap,
                                                int32_t n_layout, StepPool pool) {
    extern __shared__ __align__(16) char dyn_lds[];
    int32_t *const lds_row = (int32_t *)dyn_lds;
    const ExpandShared es = expand_at(dyn_lds, lds_cap);
    char *const table = dyn_lds + align256((size_t)lds_cap * 4) + align256(XB * (size_t)blockDim.x);
    const SmallDag sd = small_dag_at<TS>(table);
    const DualDag dd = dual_dag_at<TS>(table);
    __shared__ BlockShared sh;
    const int tid = threadIdx.x, bs = blockDim.x;
    const int njobs = *njobs_p;
    const USlot u = uslot_at(scratch + (size_t)blockIdx.x * slot_bytes, n_layout);
    // the heavy sources of every job first (the front of each job's list),
    // then the light ones (the back): a step's long sub-DAG passes start
    // early whatever job they belong to, and the light sources fill the tail
    for (int phase = 0; phase < 2; ++phase)
    for (int j = 0; j < njobs; ++j) {
        const UpdateJob &J = jobs[j];
        if (job_halted(J)) continue;
        GraphCtl *ctl = J.g.ctl;
        const int32_t n = J.g.n;
        const bool lds = n <= lds_cap;
        const int32_t count = phase == 0 ? *(volatile int32_t *)&ctl->dag_count : *(volatile int32_t *)&ctl->dag_back;
        int32_t *const next = phase == 0 ? &ctl->dag_next : &ctl->dag_next_light;
        for (;;) {
            __syncthreads();
            if (tid == 0) sh.item = atomicAdd(next, 1);
            __syncthreads();
            const int32_t item = sh.item;
            if (item >= count) break;
            const DItem it = J.g.dlist[phase == 0 ? item : n - 1 - item];
            if (lds) {
                const int32_t *Dg = J.g.D + (size_t)it.s * n;
                for (int32_t t = tid; t < n; t += bs) lds_row[t] = Dg[t];
                __syncthreads();
            }
            update_source<TS>(J, it.s, pool.t + it.off, pool.d + it.off, pool.s + it.off, it.nb, lds, lds_row, u, sh, es,
                          sd, dd);
        }
    }
}

// A row copy with U loads in flight per lane (a plain loop waits for each
// load before the next one).
template <int U, typename T>
__device__ __forceinline__ void copy_row(T *dst, const T *__restrict__ src, const int32_t n) {
    const int tid = threadIdx.x, bs = blockDim.x;
    for (int32_t t0 = tid; t0 < n; t0 += U * bs) {
        T v[U];
#pragma unroll
        for (int k = 0; k < U; ++k) v[k] = t0 + k * bs < n ? src[t0 + k * bs] : T(0);
#pragma unroll
        for (int k = 0; k < U; ++k)
            if (t0 + k * bs < n) dst[t0 + k * bs] = v[k];
    }
}

// Wide kernel (persistent, runs after the DAG kernel): the deferred sources,
// one workgroup of up to 1024 threads per unit of work.  The first
// item_regions deferred sources (over the jobs in order) run as two units on
// two workgroups at once: the old pass (it also stores the changed pairs in
// the source's item region) and the new pass (it forms the new row and path
// counts in its slot from the old ones and the changed pairs).  Neither
// writes D or sigma; k_wide_apply does afterwards.  Further deferred sources
// run as one unit each: scan, old pass, write the changed pairs, new pass.
// Every unit scans its row again into the slot's full-length list.
__global__ void __launch_bounds__(1024) k_source_wide(const UpdateJob *__restrict__ jobs,
                                                      const int32_t *__restrict__ njobs_p, char *__restrict__ scratch,
                                                      size_t slot_bytes, int32_t lds_cap, int32_t n_layout,
                                                      char *__restrict__ items, int32_t item_regions) {
    extern __shared__ __align__(16) char dyn_lds[];
    int32_t *const lds_row = (int32_t *)dyn_lds;
    const ExpandShared es = expand_at(dyn_lds, lds_cap);
    __shared__ BlockShared sh;
    const int tid = threadIdx.x, bs = blockDim.x;
    const int njobs = *njobs_p;
    const USlot u = wslot_at(scratch + (size_t)blockIdx.x * slot_bytes, n_layout);
    const size_t region_bytes = item_region_bytes(n_layout);
    int32_t region0 = 0;  // first item region of the job
    for (int j = 0; j < njobs; ++j) {
        const UpdateJob &J = jobs[j];
        GraphCtl *ctl = J.g.ctl;
        const int32_t n = J.g.n;
        const bool lds = n <= lds_cap;
        // the item regions of a job follow those of the jobs before it, halted
        // or not (k_wide_apply counts them the same way)
        const int32_t count = *(volatile int32_t *)&ctl->big_count;
        const int32_t paired = min(count, item_regions - region0);
        if (job_halted(J)) {
            region0 += paired;
            continue;
        }
        const int32_t units = 2 * paired + (count - paired);
        const RowV R = row_v_of(J);
        const int32_t t_count = *(volatile int32_t *)&ctl->t_count;
        const bool use_tlist = (int64_t)t_count * 8 <= (int64_t)n;
        const BList L{u.bl_t, u.bl_d, u.bl_s, n};
        const bool edge = one_arc_job(J);
        if (tid == 0) sh.counter = 0;
        bool ovf_s = false, ovf_d = false;
        for (;;) {
            __syncthreads();
            if (tid == 0) {
                sh.item = atomicAdd(&ctl->big_next, 1);
                sh.nb = 0;
                sh.nf = 0;
            }
            __syncthreads();
            const int32_t unit = sh.item;
            if (unit >= units) break;
            // role 0: old pass, 1: new pass, 2: the whole update of the source
            const int32_t item = unit < 2 * paired ? unit >> 1 : paired + (unit - 2 * paired);
            const int role = unit < 2 * paired ? (unit & 1) : 2;
            const int32_t s = J.g.biglist[item];
            const SrcScal sc = J.g.scal[s];
            int32_t *const pred_row = J.g.pred + (size_t)s * n;
            const int32_t *Dg = J.g.D + (size_t)s * n;
            const uint64_t *Sg = J.g.S + (size_t)s * n;
            if (lds) {
                copy_row<4>(lds_row, Dg, n);
                __syncthreads();
            }
            scan_row<4>(J, R, sc, (sc.flags & 1) != 0, lds ? lds_row : Dg, Sg, use_tlist, t_count, u.q1, n, L, sh,
                        ovf_s, ovf_d);
            __syncthreads();
            const int32_t nb = sh.nb;
            if (role == 0) {
                const ItemRegion ir = item_region_at(items + (size_t)(region0 + item) * region_bytes, n_layout);
                for (int32_t i = tid; i < nb; i += bs) {
                    ir.t[i] = u.bl_t[i];
                    ir.d[i] = u.bl_d[i];
                    ir.s[i] = u.bl_s[i];
                }
                if (tid == 0) *ir.nb = nb;
            }
            if (nb == 0) continue;
            if (role != 1 && tid == 0) sh.counter += (unsigned long long)nb;
            // a B of half the row or more makes the sub-DAG most of DAG(s):
            // take every vertex's DAG in-arcs instead of walking back from B.
            // Below that the walk is cheaper: a hub update's changed targets
            // hang mostly below the hub, so their new ancestors are little
            // more than B itself (a hub update with 19 000 deferred sources
            // took 80 ms this way, 127 ms with whole-DAG passes from 1/16)
            const bool full = (int64_t)nb * 2 >= (int64_t)n;
            bool preds_done = false;
            // phase 0: old pass (roles 0 and 2); phase 1: new pass (roles 1 and 2)
            for (int ph = role == 1 ? 1 : 0; ph <= (role == 0 ? 0 : 1); ++ph) {
                const int32_t *Dr = lds ? lds_row : Dg;
                const uint64_t *Sr = Sg;
                if (ph == 1) {
                    if (role == 1) {
                        // the new row and counts: the old ones with the changed pairs in
                        int32_t *Dn = lds ? lds_row : u.dnew;
                        if (!lds)
                            for (int32_t t = tid; t < n; t += bs) u.dnew[t] = Dg[t];
                        for (int32_t t = tid; t < n; t += bs) u.snew[t] = Sg[t];
                        __syncthreads();
                        for (int32_t i = tid; i < nb; i += bs) {
                            const int32_t t = u.bl_t[i];
                            if (edge) pred_row[t] = edge_pred(J, t, pred_row[t], u.bl_d[i] < Dn[t]);
                            Dn[t] = u.bl_d[i];
                            u.snew[t] = u.bl_s[i];
                        }
                        Dr = Dn;
                        Sr = u.snew;
                    } else {
                        int32_t *Dw = J.g.D + (size_t)s * n;
                        uint64_t *Sw = J.g.S + (size_t)s * n;
                        for (int32_t i = tid; i < nb; i += bs) {
                            const int32_t t = u.bl_t[i];
                            const int32_t d = u.bl_d[i];
                            if (edge) pred_row[t] = edge_pred(J, t, pred_row[t], d < (lds ? lds_row[t] : Dw[t]));
                            Sw[t] = u.bl_s[i];
                            Dw[t] = d;
                            if (lds) lds_row[t] = d;
                        }
                    }
                    __syncthreads();
                }
                // The old pass of a paired source tests its B vertices' E*
                // in-arcs, so it never uses a stored predecessor that its new
                // pass (another workgroup, at the same time) rewrites: its walk
                // may load one ahead, but stops at the B vertex, which is in the
                // sub-DAG from the start.  A source updated by one workgroup
                // rewrites its predecessors only after the old pass, so that
                // pass takes the B vertices' stored (old) predecessors.  The new
                // pass of a one-arc update takes theirs from Alg 2 (written
                // above); other updates test the B vertices' E* in-arcs and
                // write the predecessors from the arc record
                preds_done = restricted_pass<false, 2, 4>(
                    s, n, Dr, Sr, ph ? J.g.yc_ptr : J.g.xc_ptr, ph ? J.g.yc_src : J.g.xc_src,
                    ph ? J.g.yc_dst : J.g.xc_dst, ph ? J.g.yc_w : J.g.xc_w, u.bl_t, nb, full, u, ph ? 1.0 : -1.0,
                    J.g.bc_delta, pred_row, ph && !edge ? pred_row : nullptr, ph ? edge : role == 2, sh, es);
            }
            // the new row of the new pass: in LDS, in the slot (role 1 without
            // staging) or written back to D (role 2)
            if (role != 0 && !preds_done && !edge)
                refresh_preds<1>(lds ? lds_row : role == 1 ? u.dnew : Dg, J.g.yc_ptr, J.g.yc_src, J.g.yc_w, u.bl_t, nb,
                                 pred_row, sh, es);
        }
        if (ovf_s) atomicOr(&ctl->status, ST_SIGMA_OVF);
        if (ovf_d) atomicOr(&ctl->status, ST_DIST_OVF);
        __syncthreads();
        if (tid == 0 && sh.counter) atomicAdd(&ctl->changed_pairs, sh.counter);
        region0 += paired;
    }
}

// Writes the changed pairs of the deferred sources whose two passes ran
// apart (same item-region assignment as k_source_wide).
__global__ void __launch_bounds__(256) k_wide_apply(const UpdateJob *__restrict__ jobs,
                                                    const int32_t *__restrict__ njobs_p, char *__restrict__ items,
                                                    int32_t item_regions, int32_t n_layout) {
    const int njobs = *njobs_p;
    const size_t region_bytes = item_region_bytes(n_layout);
    int32_t region0 = 0;
    for (int j = 0; j < njobs; ++j) {
        const UpdateJob &J = jobs[j];
        const int32_t n = J.g.n;
        const int32_t count = *(volatile int32_t *)&J.g.ctl->big_count;
        const int32_t paired = min(count, item_regions - region0);
        // a job halted since (or before) the wide kernel ran gets no writes;
        // its regions are still counted, as in k_source_wide
        if (job_halted(J)) {
            region0 += paired;
            continue;
        }
        // a group of gridDim / paired workgroups (at least one) per source,
        // sharing its changed pairs (a few sources can hold tens of thousands
        // each), four in flight per lane
        constexpr int U = 4;
        const int32_t per = paired > 0 ? max(1, (int32_t)gridDim.x / paired) : 1;
        for (int32_t w = blockIdx.x; w < paired * per; w += gridDim.x) {
            const int32_t item = w / per, slice = w % per;
            const ItemRegion ir = item_region_at(items + (size_t)(region0 + item) * region_bytes, n_layout);
            const int32_t s = J.g.biglist[item];
            const int32_t nb = *ir.nb;
            int32_t *Dg = J.g.D + (size_t)s * n;
            uint64_t *Sg = J.g.S + (size_t)s * n;
            const int32_t stride = per * (int32_t)blockDim.x;
            for (int32_t i0 = slice * (int32_t)blockDim.x + (int32_t)threadIdx.x; i0 < nb; i0 += U * stride) {
                int32_t tv[U], dv[U];
                uint64_t sv[U];
#pragma unroll
                for (int k = 0; k < U; ++k) {
                    const int32_t i = i0 + k * stride;
                    tv[k] = -1;
                    if (i < nb) {
                        tv[k] = ir.t[i];
                        dv[k] = ir.d[i];
                        sv[k] = ir.s[i];
                    }
                }
#pragma unroll
                for (int k = 0; k < U; ++k)
                    if (tv[k] >= 0) {
                        Dg[tv[k]] = dv[k];
                        Sg[tv[k]] = sv[k];
                    }
            }
        }
        region0 += paired;
    }
}

// ------------------------------------------------------------ commit -------

// BC(x) += bc_delta(x) as a compensated (hi, lo) pair (Knuth's two-sum),
// then clears bc_delta and the per-update counters.
__global__ void __launch_bounds__(256) k_commit(const UpdateJob *__restrict__ jobs, const int32_t *__restrict__ njobs_p,
                                                int32_t replace) {
    const int njobs = *njobs_p;
    for (int j = blockIdx.y; j < njobs; j += gridDim.y) {  // a row of blocks per job
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
            c->big_last = c->big_count;
            // algorithmic bytes of the row scans: per affected source its
            // distance row (4n) or, with the candidate list, the distances at
            // the candidates (4|T|); sigma is read for the changed pairs only
            const unsigned long long a = (unsigned long long)c->a_count, t = (unsigned long long)c->t_count;
            const bool tl = (int64_t)c->t_count * 8 <= (int64_t)n;
            c->scan_bytes_last = a * 4ull * (tl ? t : (unsigned long long)n) + 8ull * c->changed_pairs;
            if (!replace) {
                c->updates += 1;
                c->affected_total += (unsigned long long)c->a_count;
                c->changed_total += c->changed_pairs;
                c->scan_bytes_total += c->scan_bytes_last;
            }
            c->a_count = 0;
            c->work_next = 0;
            c->big_count = 0;
            c->big_next = 0;
            c->dag_count = 0;
            c->dag_next = 0;
            c->dag_next_light = 0;
            c->dag_back = 0;
        }
    }
}

// Clears the statistics that accumulate during an update (before k_scan).
__global__ void k_begin(const UpdateJob *__restrict__ jobs, const int32_t *__restrict__ njobs_p, StepPool pool) {
    const int njobs = *njobs_p;
    if (threadIdx.x == 0) *pool.next = 0;
    for (int j = threadIdx.x; j < njobs; j += blockDim.x) {
        GraphCtl *c = jobs[j].g.ctl;
        c->changed_pairs = 0;
        c->a_count = 0;
        c->work_next = 0;
        c->t_count = 0;
        c->big_count = 0;
        c->big_next = 0;
        c->dag_count = 0;
        c->dag_next = 0;
        c->dag_next_light = 0;
        c->dag_back = 0;
    }
}

// ------------------------------------------------------------ static pass --

// Distances from every source: frontier Bellman-Ford with the row in LDS
// (atomicMin relaxations; a vertex improved in a round is queued once for
// the next round).  Positive weights make it converge to d(s,.).  The search
// relaxes the arcs of the set given by tail (sptr, sdst, sw): every arc of
// the graph, or a set known or checked to contain E* (Section 6: any arc set
// containing E* gives the same distances).
// Arcs per lane in flight in the static search's frontier expansion.
constexpr int SU = 4;

__global__ void __launch_bounds__(1024) k_sssp(const UpdateJob *__restrict__ jobs, char *__restrict__ scratch,
                                               size_t slot_bytes, int32_t lds_cap, int32_t n_layout,
                                               const int32_t *__restrict__ sptr, const int32_t *__restrict__ sdst,
                                               const int32_t *__restrict__ sw) {
    extern __shared__ __align__(16) char dyn_lds[];
    int32_t *const lds_row = (int32_t *)dyn_lds;
    const ExpandShared es = expand_at(dyn_lds, lds_cap);
    __shared__ BlockShared sh;
    const UpdateJob &J = jobs[0];
    const int32_t n = J.g.n;
    const bool lds = n <= lds_cap;
    const SSlot sl = sslot_at(scratch + (size_t)blockIdx.x * slot_bytes, n_layout);
    GraphCtl *ctl = J.g.ctl;
    const int tid = threadIdx.x, bs = blockDim.x;
    bool ovf = false;
    for (;;) {
        __syncthreads();
        if (tid == 0) sh.item = atomicAdd(&ctl->work_next, 1);
        __syncthreads();
        const int32_t s = sh.item;
        if (s >= n) break;
        // a relaxation whose sum reaches 2^31-1 is dropped; it overflows only
        // if nothing shorter ever reaches its head, which the check after the
        // search settles (long candidates that lose are no error)
        bool long_cand = false;
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
            // the frontier's out-arcs, arc-parallel: a block scan of the
            // frontier vertices' out-degrees, then SU consecutive arcs per
            // lane, so that a hub's arcs (thousands on a power-law graph)
            // spread over the workgroup instead of one lane walking them
            for (int32_t c = 0; c < qlen; c += bs) {
                const int32_t idx = c + tid;
                int32_t b0 = 0, deg = 0, da = INF32;
                if (idx < qlen) {
                    const int32_t a = cur[idx];
                    b0 = sptr[a];
                    deg = sptr[a + 1] - b0;
                    da = __atomic_load_n(&row[a], __ATOMIC_RELAXED);
                }
                int32_t total;
                const int32_t off = block_excl_scan(deg, sh.scan, total);
                es.off[tid] = off;
                es.beg[tid] = b0;
                es.dx[tid] = da;
                __syncthreads();
                const int32_t nv = min(bs, qlen - c);
                for (int32_t jb = tid * SU; jb < total; jb += bs * SU) {
                    int32_t iv[SU], ev[SU], bv[SU], wv[SU];
                    bool ok[SU];
                    chunk_arcs(es, nv, total, jb, iv, ev, ok);
#pragma unroll
                    for (int k = 0; k < SU; ++k) {
                        bv[k] = ok[k] ? sdst[ev[k]] : 0;
                        wv[k] = ok[k] ? sw[ev[k]] : 0;
                    }
#pragma unroll
                    for (int k = 0; k < SU; ++k) {
                        if (!ok[k]) continue;
                        const int64_t nd = (int64_t)es.dx[iv[k]] + wv[k];
                        if (nd >= INF32) {
                            long_cand = true;
                            continue;
                        }
                        const int32_t b = bv[k];
                        if ((int32_t)nd < __atomic_load_n(&row[b], __ATOMIC_RELAXED)) {
                            const int32_t old = atomicMin(&row[b], (int32_t)nd);
                            if ((int32_t)nd < old && atomicExch(&flag[b], 1) == 0) nxt[atomicAdd(&sh.next, 1)] = b;
                        }
                    }
                }
                __syncthreads();
            }
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
        if (__syncthreads_or(long_cand)) {
            // converged: a vertex still unreached that has an arc from a
            // reached one is reachable, and every path to it is 2^31-1 or
            // longer
            for (int32_t a = tid; a < n; a += bs) {
                if (__atomic_load_n(&row[a], __ATOMIC_RELAXED) == INF32) continue;
                const int32_t e1 = sptr[a + 1];
                for (int32_t e = sptr[a]; e < e1; ++e)
                    if (__atomic_load_n(&row[sdst[e]], __ATOMIC_RELAXED) == INF32) ovf = true;
            }
        }
        if (lds)
            for (int32_t i = tid; i < n; i += bs) Dg[i] = row[i];
    }
    if (ovf) atomicOr(&ctl->status, ST_DIST_OVF);
}

// Check of a searched arc set H against every arc of the graph (by tail in
// arc_ptr / arc_dst / arc_w), with D the distances the search over H found:
// the arcs (a,b) with w(a,b) <= D(a,b) go to the out list (up to cap; *cnt
// counts them all).  An arc of E* has w(a,b) = d(a,b) <= D(a,b), so it is
// listed unless H holds it; and when every listed arc is in H, no path can
// be shortened by an arc outside H (its weight exceeds the H-distance of its
// ends), so D is the graph's distance matrix and H contains E*.  One wave
// per tail (the tail's arcs and its distance row are contiguous).
__global__ void __launch_bounds__(256) k_search_check(const UpdateJob *__restrict__ jobs, int32_t *__restrict__ out_a,
                                                      int32_t *__restrict__ out_b, int32_t *__restrict__ out_w,
                                                      int64_t cap, unsigned long long *__restrict__ cnt) {
    const UpdateJob &J = jobs[0];
    const int32_t n = J.g.n;
    const int lane = lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t a = wave; a < n; a += nwaves) {
        const int32_t *Da = J.g.D + (size_t)a * n;
        const int32_t p0 = J.g.arc_ptr[a], p1 = J.g.arc_ptr[a + 1];
        for (int32_t base = p0; base < p1; base += 64) {
            const int32_t i = base + lane;
            bool keep = false;
            int32_t b = 0, w = 0;
            if (i < p1) {
                b = J.g.arc_dst[i];
                w = J.g.arc_w[i];
                const int32_t d = Da[b];
                keep = d == INF32 || w <= d;
            }
            const uint64_t mask = __ballot(keep);
            if (!mask) continue;
            unsigned long long b0 = 0;
            const int leader = __ffsll((unsigned long long)mask) - 1;
            if (lane == leader) b0 = atomicAdd(cnt, (unsigned long long)__popcll(mask));
            b0 = __shfl(b0, leader, 64);
            if (keep) {
                const unsigned long long o = b0 + popc_below(mask, lane);
                if ((int64_t)o < cap) {
                    out_a[o] = (int32_t)a;
                    out_b[o] = b;
                    out_w[o] = w;
                }
            }
        }
    }
}

// Per source after the distances and E* exist: path counts pushed in Kahn
// order (sigma_sb = sum over DAG predecessors a of sigma_sa, Alg 6 step 7),
// then the dependency pull, BC += delta (Alg 1 line 5).
__global__ void __launch_bounds__(1024) k_static(const UpdateJob *__restrict__ jobs, char *__restrict__ scratch,
                                                 size_t slot_bytes, int32_t lds_cap, int32_t n_layout) {
    extern __shared__ int32_t lds_row[];
    __shared__ BlockShared sh;
    const UpdateJob &J = jobs[0];
    const int32_t n = J.g.n;
    const bool lds = n <= lds_cap;
    const SSlot sl = sslot_at(scratch + (size_t)blockIdx.x * slot_bytes, n_layout);
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
        static_dag_pass(s, n, Drow, J.g.S + (size_t)s * n, J.g.pred + (size_t)s * n, J.g.x_ptr, J.g.x_src, J.g.x_dst,
                        J.g.x_w, ctl->es_m, sl, J.g.bc_delta, ctl, sh);
    }
}

__global__ void k_reset_work(GraphCtl *ctl) {
    ctl->work_next = 0;
    ctl->a_count = 0;
}

// ------------------------------------------------------------ introspection

// Dependency row of one source, delta_s.(x) = sum over all reachable t of
// delta_st(x), by the same restricted pass with B = every reachable t != s.
// Writes the row to out_row (n values, 0 at s and at unreachable x).  One
// workgroup; `scratch` is one wide-kernel slot laid out for n_layout >= n.
__device__ __forceinline__ void delta_row(const GraphPtrs &G, int32_t s, char *__restrict__ scratch, int32_t lds_cap,
                                          int32_t n_layout, double *out_row) {
    extern __shared__ __align__(16) char dyn_lds[];
    int32_t *const lds_row = (int32_t *)dyn_lds;
    const ExpandShared es = expand_at(dyn_lds, lds_cap);
    __shared__ BlockShared sh;
    const int32_t n = G.n;
    const bool lds = n <= lds_cap;
    const USlot u = wslot_at(scratch, n_layout);
    if ((*(volatile int32_t *)&G.ctl->status & ST_ESTAR_CAP) != 0) return;
    const int32_t *Dg = G.D + (size_t)s * n;
    const int32_t *Drow = Dg;
    if (threadIdx.x == 0) sh.nb = 0;
    __syncthreads();
    for (int32_t t = threadIdx.x; t < n; t += blockDim.x) {
        out_row[t] = 0.0;
        if (lds) lds_row[t] = Dg[t];
        if (t != s && Dg[t] != INF32) u.bl_t[atomicAdd(&sh.nb, 1)] = t;
    }
    if (lds) Drow = lds_row;
    __syncthreads();
    restricted_pass<true, XU>(s, n, Drow, G.S + (size_t)s * n, G.xc_ptr, G.xc_src, G.xc_dst, G.xc_w, u.bl_t, sh.nb,
                              true, u, 1.0, out_row, nullptr, nullptr, false, sh, es);
}

__global__ void __launch_bounds__(1024) k_delta_row(const UpdateJob *__restrict__ jobs, int32_t s, char *__restrict__ scratch,
                                                    int32_t lds_cap, int32_t n_layout, double *out_row) {
    delta_row(jobs[0].g, s, scratch, lds_cap, n_layout, out_row);
}

// The same with the graph's pointers passed by value (no staged job) and the
// slot in the caller-supplied scratch address (the library's fixed array).
__global__ void __launch_bounds__(1024) k_delta_row_byval(const GraphPtrs G, int32_t s, char *__restrict__ scratch,
                                                          int32_t lds_cap, int32_t n_layout, double *out_row) {
    delta_row(G, s, scratch, lds_cap, n_layout, out_row);
}

// Zero fill of a byte range (the fixed scratch array at set-up).
__global__ void __launch_bounds__(256) k_zero_fill(char *__restrict__ p, size_t bytes) {
    const size_t words = bytes / 8;
    uint64_t *q = (uint64_t *)p;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (size_t)gridDim.x * blockDim.x)
        q[i] = 0;
}

// Sticky status words of up to STATUS_GATHER graphs gathered into one device
// array by one launch, so that reading back many graphs' errors costs one
// launch and one copy instead of a copy per graph.
constexpr int STATUS_GATHER = 64;
struct StatusPtrs {
    const int32_t *p[STATUS_GATHER];
};
__global__ void __launch_bounds__(STATUS_GATHER) k_gather_status(const StatusPtrs a, int32_t count,
                                                                 int32_t *__restrict__ out) {
    const int i = threadIdx.x;
    if (i < count) out[i] = *(const volatile int32_t *)a.p[i];
}

// Arcs of DAG(s): the predicate of Eq.1 over E*.
__global__ void k_dag_arcs(const UpdateJob *__restrict__ jobs, int32_t s, int32_t *out_a, int32_t *out_b, int64_t cap,
                           unsigned long long *cnt) {
    const UpdateJob &J = jobs[0];
    if (job_dead(J)) return;
    const int32_t n = J.g.n, m = J.g.ctl->esc_m;
    const int32_t *Drow = J.g.D + (size_t)s * n;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t a = J.g.xc_src[i], b = J.g.xc_dst[i];
        const int32_t da = Drow[a], db = Drow[b];
        if (da != INF32 && db != INF32 && (int64_t)da + J.g.xc_w[i] == (int64_t)db) {
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
