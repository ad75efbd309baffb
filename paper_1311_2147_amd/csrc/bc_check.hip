// State check of libbcinc, a debugging aid (BC_FLAG_CHECK after every update
// step, bc_check on demand): the distance, path-count and stored-predecessor
// rows of chosen sources, and all of E*, are tested against their
// definitions over the graph's current arcs.  The update kernels never read
// what these kernels write, apart from the sticky status bit that halts a
// graph whose state failed a check.

namespace bcinc {

// Sticky status bit of a failed check, beside the ST_* bits.
constexpr int32_t ST_CHECK = 8;
static_assert((ST_CHECK & (ST_SIGMA_OVF | ST_DIST_OVF | ST_ESTAR_CAP)) == 0, "status bits overlap");

// Kinds of a failed check (the public BC_CHECK_* codes).
enum : int32_t {
    CK_SOURCE = 1,     // d(s,s) != 0, sigma_ss != 1 or a stored predecessor at s
    CK_RELAX = 2,      // an in-arc (a,t) with d(s,a) + w < d(s,t), or finite into an infinite d(s,t)
    CK_NO_PATH = 3,    // finite d(s,t) that no in-arc meets
    CK_SIGMA = 4,      // sigma_st is not the sum over the DAG(s) in-arcs of t
    CK_PRED = 5,       // stored predecessor not the one Eq.1 gives
    CK_UNREACHED = 6,  // infinite d(s,t) with a path count or a predecessor
    CK_SYMMETRY = 7,   // undirected graph: (s,t) and (t,s) differ
    CK_ESTAR = 8       // the E* arcs into t are not the arcs with w(a,t) = d(a,t)
};

// Per-graph record of the checks since load, in the graph's arena.
struct CheckRec {
    unsigned long long rows;   // source rows verified
    unsigned long long fails;  // conditions found false
    int32_t s, t, kind;        // the first of them: source (E*: tail, -1 if none), target (E*: head), kind
};

__device__ void check_fail(GraphCtl *ctl, CheckRec *rec, int32_t s, int32_t t, int32_t kind) {
    if (atomicAdd(&rec->fails, 1ull) == 0) {
        rec->s = s;
        rec->t = t;
        rec->kind = kind;
    }
    atomicOr(&ctl->status, ST_CHECK);
}

// Rows of the sources of the last update (alist, affected_last entries), or
// of every source (all != 0), with the current arcs by head in arcin_*.  For
// a source s and a target t != s, over the in-arcs (a,t) of weight w whose
// tail is reachable from s:
//   * none is shorter: d(s,a) + w >= d(s,t), and none reaches an infinite
//     d(s,t);
//   * finite d(s,t): some in-arc is tight (d(s,a) + w = d(s,t)), sigma_st is
//     the sum of sigma_sa over the tight ones (Eq.1 picks the DAG(s) arcs),
//     and the stored predecessor is the tail of the only tight one, or
//     PRED_MULTI for several;
//   * infinite d(s,t): sigma_st = 0 and PRED_NONE;
// at t = s: d = 0, sigma = 1, PRED_NONE; and for an undirected graph
// d(t,s) = d(s,t), sigma_ts = sigma_st.  With positive weights the first two
// fix d and sigma: following tight arcs back from t lowers d strictly and
// can stop only at s, so d(s,t) is the length of a path that no arc can
// shorten, and sigma follows by induction on d.  A thread per (s, t).
__global__ void __launch_bounds__(256) k_check_rows(const GraphPtrs G, CheckRec *__restrict__ rec, int32_t all) {
    GraphCtl *const ctl = G.ctl;
    if (*(volatile int32_t *)&ctl->status != 0) return;  // no valid state to check
    const int32_t n = G.n;
    const int64_t ns = all ? (int64_t)n : min((int64_t)ctl->affected_last, (int64_t)n);  // alist holds n
    const int64_t chunks = ((int64_t)n + blockDim.x - 1) / blockDim.x;
    for (int64_t it = blockIdx.x; it < ns * chunks; it += gridDim.x) {
        const int64_t si = it / chunks;
        const int32_t s = all ? (int32_t)si : G.alist[si];
        const int32_t t = (int32_t)((it % chunks) * blockDim.x + threadIdx.x);
        if (s < 0 || s >= n) {
            if (t == 0) check_fail(ctl, rec, s, -1, CK_SOURCE);
            continue;
        }
        if (t == 0) atomicAdd(&rec->rows, 1ull);
        if (t >= n) continue;
        const size_t row = (size_t)s * n;
        const int32_t dt = G.D[row + t];
        const uint64_t st = G.S[row + t];
        const int32_t pt = G.pred[row + t];
        int32_t kind = 0;
        if (t == s) {
            if (dt != 0 || st != 1 || pt != PRED_NONE) kind = CK_SOURCE;
        } else {
            uint64_t sum = 0;
            bool carry = false;
            int32_t tight = 0, tail = PRED_NONE;
            for (int32_t e = G.arcin_ptr[t]; e < G.arcin_ptr[t + 1]; ++e) {
                const int32_t a = G.arcin_src[e];
                const int32_t da = G.D[row + a];
                if (da == INF32) continue;
                const int64_t c = (int64_t)da + G.arcin_w[e];
                if (dt == INF32 || c < (int64_t)dt) {
                    kind = CK_RELAX;
                    break;
                }
                if (c == (int64_t)dt) {
                    const uint64_t sa = G.S[row + a];
                    carry |= sum + sa < sum;
                    sum += sa;
                    ++tight;
                    tail = a;
                }
            }
            if (kind) {
            } else if (dt == INF32) {
                if (st != 0 || pt != PRED_NONE) kind = CK_UNREACHED;
            } else if (tight == 0) {
                kind = CK_NO_PATH;
            } else if (carry || sum != st) {
                kind = CK_SIGMA;
            } else if (pt != (tight == 1 ? tail : PRED_MULTI)) {
                kind = CK_PRED;
            }
        }
        if (!kind && !G.directed && (G.D[(size_t)t * n + s] != dt || G.S[(size_t)t * n + s] != st))
            kind = CK_SYMMETRY;
        if (kind) check_fail(ctl, rec, s, t, kind);
    }
}

// E* by head (XC) against the current arcs by head (tails ascending within a
// head): the XC arcs into b are exactly the arcs (a,b) with w(a,b) = d(a,b),
// each once and with its current weight.  A thread per head.
__global__ void __launch_bounds__(256) k_check_estar(const GraphPtrs G, CheckRec *__restrict__ rec) {
    GraphCtl *const ctl = G.ctl;
    if (*(volatile int32_t *)&ctl->status != 0) return;
    const int32_t n = G.n;
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < n; b += (int64_t)gridDim.x * blockDim.x) {
        const int32_t p0 = G.arcin_ptr[b], p1 = G.arcin_ptr[b + 1];
        int32_t tight = 0;
        for (int32_t e = p0; e < p1; ++e) tight += G.D[(size_t)G.arcin_src[e] * n + b] == G.arcin_w[e];
        const int32_t x0 = G.xc_ptr[b], x1 = G.xc_ptr[b + 1];
        int32_t bad_tail = -1;
        bool bad = x0 < 0 || x1 < x0 || (int64_t)x1 > G.es_cap || x1 - x0 != tight;
        for (int32_t i = x0; i < x1 && !bad; ++i) {
            const int32_t a = G.xc_src[i], w = G.xc_w[i];
            bad = G.xc_dst[i] != b || a < 0 || a >= n || G.D[(size_t)a * n + b] != w;
            if (!bad) {
                int32_t lo = p0, hi = p1;
                while (lo < hi) {
                    const int32_t mid = (lo + hi) >> 1;
                    if (G.arcin_src[mid] < a) lo = mid + 1;
                    else hi = mid;
                }
                bad = lo == p1 || G.arcin_src[lo] != a || G.arcin_w[lo] != w;
            }
            for (int32_t k = x0; k < i && !bad; ++k) bad = G.xc_src[k] == a;
            if (bad) bad_tail = a;
        }
        if (bad) check_fail(ctl, rec, bad_tail, (int32_t)b, CK_ESTAR);
    }
}

}  // namespace bcinc
