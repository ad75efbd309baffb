/*
 * Multi-core CPU comparator for the incremental BC update.
 *
 * A plain C / OpenMP implementation of the paper's decremental-weight update
 * on the CPU, kept beside the GPU library only as a comparator: it shows how
 * much of the GPU's speed comes from the incremental algorithm itself and how
 * much from the GPU.  Nothing in the GPU library calls it, and it has no
 * fallback role.
 *
 * What one arc update (u, v) to weight w (a decrease, or an insertion) does,
 * per source s, in parallel over the sources:
 *   - Lemma 2: with c = d(s,u) + w, a source is affected when c <= d(s,v);
 *     then for every t, c + d(v,t) < d(s,t) gives d'(s,t) = c + d(v,t) and
 *     sigma'_st = sigma_su * sigma_vt, and c + d(v,t) = d(s,t) gives
 *     sigma'_st = sigma_st + sigma_su * sigma_vt.  Row v and column u do not
 *     change (a path through (u,v) back to v or to u is a cycle), so the
 *     sources never read a pair another source writes.
 *   - The changed pairs B_s are the only targets whose shortest s-t paths
 *     change, so the source dependency changes by delta'_B - delta_B, the
 *     partial dependencies over B_s (Eq.4 restricted to targets in B_s): each
 *     is accumulated over the ancestors of B_s in DAG(s) (Eq.1 over the
 *     in-arcs), in non-increasing distance order (a reverse topological
 *     order, Section 2.1), once on the old row and arcs, once on the new.
 *   - BC(x) += delta'_B(x) - delta_B(x) for every such x other than s (Eq.3).
 * A vertex update at v (Section 4) with new in-arcs E_i and out-arcs E_o
 * takes one pass over the sources, as the paper does:
 *   - Alg 4 per source over E_i: d'(s,v) (Eq.6), sigma'_sv, and the new
 *     paths sigma-hat'_sv (Eq.7) when d'(s,v) = d(s,v);
 *   - row v'' (the Out phase, Alg 4 on G'_R): d''(v,t) = min(d(v,t),
 *     min_j w'(v,x_j) + d'(x_j,t)) with sigma''_vt and the new paths
 *     sigma-hat''_vt, the rows x_j taken after the In phase;
 *   - Lemma 4 per pair, In phase with row v (d'(s,v) + d(v,t)), then on
 *     G'_R with row v'' (d'(s,v) + d''(v,t)); a tie adds only new paths.
 *   Row v is read from a snapshot, since source v rewrites it.
 * An undirected edge update {u,v} is the vertex form at u with E_i =
 * {(v,u)} and E_o = {(u,v)} (Section 3).
 *
 * Distances are int32 (INT32_MAX: unreachable; a sum that reaches it is a
 * distance overflow), path counts uint64 (every product and sum checked).
 */
#define _GNU_SOURCE /* qsort_r */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define IC_OK 0
#define IC_BAD_ARG -1
#define IC_NOT_DECREASE -2
#define IC_SIGMA_OVERFLOW -3
#define IC_DIST_OVERFLOW -4
#define IC_NOMEM -5

#define INF32 INT32_MAX

typedef struct {
    int32_t *t;     /* changed targets */
    int32_t *d;     /* their new distances */
    uint64_t *sg;   /* their new path counts */
    int32_t *list;  /* sub-DAG vertices */
    uint8_t *mark;  /* bit 0: in the sub-DAG, bit 1: in B */
    double *acc;    /* partial dependency */
    double *bcd;    /* this thread's BC change */
} scratch_t;

typedef struct {
    int32_t dv;      /* d'(s,v) */
    uint8_t same;    /* d'(s,v) = d(s,v) */
    uint8_t aff;     /* the source can change */
    uint64_t sv, hv; /* sigma'_sv, sigma-hat'_sv */
} scal_t;

typedef struct {
    int32_t n;
    int directed;
    int threads;
    /* the arcs of the update in progress: (ua, ub) gets weight uw (replacing
     * the stored arc or added); uhead marks their heads */
    int32_t nupd, upd_cap;
    int32_t *ua, *ub;
    int64_t *uw;
    uint8_t *uhead;
    scal_t *scal;                    /* per source */
    int32_t *rvD, *rvvD;             /* row v (snapshot) and row v'' */
    uint64_t *rvS, *rvvS, *rvvH;
    int32_t *D;      /* n x n */
    uint64_t *S;     /* n x n */
    double *bc;      /* n */
    int32_t *deg, *cap;
    int32_t **in_src; /* in-arcs by head */
    int64_t **in_w;
    scratch_t *sc;
} ic_t;

static int add_in_arc(ic_t *c, int32_t a, int32_t b, int64_t w) {
    if (c->deg[b] == c->cap[b]) {
        const int32_t nc = c->cap[b] ? 2 * c->cap[b] : 4;
        int32_t *ns = realloc(c->in_src[b], sizeof(int32_t) * (size_t)nc);
        if (!ns) return IC_NOMEM;
        c->in_src[b] = ns;
        int64_t *nw = realloc(c->in_w[b], sizeof(int64_t) * (size_t)nc);
        if (!nw) return IC_NOMEM;
        c->in_w[b] = nw;
        c->cap[b] = nc;
    }
    c->in_src[b][c->deg[b]] = a;
    c->in_w[b][c->deg[b]] = w;
    c->deg[b]++;
    return IC_OK;
}

/* current weight of arc (a, b), or -1 when absent */
static int64_t arc_weight(const ic_t *c, int32_t a, int32_t b) {
    for (int32_t i = 0; i < c->deg[b]; ++i)
        if (c->in_src[b][i] == a) return c->in_w[b][i];
    return -1;
}

void icpu_destroy(void *h) {
    ic_t *c = (ic_t *)h;
    if (!c) return;
    if (c->in_src)
        for (int32_t i = 0; i < c->n; ++i) free(c->in_src[i]);
    if (c->in_w)
        for (int32_t i = 0; i < c->n; ++i) free(c->in_w[i]);
    free(c->in_src);
    free(c->in_w);
    free(c->deg);
    free(c->cap);
    if (c->sc) {
        for (int i = 0; i < c->threads; ++i) {
            scratch_t *x = &c->sc[i];
            free(x->t);
            free(x->d);
            free(x->sg);
            free(x->list);
            free(x->mark);
            free(x->acc);
            free(x->bcd);
        }
        free(c->sc);
    }
    free(c->D);
    free(c->S);
    free(c->bc);
    free(c->ua);
    free(c->ub);
    free(c->uw);
    free(c->uhead);
    free(c->scal);
    free(c->rvD);
    free(c->rvvD);
    free(c->rvS);
    free(c->rvvS);
    free(c->rvvH);
    free(c);
}

/* A graph with no state yet (every pair unreachable, sigma 0, BC 0): the
 * caller sets rows and scores from a computed state before updating. */
int icpu_create(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, const int64_t *w, int directed,
                int threads, void **out) {
    if (n < 1 || m < 0 || !out || (m > 0 && (!src || !dst || !w))) return IC_BAD_ARG;
    ic_t *c = calloc(1, sizeof(ic_t));
    if (!c) return IC_NOMEM;
    c->n = n;
    c->directed = directed;
    c->threads = threads > 0 ? threads : omp_get_max_threads();
    const size_t nn = (size_t)n * (size_t)n;
    c->D = malloc(sizeof(int32_t) * nn);
    c->S = calloc(nn, sizeof(uint64_t));
    c->bc = calloc((size_t)n, sizeof(double));
    c->deg = calloc((size_t)n, sizeof(int32_t));
    c->cap = calloc((size_t)n, sizeof(int32_t));
    c->in_src = calloc((size_t)n, sizeof(int32_t *));
    c->in_w = calloc((size_t)n, sizeof(int64_t *));
    c->sc = calloc((size_t)c->threads, sizeof(scratch_t));
    c->uhead = calloc((size_t)n, 1);
    c->scal = calloc((size_t)n, sizeof(scal_t));
    c->rvD = malloc(sizeof(int32_t) * (size_t)n);
    c->rvvD = malloc(sizeof(int32_t) * (size_t)n);
    c->rvS = malloc(sizeof(uint64_t) * (size_t)n);
    c->rvvS = malloc(sizeof(uint64_t) * (size_t)n);
    c->rvvH = malloc(sizeof(uint64_t) * (size_t)n);
    if (!c->D || !c->S || !c->bc || !c->deg || !c->cap || !c->in_src || !c->in_w || !c->sc || !c->uhead || !c->scal ||
        !c->rvD || !c->rvvD || !c->rvS || !c->rvvS || !c->rvvH) {
        icpu_destroy(c);
        return IC_NOMEM;
    }
    for (size_t i = 0; i < nn; ++i) c->D[i] = INF32;
    for (int i = 0; i < c->threads; ++i) {
        scratch_t *x = &c->sc[i];
        x->t = malloc(sizeof(int32_t) * (size_t)n);
        x->d = malloc(sizeof(int32_t) * (size_t)n);
        x->sg = malloc(sizeof(uint64_t) * (size_t)n);
        x->list = malloc(sizeof(int32_t) * (size_t)n);
        x->mark = calloc((size_t)n, 1);
        x->acc = calloc((size_t)n, sizeof(double));
        x->bcd = calloc((size_t)n, sizeof(double));
        if (!x->t || !x->d || !x->sg || !x->list || !x->mark || !x->acc || !x->bcd) {
            icpu_destroy(c);
            return IC_NOMEM;
        }
    }
    for (int64_t i = 0; i < m; ++i) {
        const int32_t a = src[i], b = dst[i];
        if (a < 0 || a >= n || b < 0 || b >= n || a == b || w[i] < 1 || w[i] >= INF32) {
            icpu_destroy(c);
            return IC_BAD_ARG;
        }
        int rc = add_in_arc(c, a, b, w[i]);
        if (!rc && !directed) rc = add_in_arc(c, b, a, w[i]);
        if (rc) {
            icpu_destroy(c);
            return rc;
        }
    }
    *out = c;
    return IC_OK;
}

/* rows s0 .. s0+cnt-1 of a computed state: int64 distances (INT64_MAX:
 * unreachable) and uint64 path counts */
int icpu_set_rows(void *h, int32_t s0, int32_t cnt, const int64_t *D, const uint64_t *S) {
    ic_t *c = (ic_t *)h;
    if (!c || s0 < 0 || cnt < 0 || s0 + (int64_t)cnt > c->n) return IC_BAD_ARG;
    const size_t len = (size_t)cnt * (size_t)c->n;
    for (size_t i = 0; i < len; ++i) {
        const int64_t d = D[i];
        if (d != INT64_MAX && (d < 0 || d >= INF32)) return IC_DIST_OVERFLOW;
    }
    int32_t *Dd = c->D + (size_t)s0 * c->n;
    for (size_t i = 0; i < len; ++i) Dd[i] = D[i] == INT64_MAX ? INF32 : (int32_t)D[i];
    memcpy(c->S + (size_t)s0 * c->n, S, sizeof(uint64_t) * len);
    return IC_OK;
}

int icpu_get_rows(void *h, int32_t s0, int32_t cnt, int64_t *D, uint64_t *S) {
    ic_t *c = (ic_t *)h;
    if (!c || s0 < 0 || cnt < 0 || s0 + (int64_t)cnt > c->n) return IC_BAD_ARG;
    const size_t len = (size_t)cnt * (size_t)c->n;
    const int32_t *Dd = c->D + (size_t)s0 * c->n;
    for (size_t i = 0; i < len; ++i) D[i] = Dd[i] == INF32 ? INT64_MAX : (int64_t)Dd[i];
    memcpy(S, c->S + (size_t)s0 * c->n, sizeof(uint64_t) * len);
    return IC_OK;
}

int icpu_set_scores(void *h, const double *bc) {
    ic_t *c = (ic_t *)h;
    if (!c || !bc) return IC_BAD_ARG;
    memcpy(c->bc, bc, sizeof(double) * (size_t)c->n);
    return IC_OK;
}

int icpu_get_scores(void *h, double *bc) {
    ic_t *c = (ic_t *)h;
    if (!c || !bc) return IC_BAD_ARG;
    memcpy(bc, c->bc, sizeof(double) * (size_t)c->n);
    return IC_OK;
}

static int cmp_desc(const void *x, const void *y, void *ctx) {
    const int32_t *D = (const int32_t *)ctx;
    const int32_t a = D[*(const int32_t *)x], b = D[*(const int32_t *)y];
    return a < b ? 1 : a > b ? -1 : 0;
}

/* insertion sort for short lists, else qsort_r (both by distance, descending) */
static void sort_by_dist_desc(int32_t *v, int32_t k, const int32_t *D) {
    if (k <= 32) {
        for (int32_t i = 1; i < k; ++i) {
            const int32_t x = v[i];
            int32_t j = i - 1;
            while (j >= 0 && D[v[j]] < D[x]) {
                v[j + 1] = v[j];
                --j;
            }
            v[j + 1] = x;
        }
    } else {
        qsort_r(v, (size_t)k, sizeof(int32_t), cmp_desc, (void *)D);
    }
}

static int in_update(const ic_t *c, int32_t a, int32_t b) {
    for (int32_t k = 0; k < c->nupd; ++k)
        if (c->ua[k] == a && c->ub[k] == b) return 1;
    return 0;
}

/* The DAG in-arcs (a, x) of x in row Drow: in-arcs with d(s,a) + w =
 * d(s,x) (Eq.1).  With ovl set, the arcs of the update in progress carry
 * their new weights. */
#define FOR_DAG_IN_ARCS(c, Drow, x, ovl, BODY)                                                  \
    do {                                                                                        \
        const int32_t dx_ = (Drow)[x];                                                          \
        const int up_ = (ovl) && (c)->uhead[x];                                                 \
        for (int32_t i_ = 0; i_ < (c)->deg[x]; ++i_) {                                          \
            const int32_t a = (c)->in_src[x][i_];                                               \
            if (up_ && in_update(c, a, x)) continue;                                            \
            const int32_t da_ = (Drow)[a];                                                      \
            if (da_ != INF32 && (int64_t)da_ + (c)->in_w[x][i_] == (int64_t)dx_) { BODY }       \
        }                                                                                       \
        if (up_)                                                                                \
            for (int32_t k_ = 0; k_ < (c)->nupd; ++k_) {                                        \
                if ((c)->ub[k_] != (x)) continue;                                               \
                const int32_t a = (c)->ua[k_];                                                  \
                const int32_t da_ = (Drow)[a];                                                  \
                if (da_ != INF32 && (int64_t)da_ + (c)->uw[k_] == (int64_t)dx_) { BODY }        \
            }                                                                                   \
    } while (0)

/* delta_B(x) (Eq.4 over the targets in B) for every ancestor x of B in the
 * DAG of row (Drow, Srow); B is marked with bit 1.  Adds sign * delta_B(x)
 * to bcd[x] for x != s. */
static void partial_dependency(const ic_t *c, scratch_t *x, int32_t s, const int32_t *Drow, const uint64_t *Srow,
                               int32_t nb, double sign, int ovl) {
    int32_t k = 0;
    for (int32_t i = 0; i < nb; ++i) {
        const int32_t t = x->t[i];
        if (Drow[t] == INF32 || (x->mark[t] & 1)) continue;
        x->mark[t] |= 1;
        x->list[k++] = t;
    }
    /* backward search over DAG in-arcs: the ancestors of B */
    for (int32_t h = 0; h < k; ++h) {
        const int32_t y = x->list[h];
        FOR_DAG_IN_ARCS(c, Drow, y, ovl, {
            if (!(x->mark[a] & 1)) {
                x->mark[a] |= 1;
                x->list[k++] = a;
            }
        });
    }
    sort_by_dist_desc(x->list, k, Drow);
    for (int32_t h = 0; h < k; ++h) {
        const int32_t y = x->list[h];
        const double coef = (((x->mark[y] & 2) ? 1.0 : 0.0) + x->acc[y]) / (double)Srow[y];
        FOR_DAG_IN_ARCS(c, Drow, y, ovl, { x->acc[a] += (double)Srow[a] * coef; });
    }
    for (int32_t h = 0; h < k; ++h) {
        const int32_t y = x->list[h];
        if (y != s) x->bcd[y] += sign * x->acc[y];
        x->acc[y] = 0.0;
        x->mark[y] &= (uint8_t)~1u;
    }
}

/* The changed pairs of source s are in x->t/d/sg: old partial dependency,
 * the new values written, new partial dependency. */
static void apply_source(ic_t *c, scratch_t *x, int32_t s, int32_t nb) {
    int32_t *Ds = c->D + (size_t)s * c->n;
    uint64_t *Ss = c->S + (size_t)s * c->n;
    for (int32_t i = 0; i < nb; ++i) x->mark[x->t[i]] |= 2;
    partial_dependency(c, x, s, Ds, Ss, nb, -1.0, 0);
    for (int32_t i = 0; i < nb; ++i) {
        Ds[x->t[i]] = x->d[i];
        Ss[x->t[i]] = x->sg[i];
    }
    partial_dependency(c, x, s, Ds, Ss, nb, 1.0, 1);
    for (int32_t i = 0; i < nb; ++i) x->mark[x->t[i]] = 0;
}

/* After every source: the threads' BC changes, then the update's arcs. */
static int finish_update(ic_t *c) {
    for (int i = 0; i < c->threads; ++i) {
        double *b = c->sc[i].bcd;
        for (int32_t t = 0; t < c->n; ++t) {
            c->bc[t] += b[t];
            b[t] = 0.0;
        }
    }
    int rc = IC_OK;
    for (int32_t k = 0; k < c->nupd; ++k) {
        const int32_t a = c->ua[k], b = c->ub[k];
        c->uhead[b] = 0;
        int found = 0;
        for (int32_t i = 0; i < c->deg[b]; ++i)
            if (c->in_src[b][i] == a) {
                c->in_w[b][i] = c->uw[k];
                found = 1;
                break;
            }
        if (!found && !rc) rc = add_in_arc(c, a, b, c->uw[k]);
    }
    c->nupd = 0;
    return rc;
}

static int push_update_arc(ic_t *c, int32_t a, int32_t b, int64_t w) {
    if (c->nupd == c->upd_cap) {
        const int32_t nc = c->upd_cap ? 2 * c->upd_cap : 16;
        int32_t *na = realloc(c->ua, sizeof(int32_t) * (size_t)nc);
        if (!na) return IC_NOMEM;
        c->ua = na;
        int32_t *nb = realloc(c->ub, sizeof(int32_t) * (size_t)nc);
        if (!nb) return IC_NOMEM;
        c->ub = nb;
        int64_t *nw = realloc(c->uw, sizeof(int64_t) * (size_t)nc);
        if (!nw) return IC_NOMEM;
        c->uw = nw;
        c->upd_cap = nc;
    }
    c->ua[c->nupd] = a;
    c->ub[c->nupd] = b;
    c->uw[c->nupd] = w;
    c->nupd++;
    c->uhead[b] = 1;
    return IC_OK;
}

/* Lemma 2: the one arc (u, v) of the update list, weight w. */
static int arc_update(ic_t *c) {
    const int32_t n = c->n, u = c->ua[0], v = c->ub[0];
    const int64_t w = c->uw[0];
    int err = IC_OK;
    const int32_t *Dv = c->D + (size_t)v * n;
    const uint64_t *Sv = c->S + (size_t)v * n;
#pragma omp parallel num_threads(c->threads)
    {
        scratch_t *x = &c->sc[omp_get_thread_num()];
        int my_err = IC_OK;
#pragma omp for schedule(dynamic, 16)
        for (int32_t s = 0; s < n; ++s) {
            const int32_t *Ds = c->D + (size_t)s * n;
            const uint64_t *Ss = c->S + (size_t)s * n;
            const int32_t dsu = Ds[u];
            if (dsu == INF32 || s == v) continue;
            const int64_t cu = (int64_t)dsu + w;
            if (cu > (int64_t)Ds[v]) continue;
            const uint64_t su = Ss[u];
            int32_t nb = 0;
            for (int32_t t = 0; t < n; ++t) {
                const int32_t dvt = Dv[t];
                if (dvt == INF32 || t == s) continue;
                const int64_t nd = cu + dvt;
                const int32_t dst = Ds[t];
                if (nd > (int64_t)dst) continue;
                if (nd >= INF32) {
                    my_err = IC_DIST_OVERFLOW;
                    continue;
                }
                uint64_t add;
                if (__builtin_mul_overflow(su, Sv[t], &add)) {
                    my_err = IC_SIGMA_OVERFLOW;
                    continue;
                }
                uint64_t ns = add;
                if (nd == (int64_t)dst && __builtin_add_overflow(Ss[t], add, &ns)) {
                    my_err = IC_SIGMA_OVERFLOW;
                    continue;
                }
                if (nd == (int64_t)dst && add == 0) continue;
                x->t[nb] = t;
                x->d[nb] = (int32_t)nd;
                x->sg[nb] = ns;
                ++nb;
            }
            if (nb) apply_source(c, x, s, nb);
        }
        if (my_err) {
#pragma omp critical
            err = my_err;
        }
    }
    const int rc = finish_update(c);
    return err ? err : rc;
}

/* Section 4: the update list holds arcs into v (E_i) and out of v (E_o). */
static int vertex_update(ic_t *c, int32_t v) {
    const int32_t n = c->n;
    int32_t nout = 0;
    for (int32_t k = 0; k < c->nupd; ++k) nout += c->ua[k] == v;
    int err = IC_OK;
    memcpy(c->rvD, c->D + (size_t)v * n, sizeof(int32_t) * (size_t)n);
    memcpy(c->rvS, c->S + (size_t)v * n, sizeof(uint64_t) * (size_t)n);
    const int32_t *rvD = c->rvD;
    const uint64_t *rvS = c->rvS;
    /* Alg 4 over E_i per source, and whether the source can change */
#pragma omp parallel for num_threads(c->threads) schedule(static)
    for (int32_t s = 0; s < n; ++s) {
        const int32_t *Ds = c->D + (size_t)s * n;
        const uint64_t *Ss = c->S + (size_t)s * n;
        const int32_t dsv = Ds[v];
        int64_t cur = dsv;
        uint64_t sig = Ss[v], hat = 0;
        int bad = 0;
        for (int32_t k = 0; k < c->nupd; ++k) {
            if (c->ub[k] != v) continue;
            const int32_t du = Ds[c->ua[k]];
            if (du == INF32) continue;
            const int64_t cc = (int64_t)du + c->uw[k];
            if (cc >= INF32) {
                bad = IC_DIST_OVERFLOW;
                continue;
            }
            const uint64_t su = Ss[c->ua[k]];
            if (cc == cur) {
                if (__builtin_add_overflow(sig, su, &sig) || __builtin_add_overflow(hat, su, &hat))
                    bad = IC_SIGMA_OVERFLOW;
            } else if (cc < cur) {
                cur = cc;
                sig = su;
                hat = 0;
            }
        }
        scal_t sc;
        sc.dv = (int32_t)cur;
        sc.same = cur == (int64_t)dsv;
        sc.sv = sig;
        sc.hv = hat;
        sc.aff = cur < (int64_t)dsv || hat != 0;
        if (!sc.aff && cur != INF32 && nout)
            for (int32_t k = 0; k < c->nupd && !sc.aff; ++k) {
                if (c->ua[k] != v) continue;
                const int32_t xh = c->ub[k];
                int64_t d1 = Ds[xh];
                if (rvD[xh] != INF32 && cur + rvD[xh] < d1) d1 = cur + rvD[xh];
                const int64_t cc = cur + c->uw[k];
                if (cc < INF32 && cc <= d1) sc.aff = 1;
            }
        c->scal[s] = sc;
        if (bad) {
#pragma omp critical
            err = bad;
        }
    }
    /* row v'': Alg 4 on G'_R over E_o, the rows x_j after the In phase */
    if (nout) {
#pragma omp parallel for num_threads(c->threads) schedule(static)
        for (int32_t t = 0; t < n; ++t) {
            const int32_t dvt = rvD[t];
            int64_t best = dvt;
            uint64_t sig = rvS[t], hat = 0;
            int bad = 0;
            for (int32_t k = 0; k < c->nupd; ++k) {
                if (c->ua[k] != v) continue;
                const int32_t xh = c->ub[k];
                const scal_t sx = c->scal[xh];
                int64_t d1 = c->D[(size_t)xh * n + t];
                uint64_t s1 = c->S[(size_t)xh * n + t];
                if (sx.dv != INF32 && dvt != INF32) {
                    const int64_t cc = (int64_t)sx.dv + dvt;
                    if (cc <= d1) {
                        uint64_t add;
                        if (cc >= INF32) {
                            bad = IC_DIST_OVERFLOW;
                        } else if (__builtin_mul_overflow(cc < d1 || !sx.same ? sx.sv : sx.hv, rvS[t], &add)) {
                            bad = IC_SIGMA_OVERFLOW;
                        } else if (cc < d1) {
                            d1 = cc;
                            s1 = add;
                        } else if (__builtin_add_overflow(s1, add, &s1)) {
                            bad = IC_SIGMA_OVERFLOW;
                        }
                    }
                }
                if (d1 == INF32) continue;
                const int64_t c2 = c->uw[k] + d1;
                if (c2 >= INF32) {
                    bad = IC_DIST_OVERFLOW;
                    continue;
                }
                if (c2 < best) {
                    best = c2;
                    sig = s1;
                    hat = 0;
                } else if (c2 == best) {
                    if (__builtin_add_overflow(sig, s1, &sig) || __builtin_add_overflow(hat, s1, &hat))
                        bad = IC_SIGMA_OVERFLOW;
                }
            }
            c->rvvD[t] = (int32_t)best;
            c->rvvS[t] = sig;
            c->rvvH[t] = hat;
            if (bad) {
#pragma omp critical
                err = bad;
            }
        }
    }
    const int32_t *rvvD = c->rvvD;
    const uint64_t *rvvS = c->rvvS, *rvvH = c->rvvH;
    /* Lemma 4 per pair of every source that can change */
#pragma omp parallel num_threads(c->threads)
    {
        scratch_t *x = &c->sc[omp_get_thread_num()];
        int my_err = IC_OK;
#pragma omp for schedule(dynamic, 16)
        for (int32_t s = 0; s < n; ++s) {
            const scal_t sc = c->scal[s];
            if (!sc.aff) continue;
            const int32_t *Ds = c->D + (size_t)s * n;
            const uint64_t *Ss = c->S + (size_t)s * n;
            int32_t nb = 0;
            for (int32_t t = 0; t < n; ++t) {
                const int32_t d0 = Ds[t];
                int64_t d = d0;
                uint64_t sg = 0;
                int known = 0;
                if (sc.dv != INF32 && rvD[t] != INF32) {
                    const int64_t cc = (int64_t)sc.dv + rvD[t];
                    if (cc <= d0) {
                        uint64_t add;
                        if (cc >= INF32) {
                            my_err = IC_DIST_OVERFLOW;
                        } else if (__builtin_mul_overflow(cc < d0 || !sc.same ? sc.sv : sc.hv, rvS[t], &add)) {
                            my_err = IC_SIGMA_OVERFLOW;
                        } else if (cc < d0) {
                            d = cc;
                            sg = add;
                            known = 1;
                        } else if (add != 0) {
                            if (__builtin_add_overflow(Ss[t], add, &sg)) my_err = IC_SIGMA_OVERFLOW;
                            known = 1;
                        }
                    }
                }
                if (nout && sc.dv != INF32 && rvvD[t] != INF32) {
                    const int64_t cc = (int64_t)sc.dv + rvvD[t];
                    if (cc <= d) {
                        uint64_t add;
                        const uint64_t mult = (cc < d || rvvD[t] != rvD[t]) ? rvvS[t] : rvvH[t];
                        if (cc >= INF32) {
                            my_err = IC_DIST_OVERFLOW;
                        } else if (__builtin_mul_overflow(sc.sv, mult, &add)) {
                            my_err = IC_SIGMA_OVERFLOW;
                        } else if (cc < d) {
                            d = cc;
                            sg = add;
                            known = 1;
                        } else if (add != 0) {
                            if (__builtin_add_overflow(known ? sg : Ss[t], add, &sg)) my_err = IC_SIGMA_OVERFLOW;
                            known = 1;
                        }
                    }
                }
                if (!known) continue;
                x->t[nb] = t;
                x->d[nb] = (int32_t)d;
                x->sg[nb] = sg;
                ++nb;
            }
            if (nb) apply_source(c, x, s, nb);
        }
        if (my_err) {
#pragma omp critical
            err = my_err;
        }
    }
    const int rc = finish_update(c);
    return err ? err : rc;
}

static int check_arc(const ic_t *c, int32_t a, int32_t b, int64_t w) {
    if (a < 0 || a >= c->n || b < 0 || b >= c->n || a == b || w < 1 || w >= INF32) return IC_BAD_ARG;
    const int64_t cur = arc_weight(c, a, b);
    if (cur >= 0 && w >= cur) return IC_NOT_DECREASE;
    return IC_OK;
}

/* Decrease or insert edge (u, v) to weight w: Lemma 2 for an arc, the
 * vertex form at u for an undirected edge. */
int icpu_update_edge(void *h, int32_t u, int32_t v, int64_t w) {
    ic_t *c = (ic_t *)h;
    if (!c) return IC_BAD_ARG;
    int rc = check_arc(c, u, v, w);
    if (rc) return rc;
    if (c->directed) {
        if ((rc = push_update_arc(c, u, v, w))) return rc;
        return arc_update(c);
    }
    if ((rc = push_update_arc(c, v, u, w)) || (rc = push_update_arc(c, u, v, w))) {
        c->nupd = 0;
        return rc;
    }
    return vertex_update(c, u);
}

/* Vertex update at v: k edges (a[i], b[i]) each incident to v, each a
 * decrease or an insertion, no edge twice. */
int icpu_update_vertex(void *h, int32_t v, int32_t k, const int32_t *a, const int32_t *b, const int64_t *w) {
    ic_t *c = (ic_t *)h;
    if (!c || k < 0 || (k > 0 && (!a || !b || !w)) || v < 0 || v >= c->n) return IC_BAD_ARG;
    for (int32_t i = 0; i < k; ++i) {
        if (a[i] != v && b[i] != v) return IC_BAD_ARG;
        const int rc = check_arc(c, a[i], b[i], w[i]);
        if (rc) return rc;
        for (int32_t j = 0; j < i; ++j) {
            const int same = (a[j] == a[i] && b[j] == b[i]) || (!c->directed && a[j] == b[i] && b[j] == a[i]);
            if (same) return IC_BAD_ARG;
        }
    }
    if (k == 0) return IC_OK;
    for (int32_t i = 0; i < k; ++i) {
        int rc = push_update_arc(c, a[i], b[i], w[i]);
        if (!rc && !c->directed) rc = push_update_arc(c, b[i], a[i], w[i]);
        if (rc) {
            for (int32_t j = 0; j < c->nupd; ++j) c->uhead[c->ub[j]] = 0;
            c->nupd = 0;
            return rc;
        }
    }
    return vertex_update(c, v);
}
