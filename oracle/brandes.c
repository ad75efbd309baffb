/*
 * CPU oracle for incremental betweenness centrality: a plain, from-scratch
 * Brandes computation.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may call, link or
 * load this file or the library built from it; only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg use it.  It shares no
 * code, header or table with the GPU library.
 *
 * Why a from-scratch recompute is the right reference: the incremental
 * update of the paper (Lemma 2, Lemma 3, Lemma 4, Lemma 5, Theorem 1) is
 * exact, so after every update the maintained distances, path counts, DAGs
 * and BC scores must equal the ones a static computation finds on the
 * updated graph.
 *
 * What is computed, in the paper's notation (Section 2):
 *   d(s,t)    shortest-path distance, int64, INT64_MAX when t is unreachable;
 *   sigma_st  number of shortest s-t paths, uint64, sigma_ss = 1, 0 when
 *             unreachable; every addition is overflow-checked;
 *   P_s(t)    predecessor set of Eq.1: arcs (a,t) with d(s,t) = d(s,a) + w(a,t);
 *   delta_s.  source dependency, accumulated by Alg 1 (Eq.4) over the vertices
 *             in non-increasing distance order (Brandes' stack, Alg 7);
 *   BC(v)     Eq.3 over ordered pairs s != v != t, as the sum of delta_s.(v).
 *
 * Undirected graphs are taken as their directed double G_D (Section 3,
 * "Undirected graphs"): every edge {a,b} becomes arcs (a,b) and (b,a), so BC
 * counts ordered pairs and is not halved.
 *
 * Dijkstra uses a binary heap with lazy deletion; sources are spread over
 * POSIX threads.  BC partial sums are kept per fixed block of sources and
 * added in block order, so the result does not depend on the thread count.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_BAD_INPUT -1
#define OR_SELF_LOOP -2
#define OR_BAD_WEIGHT -3
#define OR_DUPLICATE -4
#define OR_SIGMA_OVERFLOW -5
#define OR_NOMEM -6

#define INF64 INT64_MAX
#define N_BLOCKS 64

typedef struct {
    int32_t n;
    int64_t m;          /* number of arcs of G (G_D when undirected) */
    int64_t *out_ptr;   /* CSR by tail */
    int32_t *out_dst;
    int64_t *out_w;
    int64_t *in_ptr;    /* CSR by head, for predecessor sets */
    int32_t *in_src;
    int64_t *in_w;
    int64_t *in_eid;    /* arc id: directed i, undirected 2i (a->b) / 2i+1 (b->a) */
} graph_t;

static void graph_free(graph_t *g) {
    free(g->out_ptr); free(g->out_dst); free(g->out_w);
    free(g->in_ptr); free(g->in_src); free(g->in_w); free(g->in_eid);
}

static int cmp_i64(const void *a, const void *b) {
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

/* Build both CSR views; validates the input the way the problem statement
 * requires (positive weights, no self-loops, E is a set). */
static int graph_build(graph_t *g, int32_t n, int64_t m_in, const int32_t *src, const int32_t *dst,
                       const int64_t *w, int directed) {
    memset(g, 0, sizeof(*g));
    if (n <= 0 || m_in < 0) return OR_BAD_INPUT;
    int64_t m = directed ? m_in : 2 * m_in;
    g->n = n;
    g->m = m;
    int64_t *keys = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
    g->out_ptr = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    g->in_ptr = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    g->out_dst = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    g->out_w = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
    g->in_src = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    g->in_w = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
    g->in_eid = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
    if (!keys || !g->out_ptr || !g->in_ptr || !g->out_dst || !g->out_w || !g->in_src || !g->in_w || !g->in_eid) {
        free(keys);
        graph_free(g);
        return OR_NOMEM;
    }
    for (int64_t i = 0; i < m_in; i++) {
        int32_t a = src[i], b = dst[i];
        if (a < 0 || a >= n || b < 0 || b >= n) { free(keys); graph_free(g); return OR_BAD_INPUT; }
        if (a == b) { free(keys); graph_free(g); return OR_SELF_LOOP; }
        if (w[i] <= 0) { free(keys); graph_free(g); return OR_BAD_WEIGHT; }
    }
    int64_t k = 0;
    for (int64_t i = 0; i < m_in; i++) {
        keys[k++] = (int64_t)src[i] * n + dst[i];
        if (!directed) keys[k++] = (int64_t)dst[i] * n + src[i];
    }
    qsort(keys, (size_t)m, sizeof(int64_t), cmp_i64);
    for (int64_t i = 1; i < m; i++)
        if (keys[i] == keys[i - 1]) { free(keys); graph_free(g); return OR_DUPLICATE; }
    free(keys);
    for (int64_t i = 0; i < m_in; i++) {
        g->out_ptr[src[i] + 1]++;
        g->in_ptr[dst[i] + 1]++;
        if (!directed) { g->out_ptr[dst[i] + 1]++; g->in_ptr[src[i] + 1]++; }
    }
    for (int32_t v = 0; v < n; v++) {
        g->out_ptr[v + 1] += g->out_ptr[v];
        g->in_ptr[v + 1] += g->in_ptr[v];
    }
    int64_t *fo = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *fi = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    if (!fo || !fi) { free(fo); free(fi); graph_free(g); return OR_NOMEM; }
    memcpy(fo, g->out_ptr, sizeof(int64_t) * (size_t)n);
    memcpy(fi, g->in_ptr, sizeof(int64_t) * (size_t)n);
    for (int64_t i = 0; i < m_in; i++) {
        int32_t a = src[i], b = dst[i];
        int64_t o = fo[a]++, q = fi[b]++;
        g->out_dst[o] = b; g->out_w[o] = w[i];
        g->in_src[q] = a; g->in_w[q] = w[i];
        g->in_eid[q] = directed ? i : 2 * i;
        if (!directed) {
            o = fo[b]++; q = fi[a]++;
            g->out_dst[o] = a; g->out_w[o] = w[i];
            g->in_src[q] = b; g->in_w[q] = w[i];
            g->in_eid[q] = 2 * i + 1;
        }
    }
    free(fo);
    free(fi);
    return OR_OK;
}

/* ---------------------------------------------------------------- heap --- */

typedef struct { int64_t d; int32_t v; } hitem;

typedef struct { hitem *a; int64_t len, cap; } heap_t;

static int heap_push(heap_t *h, int64_t d, int32_t v) {
    if (h->len == h->cap) {
        int64_t nc = h->cap ? 2 * h->cap : 1024;
        hitem *na = (hitem *)realloc(h->a, sizeof(hitem) * (size_t)nc);
        if (!na) return OR_NOMEM;
        h->a = na;
        h->cap = nc;
    }
    int64_t i = h->len++;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (h->a[p].d < d || (h->a[p].d == d && h->a[p].v <= v)) break;
        h->a[i] = h->a[p];
        i = p;
    }
    h->a[i].d = d;
    h->a[i].v = v;
    return OR_OK;
}

static hitem heap_pop(heap_t *h) {
    hitem top = h->a[0];
    hitem last = h->a[--h->len];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, c = i;
        hitem best = last;
        if (l < h->len && (h->a[l].d < best.d || (h->a[l].d == best.d && h->a[l].v < best.v))) { c = l; best = h->a[l]; }
        if (r < h->len && (h->a[r].d < best.d || (h->a[r].d == best.d && h->a[r].v < best.v))) { c = r; best = h->a[r]; }
        if (c == i) break;
        h->a[i] = h->a[c];
        i = c;
    }
    if (h->len > 0) h->a[i] = last;
    return top;
}

/* ------------------------------------------------------- single source --- */

typedef struct {
    int64_t *dist;
    uint64_t *sigma;
    double *delta;
    int32_t *order;   /* Dijkstra settle order = non-decreasing distance */
    uint8_t *done;
    heap_t heap;
    int32_t settled;
} work_t;

static int work_init(work_t *wk, int32_t n) {
    memset(wk, 0, sizeof(*wk));
    wk->dist = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    wk->sigma = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
    wk->delta = (double *)malloc(sizeof(double) * (size_t)n);
    wk->order = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    wk->done = (uint8_t *)malloc((size_t)n);
    return (wk->dist && wk->sigma && wk->delta && wk->order && wk->done) ? OR_OK : OR_NOMEM;
}

static void work_free(work_t *wk) {
    free(wk->dist); free(wk->sigma); free(wk->delta); free(wk->order); free(wk->done); free(wk->heap.a);
}

/* Dijkstra from s computing d(s,.) and sigma_s. (Alg 7, line "run Dijkstra's
 * SSSP from s and compute sigma_st and P_s(t)").  When a relaxation
 * d(s,a) + w(a,b) beats d(s,b), b's count restarts from sigma_sa; on a tie it
 * grows by sigma_sa.  Positive weights make sigma_sa final when a settles. */
static int sssp(const graph_t *g, int32_t s, work_t *wk) {
    int32_t n = g->n;
    for (int32_t v = 0; v < n; v++) { wk->dist[v] = INF64; wk->sigma[v] = 0; wk->done[v] = 0; }
    wk->dist[s] = 0;
    wk->sigma[s] = 1;
    wk->heap.len = 0;
    wk->settled = 0;
    if (heap_push(&wk->heap, 0, s)) return OR_NOMEM;
    while (wk->heap.len > 0) {
        hitem it = heap_pop(&wk->heap);
        int32_t a = it.v;
        if (wk->done[a] || it.d != wk->dist[a]) continue;
        wk->done[a] = 1;
        wk->order[wk->settled++] = a;
        for (int64_t e = g->out_ptr[a]; e < g->out_ptr[a + 1]; e++) {
            int32_t b = g->out_dst[e];
            int64_t nd = wk->dist[a] + g->out_w[e];
            if (nd < wk->dist[b]) {
                wk->dist[b] = nd;
                wk->sigma[b] = wk->sigma[a];
                if (heap_push(&wk->heap, nd, b)) return OR_NOMEM;
            } else if (nd == wk->dist[b]) {
                if (__builtin_add_overflow(wk->sigma[b], wk->sigma[a], &wk->sigma[b])) return OR_SIGMA_OVERFLOW;
            }
        }
    }
    return OR_OK;
}

/* Alg 1 (Accumulate-dependency) with Brandes' stack: pop vertices in
 * non-increasing distance; each w hands sigma_sv/sigma_sw * (1 + delta(w)) to
 * every v in P_s(w) (Eq.4).  P_s(w) is read straight from Eq.1 over the
 * in-arcs of w.  If bc is non-null, delta(w) is added to bc[w] for w != s. */
static void accumulate(const graph_t *g, int32_t s, work_t *wk, double *bc) {
    int32_t n = g->n;
    for (int32_t v = 0; v < n; v++) wk->delta[v] = 0.0;
    for (int32_t i = wk->settled - 1; i >= 0; i--) {
        int32_t x = wk->order[i];
        for (int64_t e = g->in_ptr[x]; e < g->in_ptr[x + 1]; e++) {
            int32_t a = g->in_src[e];
            if (wk->dist[a] != INF64 && wk->dist[a] + g->in_w[e] == wk->dist[x])
                wk->delta[a] += (double)wk->sigma[a] / (double)wk->sigma[x] * (1.0 + wk->delta[x]);
        }
        if (x != s && bc) bc[x] += wk->delta[x];
    }
    /* Eq.3 never pairs s with itself; the dependency row reports 0 there. */
    wk->delta[s] = 0.0;
}

/* --------------------------------------------------------- all sources --- */

/* E* (Section 1): the arcs lying on some shortest path, i.e. the union of the
 * DAG(s) over all sources.  Each source marks the arcs of its own DAG(s). */
static void mark_dag_arcs(const graph_t *g, const work_t *wk, uint8_t *estar) {
    for (int32_t i = 0; i < wk->settled; i++) {
        int32_t b = wk->order[i];
        for (int64_t e = g->in_ptr[b]; e < g->in_ptr[b + 1]; e++) {
            int32_t a = g->in_src[e];
            if (wk->dist[a] != INF64 && wk->dist[a] + g->in_w[e] == wk->dist[b])
                __atomic_store_n(&estar[g->in_eid[e]], (uint8_t)1, __ATOMIC_RELAXED);
        }
    }
}

typedef struct {
    const graph_t *g;
    int64_t *D;
    uint64_t *S;
    double *partials; /* N_BLOCKS x n */
    uint8_t *estar;   /* per arc id: 1 when the arc lies on some DAG(s) */
    int next_block;
    int status;
    pthread_mutex_t mu;
} job_t;

static void *worker(void *arg) {
    job_t *job = (job_t *)arg;
    const graph_t *g = job->g;
    int32_t n = g->n;
    work_t wk;
    if (work_init(&wk, n)) {
        pthread_mutex_lock(&job->mu);
        job->status = OR_NOMEM;
        pthread_mutex_unlock(&job->mu);
        work_free(&wk);
        return NULL;
    }
    for (;;) {
        pthread_mutex_lock(&job->mu);
        int b = job->next_block++;
        int stop = job->status != OR_OK;
        pthread_mutex_unlock(&job->mu);
        if (b >= N_BLOCKS || stop) break;
        int64_t s0 = (int64_t)n * b / N_BLOCKS, s1 = (int64_t)n * (b + 1) / N_BLOCKS;
        double *bc = job->partials + (size_t)b * n;
        for (int64_t s = s0; s < s1; s++) {
            int rc = sssp(g, (int32_t)s, &wk);
            if (rc) {
                pthread_mutex_lock(&job->mu);
                if (job->status == OR_OK) job->status = rc;
                pthread_mutex_unlock(&job->mu);
                break;
            }
            accumulate(g, (int32_t)s, &wk, bc);
            if (job->estar) mark_dag_arcs(g, &wk, job->estar);
            if (job->D) memcpy(job->D + (size_t)s * n, wk.dist, sizeof(int64_t) * (size_t)n);
            if (job->S) memcpy(job->S + (size_t)s * n, wk.sigma, sizeof(uint64_t) * (size_t)n);
        }
    }
    work_free(&wk);
    return NULL;
}

/* All-pairs d, sigma and BC of the graph (Alg 7).  D and S may be NULL (n*n
 * row-major otherwise); bc receives n values; estar (may be NULL) receives one
 * byte per arc id (m, or 2m when undirected: 2i for a->b, 2i+1 for b->a) set
 * to 1 when the arc lies on some shortest path.  Returns 0 or a negative code. */
int oracle_brandes(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, const int64_t *w, int32_t directed,
                   int64_t *D, uint64_t *S, double *bc, uint8_t *estar, int32_t nthreads) {
    graph_t g;
    int rc = graph_build(&g, n, m, src, dst, w, directed);
    if (rc) return rc;
    job_t job;
    memset(&job, 0, sizeof(job));
    job.g = &g;
    job.D = D;
    job.S = S;
    job.estar = estar;
    if (estar) memset(estar, 0, (size_t)(directed ? m : 2 * m));
    job.partials = (double *)calloc((size_t)N_BLOCKS * (size_t)n, sizeof(double));
    if (!job.partials) { graph_free(&g); return OR_NOMEM; }
    pthread_mutex_init(&job.mu, NULL);
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    int started = 0;
    for (int i = 0; i < nthreads; i++)
        if (pthread_create(&th[i], NULL, worker, &job) == 0) started++;
        else break;
    if (started == 0) worker(&job);
    for (int i = 0; i < started; i++) pthread_join(th[i], NULL);
    pthread_mutex_destroy(&job.mu);
    for (int32_t v = 0; v < n; v++) {
        double acc = 0.0;
        for (int b = 0; b < N_BLOCKS; b++) acc += job.partials[(size_t)b * n + v];
        bc[v] = acc;
    }
    free(job.partials);
    graph_free(&g);
    return job.status;
}

/* One source s: rows d(s,.), sigma_s., delta_s.(.) and the arcs of DAG(s)
 * (Eq.1), listed grouped by head.  dag_a/dag_b may be NULL; *dag_cnt gets the
 * number of DAG arcs (capacity is the arc count of G_D). */
int oracle_source(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, const int64_t *w, int32_t directed,
                  int32_t s, int64_t *drow, uint64_t *srow, double *delta, int32_t *dag_a, int32_t *dag_b,
                  int64_t *dag_cnt) {
    graph_t g;
    int rc = graph_build(&g, n, m, src, dst, w, directed);
    if (rc) return rc;
    if (s < 0 || s >= n) { graph_free(&g); return OR_BAD_INPUT; }
    work_t wk;
    if (work_init(&wk, n)) { work_free(&wk); graph_free(&g); return OR_NOMEM; }
    rc = sssp(&g, s, &wk);
    if (rc == OR_OK) {
        accumulate(&g, s, &wk, NULL);
        if (drow) memcpy(drow, wk.dist, sizeof(int64_t) * (size_t)n);
        if (srow) memcpy(srow, wk.sigma, sizeof(uint64_t) * (size_t)n);
        if (delta) memcpy(delta, wk.delta, sizeof(double) * (size_t)n);
        int64_t cnt = 0;
        for (int32_t b = 0; b < n; b++) {
            if (wk.dist[b] == INF64) continue;
            for (int64_t e = g.in_ptr[b]; e < g.in_ptr[b + 1]; e++) {
                int32_t a = g.in_src[e];
                if (wk.dist[a] != INF64 && wk.dist[a] + g.in_w[e] == wk.dist[b]) {
                    if (dag_a) dag_a[cnt] = a;
                    if (dag_b) dag_b[cnt] = b;
                    cnt++;
                }
            }
        }
        if (dag_cnt) *dag_cnt = cnt;
    }
    work_free(&wk);
    graph_free(&g);
    return rc;
}

/* Several sources at once (sampled checks on large graphs): rows for each
 * s in srcs[0..k), written to drows/srows/deltas (k x n, any may be NULL). */
typedef struct {
    const graph_t *g;
    const int32_t *srcs;
    int32_t k;
    int64_t *drows;
    uint64_t *srows;
    double *deltas;
    int next;
    int status;
    pthread_mutex_t mu;
} rows_job_t;

static void *rows_worker(void *arg) {
    rows_job_t *job = (rows_job_t *)arg;
    int32_t n = job->g->n;
    work_t wk;
    if (work_init(&wk, n)) { work_free(&wk); job->status = OR_NOMEM; return NULL; }
    for (;;) {
        pthread_mutex_lock(&job->mu);
        int i = job->next++;
        pthread_mutex_unlock(&job->mu);
        if (i >= job->k) break;
        int32_t s = job->srcs[i];
        int rc = (s < 0 || s >= n) ? OR_BAD_INPUT : sssp(job->g, s, &wk);
        if (rc) {
            pthread_mutex_lock(&job->mu);
            job->status = rc;
            pthread_mutex_unlock(&job->mu);
            continue;
        }
        accumulate(job->g, s, &wk, NULL);
        if (job->drows) memcpy(job->drows + (size_t)i * n, wk.dist, sizeof(int64_t) * (size_t)n);
        if (job->srows) memcpy(job->srows + (size_t)i * n, wk.sigma, sizeof(uint64_t) * (size_t)n);
        if (job->deltas) memcpy(job->deltas + (size_t)i * n, wk.delta, sizeof(double) * (size_t)n);
    }
    work_free(&wk);
    return NULL;
}

int oracle_rows(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, const int64_t *w, int32_t directed,
                int32_t k, const int32_t *srcs, int64_t *drows, uint64_t *srows, double *deltas, int32_t nthreads) {
    graph_t g;
    int rc = graph_build(&g, n, m, src, dst, w, directed);
    if (rc) return rc;
    rows_job_t job;
    memset(&job, 0, sizeof(job));
    job.g = &g;
    job.srcs = srcs;
    job.k = k;
    job.drows = drows;
    job.srows = srows;
    job.deltas = deltas;
    pthread_mutex_init(&job.mu, NULL);
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    int started = 0;
    for (int i = 0; i < nthreads; i++)
        if (pthread_create(&th[i], NULL, rows_worker, &job) == 0) started++;
        else break;
    if (started == 0) rows_worker(&job);
    for (int i = 0; i < started; i++) pthread_join(th[i], NULL);
    pthread_mutex_destroy(&job.mu);
    graph_free(&g);
    return job.status;
}
