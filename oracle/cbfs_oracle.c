/*
 * Cluster-BFS oracle: plain, slow, obviously correct CPU reference.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link,
 * load or call this file; only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header or table with the
 * HIP library.
 *
 * What it computes (paper, Section 3.1, the subset equation, re-based on the
 * cluster center as in the star-center storage of Section 5.3): for a graph G
 * given as CSR and a cluster with ordered sources s_0 (the center), s_1, ...,
 * s_{k-1}, and an offset radius R,
 *
 *     dist[v]            = delta(s_0, v)                (UINT32_MAX if unreachable)
 *     bit i of mask[o][v] = 1  iff  delta(s_i, v) = delta(s_0, v) + o,  o in [-R, R]
 *
 * where delta is the hop distance.  It is that definition written out: one
 * plain FIFO breadth-first search per source (the sequential form of the
 * paper's single-source BFS, Appendix A), then a direct encode of the
 * distances.  A source farther than R from the center in offset at some
 * reachable vertex (or reaching a vertex the center does not reach) makes the
 * cluster's status CBFS_E_RADIUS; the Fact and Corollary of Section 3.1 bound
 * every offset by the source's distance to the center.  Such a cluster's
 * outputs are then defined as dist = UINT32_MAX and every mask word 0 (the
 * problem statement takes the cluster's diameter as given; a cluster that
 * breaks it gets no partial answer).
 *
 * Layouts (all row-major):
 *   row_ptr[n+1], col[m]            int32 CSR, rows = out-neighbours
 *   cluster_ptr[C+1], sources[...]  sources of cluster c are
 *                                   sources[cluster_ptr[c] .. cluster_ptr[c+1])
 *   dist[C][n]                      uint32
 *   masks[C][2R+1][n][W]            uint64; source i -> bit (i % 64) of word i/64
 *   status[C]                       0 or -5 (radius violated)
 *
 * Also here: graph cleanup into the CSR the searches run on (drop self-loops,
 * add reverse arcs, drop duplicate arcs, keep the largest connected component,
 * relabel in ascending original-id order), the brute-force landmark-labeling query (Algorithm "Framework of
 * Landmark Labeling", Query: min over landmarks of the two distances), the
 * same query evaluated from this oracle's own encoded labels by the lowest
 * non-empty intersection (Section 4.2, answering queries with clustered
 * landmarks), and a BFS-certificate checker for any encoded output.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#define OR_OK 0
#define OR_E_ARG (-1)
#define OR_E_RADIUS (-5)
#define OR_E_NOMEM (-8)
#define OR_E_CAPACITY (-9)
#define UNREACHED (-1)

#define MAX_THREADS 256

/* Threads to use: the request, else OMP_NUM_THREADS, else the online CPUs. */
static int nthreads_or_default(int32_t nthreads)
{
    if (nthreads <= 0) {
        const char *env = getenv("OMP_NUM_THREADS");
        nthreads = env ? atoi(env) : 0;
        if (nthreads <= 0) nthreads = (int32_t)sysconf(_SC_NPROCESSORS_ONLN);
    }
    if (nthreads < 1) nthreads = 1;
    if (nthreads > MAX_THREADS) nthreads = MAX_THREADS;
    return nthreads;
}

/* A plain pthread parallel-for: fn(lo, hi, tid, ctx) over chunks of `grain`
 * indices of [0, n), handed out in order to nt threads (tid in [0, nt)). */
typedef void (*range_fn)(int64_t lo, int64_t hi, int tid, void *ctx);
typedef struct {
    int64_t n, grain, next;
    pthread_mutex_t mu;
    range_fn fn;
    void *ctx;
} pfor_job;
typedef struct {
    pfor_job *job;
    int tid;
} pfor_arg;

static void *pfor_worker(void *p)
{
    pfor_arg *a = (pfor_arg *)p;
    pfor_job *j = a->job;
    for (;;) {
        pthread_mutex_lock(&j->mu);
        const int64_t lo = j->next;
        const int64_t hi = lo + j->grain < j->n ? lo + j->grain : j->n;
        j->next = hi;
        pthread_mutex_unlock(&j->mu);
        if (lo >= j->n) break;
        j->fn(lo, hi, a->tid, j->ctx);
    }
    return NULL;
}

static void parallel_for(int64_t n, int64_t grain, int nt, range_fn fn, void *ctx)
{
    if (grain < 1) grain = 1;
    if (nt <= 1 || n <= grain) {
        if (n > 0) fn(0, n, 0, ctx);
        return;
    }
    pfor_job job;
    job.n = n;
    job.grain = grain;
    job.next = 0;
    job.fn = fn;
    job.ctx = ctx;
    pthread_mutex_init(&job.mu, NULL);
    pthread_t th[MAX_THREADS];
    pfor_arg args[MAX_THREADS];
    int started = 1;
    for (int t = 0; t < nt; t++) {
        args[t].job = &job;
        args[t].tid = t;
    }
    for (int t = 1; t < nt; t++) {
        if (pthread_create(&th[t], NULL, pfor_worker, &args[t]) != 0) break;
        started++;
    }
    pfor_worker(&args[0]);
    for (int t = 1; t < started; t++) pthread_join(th[t], NULL);
    pthread_mutex_destroy(&job.mu);
}

/* Plain FIFO BFS from src.  dist[v] = hops from src, -1 when unreachable.
 * queue must hold n entries. */
static void bfs(int64_t n, const int32_t *row_ptr, const int32_t *col, int32_t src,
                int32_t *dist, int32_t *queue)
{
    for (int64_t v = 0; v < n; v++) dist[v] = UNREACHED;
    int64_t head = 0, tail = 0;
    dist[src] = 0;
    queue[tail++] = src;
    while (head < tail) {
        int32_t u = queue[head++];
        for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; e++) {
            int32_t v = col[e];
            if (dist[v] == UNREACHED) {
                dist[v] = dist[u] + 1;
                queue[tail++] = v;
            }
        }
    }
}

int oracle_bfs(int64_t n, const int32_t *row_ptr, const int32_t *col, int32_t src, int32_t *dist)
{
    if (n <= 0 || src < 0 || src >= n) return OR_E_ARG;
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!queue) return OR_E_NOMEM;
    bfs(n, row_ptr, col, src, dist, queue);
    free(queue);
    return OR_OK;
}

/* Distances from a batch of sources, one BFS per source, in parallel over sources.
 * d[j*n + v] = delta(src[j], v). */
typedef struct {
    int64_t n;
    const int32_t *row_ptr, *col, *src;
    int32_t *d, *queues;
} bfs_batch_ctx;

static void bfs_batch_body(int64_t lo, int64_t hi, int tid, void *p)
{
    bfs_batch_ctx *c = (bfs_batch_ctx *)p;
    for (int64_t j = lo; j < hi; j++)
        bfs(c->n, c->row_ptr, c->col, c->src[j], c->d + (size_t)j * (size_t)c->n,
            c->queues + (size_t)tid * (size_t)c->n);
}

static int bfs_batch(int64_t n, const int32_t *row_ptr, const int32_t *col,
                     const int32_t *src, int32_t count, int32_t *d, int nthreads)
{
    int nt = nthreads < count ? nthreads : count;
    if (nt < 1) nt = 1;
    int32_t *queues = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * (size_t)nt);
    if (!queues) return OR_E_NOMEM;
    bfs_batch_ctx c = {n, row_ptr, col, src, d, queues};
    parallel_for(count, 1, nt, bfs_batch_body, &c);
    free(queues);
    return OR_OK;
}

/* Encode sources i0 .. i0+cnt-1 at every vertex: bit i goes to the plane of
 * its offset delta_i(v) - delta_0(v); offsets beyond [-R, R], and sources
 * reaching a vertex the center does not (or the reverse), flag a violation. */
typedef struct {
    int64_t n;
    const int32_t *d0, *db;
    int32_t cnt, i0, R, W;
    uint64_t *mc;
    int violated;
} encode_ctx;

static void encode_body(int64_t lo, int64_t hi, int tid, void *p)
{
    (void)tid;
    encode_ctx *e = (encode_ctx *)p;
    const int64_t n = e->n;
    const int32_t R = e->R, W = e->W;
    int bad = 0;
    for (int64_t v = lo; v < hi; v++) {
        for (int32_t j = 0; j < e->cnt; j++) {
            const int32_t i = e->i0 + j;
            const int32_t di = e->db[(size_t)j * (size_t)n + (size_t)v];
            const int32_t dc = e->d0[v];
            if (dc == UNREACHED || di == UNREACHED) {
                if (dc != di) bad = 1;
                continue;
            }
            const int32_t off = di - dc;
            if (off < -R || off > R) {
                bad = 1;
                continue;
            }
            e->mc[((size_t)(off + R) * (size_t)n + (size_t)v) * (size_t)W + (size_t)(i / 64)] |=
                (uint64_t)1 << (i % 64);
        }
    }
    if (bad) __atomic_store_n(&e->violated, 1, __ATOMIC_RELAXED);
}

int oracle_cbfs(int64_t n, const int32_t *row_ptr, const int32_t *col,
                int32_t num_clusters, const int32_t *cluster_ptr, const int32_t *sources,
                int32_t R, int32_t W, uint32_t *dist, uint64_t *masks, int32_t *status,
                int32_t nthreads)
{
    if (n <= 0 || num_clusters < 0 || R < 0 || W < 1) return OR_E_ARG;
    int nt = nthreads_or_default(nthreads);
    const int64_t P = 2 * (int64_t)R + 1;
    const int32_t batch = nt;
    int32_t *d0 = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *db = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * (size_t)batch);
    if (!d0 || !db) {
        free(d0);
        free(db);
        return OR_E_NOMEM;
    }
    int rc = OR_OK;
    for (int32_t c = 0; c < num_clusters && rc == OR_OK; c++) {
        const int32_t *S = sources + cluster_ptr[c];
        const int32_t k = cluster_ptr[c + 1] - cluster_ptr[c];
        if (k < 1 || k > 64 * W) { rc = OR_E_ARG; break; }
        uint32_t *dc = dist + (size_t)c * (size_t)n;
        uint64_t *mc = masks + (size_t)c * (size_t)P * (size_t)n * (size_t)W;
        memset(mc, 0, sizeof(uint64_t) * (size_t)P * (size_t)n * (size_t)W);
        int violated = 0;

        /* distance from the center s_0 */
        rc = bfs_batch(n, row_ptr, col, S, 1, d0, 1);
        if (rc != OR_OK) break;
        for (int64_t v = 0; v < n; v++) dc[v] = d0[v] == UNREACHED ? UINT32_MAX : (uint32_t)d0[v];

        /* every source, a batch at a time, then encode its offsets */
        for (int32_t i0 = 0; i0 < k && rc == OR_OK; i0 += batch) {
            int32_t cnt = k - i0 < batch ? k - i0 : batch;
            rc = bfs_batch(n, row_ptr, col, S + i0, cnt, db, nt);
            if (rc != OR_OK) break;
            encode_ctx ec = {n, d0, db, cnt, i0, R, W, mc, 0};
            parallel_for(n, 4096, nt, encode_body, &ec);
            if (ec.violated) violated = 1;
        }
        status[c] = violated ? OR_E_RADIUS : OR_OK;
        if (violated) {
            /* the boundary's definition of a violating cluster's outputs:
             * unreachable everywhere, no source at any offset */
            for (int64_t v = 0; v < n; v++) dc[v] = UINT32_MAX;
            memset(mc, 0, sizeof(uint64_t) * (size_t)P * (size_t)n * (size_t)W);
        }
    }
    free(d0);
    free(db);
    return rc;
}

/* ------------------------------------------------------------------------
 * The cluster distance vector in the paper's own form (Section 3.1, the
 * subset equation): for a cluster S of diameter d and every vertex v,
 *     Delta_v  = min over s in S of delta(s, v)              (UINT32_MAX if unreachable)
 *     S_v[i]   = {s in S : delta(s, v) = Delta_v + i},  i = 0..d
 * (d+1 subsets; by the Fact of Section 3.1 every source lies within d of
 * Delta_v).  Written out from one plain BFS per source: first the minimum
 * over the sources, then each source's bit into subset delta_j(v) - Delta_v.
 * A source at more than d beyond Delta_v, or a source that does not reach a
 * vertex another source reaches, breaks the given diameter: the cluster's
 * status is -5 and its outputs are UINT32_MAX and all-zero subsets.
 * Layout: delta[C][n] uint32, subsets[C][d+1][n][W] uint64. */
typedef struct {
    int64_t n;
    const int32_t *db;   /* [cnt][n] distances of sources i0 .. i0+cnt-1 */
    int32_t cnt, i0, D, W;
    const uint32_t *dmin;
    uint64_t *mc;
    int violated;
} minenc_ctx;

static void minenc_body(int64_t lo, int64_t hi, int tid, void *p)
{
    (void)tid;
    minenc_ctx *e = (minenc_ctx *)p;
    const int64_t n = e->n;
    int bad = 0;
    for (int64_t v = lo; v < hi; v++) {
        const uint32_t m = e->dmin[v];
        for (int32_t j = 0; j < e->cnt; j++) {
            const int32_t dj = e->db[(size_t)j * (size_t)n + (size_t)v];
            const int32_t i = e->i0 + j;
            if (dj == UNREACHED) {
                if (m != UINT32_MAX) bad = 1; /* another source reaches v */
                continue;
            }
            const int64_t off = (int64_t)dj - (int64_t)m;
            if (off > e->D) {
                bad = 1;
                continue;
            }
            e->mc[((size_t)off * (size_t)n + (size_t)v) * (size_t)e->W + (size_t)(i / 64)] |=
                (uint64_t)1 << (i % 64);
        }
    }
    if (bad) __atomic_store_n(&e->violated, 1, __ATOMIC_RELAXED);
}

int oracle_cbfs_min(int64_t n, const int32_t *row_ptr, const int32_t *col,
                    int32_t num_clusters, const int32_t *cluster_ptr, const int32_t *sources,
                    int32_t D, int32_t W, uint32_t *delta, uint64_t *subsets, int32_t *status,
                    int32_t nthreads)
{
    if (n <= 0 || num_clusters < 0 || D < 0 || W < 1) return OR_E_ARG;
    int nt = nthreads_or_default(nthreads);
    const int64_t P = (int64_t)D + 1;
    int32_t *db = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * (size_t)nt);
    if (!db) return OR_E_NOMEM;
    int rc = OR_OK;
    for (int32_t c = 0; c < num_clusters && rc == OR_OK; c++) {
        const int32_t *S = sources + cluster_ptr[c];
        const int32_t k = cluster_ptr[c + 1] - cluster_ptr[c];
        if (k < 1 || k > 64 * W) { rc = OR_E_ARG; break; }
        uint32_t *dc = delta + (size_t)c * (size_t)n;
        uint64_t *mc = subsets + (size_t)c * (size_t)P * (size_t)n * (size_t)W;
        memset(mc, 0, sizeof(uint64_t) * (size_t)P * (size_t)n * (size_t)W);
        for (int64_t v = 0; v < n; v++) dc[v] = UINT32_MAX;
        /* pass 1: Delta_v, the minimum over the sources */
        for (int32_t i0 = 0; i0 < k && rc == OR_OK; i0 += nt) {
            int32_t cnt = k - i0 < nt ? k - i0 : nt;
            rc = bfs_batch(n, row_ptr, col, S + i0, cnt, db, nt);
            for (int32_t j = 0; j < cnt && rc == OR_OK; j++)
                for (int64_t v = 0; v < n; v++) {
                    const int32_t x = db[(size_t)j * (size_t)n + (size_t)v];
                    if (x != UNREACHED && (uint32_t)x < dc[v]) dc[v] = (uint32_t)x;
                }
        }
        /* pass 2: each source's bit into subset delta_j(v) - Delta_v */
        int violated = 0;
        for (int32_t i0 = 0; i0 < k && rc == OR_OK; i0 += nt) {
            int32_t cnt = k - i0 < nt ? k - i0 : nt;
            rc = bfs_batch(n, row_ptr, col, S + i0, cnt, db, nt);
            if (rc != OR_OK) break;
            minenc_ctx ec = {n, db, cnt, i0, D, W, dc, mc, 0};
            parallel_for(n, 4096, nt, minenc_body, &ec);
            if (ec.violated) violated = 1;
        }
        status[c] = violated ? OR_E_RADIUS : OR_OK;
        if (violated) {
            for (int64_t v = 0; v < n; v++) dc[v] = UINT32_MAX;
            memset(mc, 0, sizeof(uint64_t) * (size_t)P * (size_t)n * (size_t)W);
        }
    }
    free(db);
    return rc;
}

typedef struct {
    int64_t n;
    const int32_t *db;
    int32_t cnt;
    const int32_t *qs, *qt;
    uint32_t *ans;
} query_ctx;

static void query_body(int64_t lo, int64_t hi, int tid, void *p)
{
    (void)tid;
    query_ctx *c = (query_ctx *)p;
    for (int32_t j = 0; j < c->cnt; j++) {
        const int32_t *d = c->db + (size_t)j * (size_t)c->n;
        for (int64_t k = lo; k < hi; k++) {
            const int32_t a = d[c->qs[k]], b = d[c->qt[k]];
            if (a == UNREACHED || b == UNREACHED) continue;
            const uint32_t val = (uint32_t)(a + b);
            if (val < c->ans[k]) c->ans[k] = val;
        }
    }
}

/* Landmark-labeling query by brute force: for each pair (s, t),
 * ans = min over every cluster c and every source x of c of delta(x,s)+delta(x,t),
 * UINT32_MAX if no landmark reaches both. */
int oracle_query_landmarks(int64_t n, const int32_t *row_ptr, const int32_t *col,
                           int32_t num_clusters, const int32_t *cluster_ptr, const int32_t *sources,
                           int64_t q, const int32_t *qs, const int32_t *qt, uint32_t *ans,
                           int32_t nthreads)
{
    if (n <= 0 || q < 0 || num_clusters < 0) return OR_E_ARG;
    int nt = nthreads_or_default(nthreads);
    for (int64_t j = 0; j < q; j++) {
        if (qs[j] < 0 || qs[j] >= n || qt[j] < 0 || qt[j] >= n) return OR_E_ARG;
        ans[j] = UINT32_MAX;
    }
    const int32_t total = cluster_ptr[num_clusters];
    int32_t *db = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * (size_t)nt);
    if (!db) return OR_E_NOMEM;
    int rc = OR_OK;
    for (int32_t x0 = 0; x0 < total && rc == OR_OK; x0 += nt) {
        int32_t cnt = total - x0 < nt ? total - x0 : nt;
        rc = bfs_batch(n, row_ptr, col, sources + x0, cnt, db, nt);
        if (rc != OR_OK) break;
        query_ctx qc = {n, db, cnt, qs, qt, ans};
        parallel_for(q, 4096, nt, query_body, &qc);
    }
    free(db);
    return rc;
}

/* Exact hop distance of each pair: out[j] = delta(qs[j], qt[j]) from one
 * plain FIFO BFS rooted at qs[j] (UINT32_MAX when qt[j] is unreachable).
 * The ground truth a landmark answer is bounded by from below (Section 4.2:
 * a landmark x gives delta(x,s) + delta(x,t) >= delta(s,t), the triangle
 * inequality).  Parallel over pairs, one BFS buffer pair per thread. */
typedef struct {
    int64_t n;
    const int32_t *row_ptr, *col, *qs, *qt;
    uint32_t *out;
    int32_t *bufs;
} pair_ctx;

static void pair_body(int64_t lo, int64_t hi, int tid, void *p)
{
    pair_ctx *c = (pair_ctx *)p;
    int32_t *d = c->bufs + (size_t)tid * 2 * (size_t)c->n;
    int32_t *queue = d + c->n;
    for (int64_t j = lo; j < hi; j++) {
        bfs(c->n, c->row_ptr, c->col, c->qs[j], d, queue);
        const int32_t x = d[c->qt[j]];
        c->out[j] = x == UNREACHED ? UINT32_MAX : (uint32_t)x;
    }
}

int oracle_pair_distances(int64_t n, const int32_t *row_ptr, const int32_t *col, int64_t q,
                          const int32_t *qs, const int32_t *qt, uint32_t *out, int32_t nthreads)
{
    if (n <= 0 || q < 0) return OR_E_ARG;
    for (int64_t j = 0; j < q; j++)
        if (qs[j] < 0 || qs[j] >= n || qt[j] < 0 || qt[j] >= n) return OR_E_ARG;
    int nt = nthreads_or_default(nthreads);
    if (nt > q) nt = q > 0 ? (int)q : 1;
    int32_t *bufs = (int32_t *)malloc(sizeof(int32_t) * 2 * (size_t)n * (size_t)nt);
    if (!bufs) return OR_E_NOMEM;
    pair_ctx c = {n, row_ptr, col, qs, qt, out, bufs};
    parallel_for(q, 1, nt, pair_body, &c);
    free(bufs);
    return OR_OK;
}

/* Bidirectional local search of the query path (Appendix B, "Applying
 * Bi-Directional Search in the Queries"): from each endpoint, the first tau
 * vertices a plain FIFO BFS discovers (the root first, then each dequeued
 * vertex's neighbours in row order, a vertex counted when it is first seen),
 * each with its exact distance; the answer is the minimum over the vertices
 * both searches discovered of d(s,x) + d(t,x), UINT32_MAX if they share none.
 * It is combined with the landmark answer by a minimum (the common vertices
 * act as landmarks found on the fly). */
static void local_bfs(const int32_t *row_ptr, const int32_t *col, int32_t root, int32_t tau,
                      int32_t *dist, int32_t *list, int32_t *count)
{
    int32_t head = 0, cnt = 0;
    list[cnt++] = root;
    dist[root] = 0;
    while (head < cnt && cnt < tau) {
        const int32_t u = list[head++];
        for (int32_t e = row_ptr[u]; e < row_ptr[u + 1] && cnt < tau; e++) {
            const int32_t v = col[e];
            if (dist[v] == UNREACHED) {
                dist[v] = dist[u] + 1;
                list[cnt++] = v;
            }
        }
    }
    *count = cnt;
}

typedef struct {
    int64_t n;
    const int32_t *row_ptr, *col, *qs, *qt;
    int32_t tau;
    uint32_t *out;
    int32_t *bufs;
} local_ctx;

static void local_body(int64_t lo, int64_t hi, int tid, void *p)
{
    local_ctx *c = (local_ctx *)p;
    const int64_t n = c->n;
    int32_t *ds = c->bufs + (size_t)tid * 2 * ((size_t)n + (size_t)c->tau);
    int32_t *dt = ds + n;
    int32_t *ls = dt + n;
    int32_t *lt = ls + c->tau;
    for (int64_t v = 0; v < n; v++) ds[v] = dt[v] = UNREACHED;
    for (int64_t j = lo; j < hi; j++) {
        int32_t cs = 0, ct = 0;
        local_bfs(c->row_ptr, c->col, c->qs[j], c->tau, ds, ls, &cs);
        local_bfs(c->row_ptr, c->col, c->qt[j], c->tau, dt, lt, &ct);
        uint32_t best = UINT32_MAX;
        for (int32_t k = 0; k < cs; k++) {
            const int32_t x = ls[k];
            if (dt[x] != UNREACHED) {
                const uint32_t cand = (uint32_t)(ds[x] + dt[x]);
                if (cand < best) best = cand;
            }
        }
        c->out[j] = best;
        for (int32_t k = 0; k < cs; k++) ds[ls[k]] = UNREACHED;  /* reset only what was touched */
        for (int32_t k = 0; k < ct; k++) dt[lt[k]] = UNREACHED;
    }
}

int oracle_local_search(int64_t n, const int32_t *row_ptr, const int32_t *col, int64_t q,
                        const int32_t *qs, const int32_t *qt, int32_t tau, uint32_t *out, int32_t nthreads)
{
    if (n <= 0 || q < 0 || tau < 1) return OR_E_ARG;
    for (int64_t j = 0; j < q; j++)
        if (qs[j] < 0 || qs[j] >= n || qt[j] < 0 || qt[j] >= n) return OR_E_ARG;
    int nt = nthreads_or_default(nthreads);
    if (nt > q) nt = q > 0 ? (int)q : 1;
    int32_t *bufs = (int32_t *)malloc(sizeof(int32_t) * 2 * ((size_t)n + (size_t)tau) * (size_t)nt);
    if (!bufs) return OR_E_NOMEM;
    local_ctx c = {n, row_ptr, col, qs, qt, tau, out, bufs};
    parallel_for(q, 64, nt, local_body, &c);
    free(bufs);
    return OR_OK;
}

/* The same query from encoded labels (dist[C][n], masks[C][2R+1][n][1], k <= 64):
 * per cluster, scan offset pairs (a, b) in increasing order of a + b and stop at
 * the first non-empty intersection mask[a][s] & mask[b][t]; the candidate is
 * dist[s] + dist[t] + a + b.  The answer is the minimum over clusters. */
/* Landmark-label answer for one pair from cluster-major encoded labels:
 * per cluster the lowest offset sum whose subsets at s and t intersect. */
static uint32_t label_pair(int64_t n, int32_t num_clusters, int32_t R, const uint32_t *dist,
                           const uint64_t *masks, int32_t s, int32_t t)
{
    const int64_t P = 2 * (int64_t)R + 1;
    uint32_t best = UINT32_MAX;
    for (int32_t c = 0; c < num_clusters; c++) {
        const uint32_t ds = dist[(size_t)c * n + s], dt = dist[(size_t)c * n + t];
        if (ds == UINT32_MAX || dt == UINT32_MAX) continue;
        const uint64_t *mc = masks + (size_t)c * (size_t)P * (size_t)n;
        int found = 0;
        for (int32_t sum = -2 * R; sum <= 2 * R && !found; sum++) {
            for (int32_t a = -R; a <= R; a++) {
                int32_t b = sum - a;
                if (b < -R || b > R) continue;
                if (mc[(size_t)(a + R) * n + s] & mc[(size_t)(b + R) * n + t]) {
                    int64_t val = (int64_t)ds + (int64_t)dt + sum;
                    if ((uint64_t)val < best) best = (uint32_t)val;
                    found = 1;
                    break;
                }
            }
        }
    }
    return best;
}

int oracle_query_labels(int64_t n, int32_t num_clusters, int32_t R, const uint32_t *dist,
                        const uint64_t *masks, int64_t q, const int32_t *qs, const int32_t *qt,
                        uint32_t *ans)
{
    if (n <= 0 || R < 0 || q < 0) return OR_E_ARG;
    for (int64_t p = 0; p < q; p++) {
        const int32_t s = qs[p], t = qt[p];
        if (s < 0 || s >= n || t < 0 || t >= n) return OR_E_ARG;
        ans[p] = label_pair(n, num_clusters, R, dist, masks, s, t);
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------
 * Exact 2-hop labels by pruned BFS (the exact distance oracle of the paper's
 * appendix: pruned landmark labeling, phase 2, run in batches of growing
 * size).
 *
 * Roots are taken in rank order (order[0] first).  Batch i holds the next
 * b_i roots, b_0 = first, b_{i+1} = min(max_batch, floor(b_i * growth)).  Each
 * root h of a batch runs a FIFO BFS; at a vertex u reached at distance d it
 * asks the index as it stood when the batch began: the phase-1 cluster labels
 * (the landmark query over every cluster) and the pairs (r, d_r) already in
 * the labels of both h and u.  If that answer is at most d, u is pruned: it
 * gets no label and is not expanded.  Otherwise (rank(h), d) joins u's label
 * and u's neighbours are visited.  Labels added in a batch become visible to
 * the next batch.  Each vertex's label ends sorted by rank; an entry is
 * (rank << 32) | distance.
 * ------------------------------------------------------------------------ */
typedef struct {
    int64_t n;
    const int32_t *row_ptr, *col;
    int32_t num_clusters, R;
    const uint32_t *bp_dist;
    const uint64_t *bp_masks;
    const int32_t *order;
    int64_t lo_rank;
    int32_t label_cap;
    const int32_t *cnt0;      /* label sizes when the batch began */
    const uint64_t *labels;   /* [n][label_cap] */
    int32_t *dist;            /* [nthreads][n], -1 */
    int32_t *queue;           /* [nthreads][n] */
    uint32_t *root_map;       /* [nthreads][count]: distance of the root to a rank, UINT32_MAX if none */
    uint64_t **out;           /* [nthreads] growable: labelled vertex of each new entry */
    int64_t *out_len, *out_cap;
    uint64_t **out_e;         /* [nthreads] the new entries, (rank << 32) | distance */
    int failed;
} pll_ctx;

static int pll_push(pll_ctx *c, int tid, int32_t v, uint64_t entry)
{
    if (c->out_len[tid] == c->out_cap[tid]) {
        int64_t cap = c->out_cap[tid] ? 2 * c->out_cap[tid] : 1024;
        uint64_t *a = (uint64_t *)realloc(c->out[tid], sizeof(uint64_t) * (size_t)cap);
        uint64_t *b = (uint64_t *)realloc(c->out_e[tid], sizeof(uint64_t) * (size_t)cap);
        if (!a || !b) {
            if (a) c->out[tid] = a;
            if (b) c->out_e[tid] = b;
            return -1;
        }
        c->out[tid] = a;
        c->out_e[tid] = b;
        c->out_cap[tid] = cap;
    }
    c->out[tid][c->out_len[tid]] = (uint64_t)(uint32_t)v;
    c->out_e[tid][c->out_len[tid]] = entry;
    c->out_len[tid]++;
    return 0;
}

static void pll_body(int64_t lo, int64_t hi, int tid, void *p)
{
    pll_ctx *c = (pll_ctx *)p;
    const int64_t n = c->n;
    int32_t *dist = c->dist + (size_t)tid * n;
    int32_t *queue = c->queue + (size_t)tid * n;
    uint32_t *rmap = c->root_map + (size_t)tid * n;
    for (int64_t j = lo; j < hi; j++) {
        const int64_t rank = c->lo_rank + j;
        const int32_t h = c->order[rank];
        const uint64_t *lh = c->labels + (size_t)h * c->label_cap;
        for (int32_t e = 0; e < c->cnt0[h]; e++) rmap[lh[e] >> 32] = (uint32_t)lh[e];
        int64_t head = 0, tail = 0;
        queue[tail++] = h;
        dist[h] = 0;
        while (head < tail) {
            const int32_t u = queue[head++];
            const int32_t d = dist[u];
            /* the index's answer for (h, u) */
            uint32_t q = c->num_clusters ? label_pair(n, c->num_clusters, c->R, c->bp_dist, c->bp_masks, h, u)
                                         : UINT32_MAX;
            const uint64_t *lu = c->labels + (size_t)u * c->label_cap;
            for (int32_t e = 0; e < c->cnt0[u]; e++) {
                const uint32_t dh = rmap[lu[e] >> 32];
                if (dh == UINT32_MAX) continue;
                const uint64_t sum = (uint64_t)dh + (uint32_t)lu[e];
                if (sum < q) q = (uint32_t)sum;
            }
            if (q <= (uint32_t)d) continue; /* pruned */
            if (pll_push(c, tid, u, ((uint64_t)rank << 32) | (uint32_t)d) != 0) {
                c->failed = OR_E_NOMEM;
                break;
            }
            for (int32_t a = c->row_ptr[u]; a < c->row_ptr[u + 1]; a++) {
                const int32_t w = c->col[a];
                if (dist[w] == UNREACHED) {
                    dist[w] = d + 1;
                    queue[tail++] = w;
                }
            }
        }
        for (int64_t k = 0; k < tail; k++) dist[queue[k]] = UNREACHED;
        for (int32_t e = 0; e < c->cnt0[h]; e++) rmap[lh[e] >> 32] = UINT32_MAX;
    }
}

static int cmp_u64(const void *a, const void *b)
{
    const uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

int oracle_pll(int64_t n, const int32_t *row_ptr, const int32_t *col, int32_t num_clusters, int32_t R,
               const uint32_t *bp_dist, const uint64_t *bp_masks, int64_t count, const int32_t *order,
               int32_t first, double growth, int32_t max_batch, int32_t label_cap, int32_t *lab_cnt,
               uint64_t *labels, int32_t nthreads)
{
    if (n <= 0 || count < 0 || count > n || num_clusters < 0 || R < 0 || first < 1 || !(growth >= 1.0) ||
        max_batch < 1 || label_cap < 1 || (num_clusters > 0 && (!bp_dist || !bp_masks)))
        return OR_E_ARG;
    for (int64_t k = 0; k < count; k++)
        if (order[k] < 0 || order[k] >= n) return OR_E_ARG;
    int nt = nthreads_or_default(nthreads);
    int32_t *dist = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * nt);
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * nt);
    uint32_t *rmap = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n * nt);
    int32_t *cnt0 = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    uint64_t **out = (uint64_t **)calloc((size_t)nt, sizeof(uint64_t *));
    uint64_t **out_e = (uint64_t **)calloc((size_t)nt, sizeof(uint64_t *));
    int64_t *out_len = (int64_t *)calloc((size_t)nt, sizeof(int64_t));
    int64_t *out_cap = (int64_t *)calloc((size_t)nt, sizeof(int64_t));
    int rc = OR_OK;
    if (!dist || !queue || !rmap || !cnt0 || !out || !out_e || !out_len || !out_cap) {
        rc = OR_E_NOMEM;
        goto done;
    }
    for (size_t k = 0; k < (size_t)n * nt; k++) {
        dist[k] = UNREACHED;
        rmap[k] = UINT32_MAX;
    }
    for (int64_t v = 0; v < n; v++) lab_cnt[v] = 0;
    pll_ctx c;
    memset(&c, 0, sizeof(c));
    c.n = n;
    c.row_ptr = row_ptr;
    c.col = col;
    c.num_clusters = num_clusters;
    c.R = R;
    c.bp_dist = bp_dist;
    c.bp_masks = bp_masks;
    c.order = order;
    c.label_cap = label_cap;
    c.cnt0 = cnt0;
    c.labels = labels;
    c.dist = dist;
    c.queue = queue;
    c.root_map = rmap;
    c.out = out;
    c.out_e = out_e;
    c.out_len = out_len;
    c.out_cap = out_cap;
    int64_t b = first;
    for (int64_t lo = 0; lo < count;) {
        const int64_t size = b < count - lo ? b : count - lo;
        memcpy(cnt0, lab_cnt, sizeof(int32_t) * (size_t)n);
        c.lo_rank = lo;
        for (int t = 0; t < nt; t++) out_len[t] = 0;
        parallel_for(size, 1, nt, pll_body, &c);
        if (c.failed) {
            rc = c.failed;
            goto done;
        }
        for (int t = 0; t < nt; t++)
            for (int64_t k = 0; k < out_len[t]; k++) {
                const int32_t v = (int32_t)out[t][k];
                if (lab_cnt[v] >= label_cap) {
                    rc = OR_E_CAPACITY;
                    goto done;
                }
                labels[(size_t)v * label_cap + lab_cnt[v]++] = out_e[t][k];
            }
        lo += size;
        int64_t nb = (int64_t)((double)b * growth);
        b = nb < max_batch ? nb : max_batch;
        if (b < 1) b = 1;
    }
    for (int64_t v = 0; v < n; v++) qsort(labels + (size_t)v * label_cap, (size_t)lab_cnt[v], sizeof(uint64_t), cmp_u64);
done:
    if (out)
        for (int t = 0; t < nt; t++) free(out[t]);
    if (out_e)
        for (int t = 0; t < nt; t++) free(out_e[t]);
    free(out);
    free(out_e);
    free(out_len);
    free(out_cap);
    free(dist);
    free(queue);
    free(rmap);
    free(cnt0);
    return rc;
}

/* Query of the exact oracle: the lowest of the phase-1 landmark answer and
 * min over ranks in both labels of the two distances' sum (labels sorted by
 * rank, merged). */
int oracle_pll_query(int64_t n, int32_t num_clusters, int32_t R, const uint32_t *bp_dist,
                     const uint64_t *bp_masks, int32_t label_cap, const int32_t *lab_cnt, const uint64_t *labels,
                     int64_t q, const int32_t *qs, const int32_t *qt, uint32_t *ans)
{
    if (n <= 0 || num_clusters < 0 || R < 0 || label_cap < 1 || q < 0) return OR_E_ARG;
    for (int64_t p = 0; p < q; p++) {
        const int32_t s = qs[p], t = qt[p];
        if (s < 0 || s >= n || t < 0 || t >= n) return OR_E_ARG;
        uint32_t best = num_clusters ? label_pair(n, num_clusters, R, bp_dist, bp_masks, s, t) : UINT32_MAX;
        const uint64_t *ls = labels + (size_t)s * label_cap, *lt = labels + (size_t)t * label_cap;
        int32_t i = 0, j = 0;
        while (i < lab_cnt[s] && j < lab_cnt[t]) {
            const uint64_t rs = ls[i] >> 32, rt = lt[j] >> 32;
            if (rs < rt) i++;
            else if (rt < rs) j++;
            else {
                const uint64_t sum = (uint64_t)(uint32_t)ls[i] + (uint32_t)lt[j];
                if (sum < best) best = (uint32_t)sum;
                i++;
                j++;
            }
        }
        ans[p] = best;
    }
    return OR_OK;
}

/* BFS certificate for one encoded cluster output (no oracle run needed).
 * With delta_i(v) = dist[v] + offset of bit i at v, the decoded distances are
 * the true hop distances iff: delta_i(s_i) = 0 and no other vertex is 0; every
 * arc (u, v) has |delta_i(u) - delta_i(v)| <= 1 (unreached on both ends or on
 * neither); every reached v != s_i has a neighbour at delta_i(v) - 1.  Each
 * reached v must carry bit i in exactly one plane; unreached v carry no bits.
 * Returns the number of violations found (0 = certified), or a negative error. */
typedef struct {
    int64_t n;
    const int32_t *row_ptr, *col;
    int32_t k;
    const int32_t *S;
    int32_t R, W;
    int64_t P;
    const uint32_t *dist;
    const uint64_t *masks;
    int32_t *d;
    int64_t *bad;
} cert_ctx;

static void cert_decode_body(int64_t lo, int64_t hi, int tid, void *p)
{
    cert_ctx *c = (cert_ctx *)p;
    const int64_t n = c->n;
    int64_t bad = 0;
    for (int64_t v = lo; v < hi; v++) {
        for (int32_t i = 0; i < c->k; i++) {
            int32_t found = 0, off = 0;
            for (int64_t pl = 0; pl < c->P; pl++) {
                const uint64_t w = c->masks[((size_t)pl * n + v) * c->W + (size_t)(i / 64)];
                if ((w >> (i % 64)) & 1) {
                    found++;
                    off = (int32_t)(pl - c->R);
                }
            }
            if (c->dist[v] == UINT32_MAX) {
                if (found) bad++;
                c->d[(size_t)i * n + v] = UNREACHED;
            } else {
                if (found != 1) bad++;
                c->d[(size_t)i * n + v] = (int32_t)c->dist[v] + off;
            }
        }
    }
    c->bad[tid] += bad;
}

static void cert_check_body(int64_t lo, int64_t hi, int tid, void *p)
{
    cert_ctx *c = (cert_ctx *)p;
    const int64_t n = c->n;
    int64_t bad = 0;
    for (int64_t v = lo; v < hi; v++) {
        for (int32_t i = 0; i < c->k; i++) {
            const int32_t dv = c->d[(size_t)i * n + v];
            if (v == c->S[i]) {
                if (dv != 0) bad++;
            } else if (dv == 0) {
                bad++;
            }
            int has_parent = 0;
            for (int32_t e = c->row_ptr[v]; e < c->row_ptr[v + 1]; e++) {
                const int32_t du = c->d[(size_t)i * n + c->col[e]];
                if ((du == UNREACHED) != (dv == UNREACHED)) {
                    bad++;
                    continue;
                }
                if (dv == UNREACHED) continue;
                if (du - dv > 1 || dv - du > 1) bad++;
                if (du == dv - 1) has_parent = 1;
            }
            if (dv > 0 && !has_parent) bad++;
        }
    }
    c->bad[tid] += bad;
}

int64_t oracle_certificate(int64_t n, const int32_t *row_ptr, const int32_t *col, int32_t k,
                           const int32_t *S, int32_t R, int32_t W, const uint32_t *dist,
                           const uint64_t *masks, int32_t nthreads)
{
    if (n <= 0 || k < 1 || k > 64 * W || R < 0) return OR_E_ARG;
    int nt = nthreads_or_default(nthreads);
    const int64_t P = 2 * (int64_t)R + 1;
    int32_t *d = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * (size_t)k);
    if (!d) return OR_E_NOMEM;
    int64_t bad_by_thread[MAX_THREADS] = {0};
    cert_ctx cc = {n, row_ptr, col, k, S, R, W, P, dist, masks, d, bad_by_thread};
    parallel_for(n, 4096, nt, cert_decode_body, &cc);
    parallel_for(n, 1024, nt, cert_check_body, &cc);
    int64_t bad = 0;
    for (int t = 0; t < nt; t++) bad += bad_by_thread[t];
    free(d);
    return bad;
}

/* The same certificate evaluated a word of sources at a time, for clusters
 * too large to decode per source.  For a reached vertex v, level t holds
 * L_v(t) = {i : delta_i(v) = t}: the plane t - dist[v] + R (empty outside
 * [0, 2R]).  Per 64-bit word the conditions are:
 *   the planes of v are pairwise disjoint and together hold every source of
 *   the cluster (reached v), or are all empty (unreached v);
 *   the center (bit 0) sits at offset 0, so dist[v] = delta_0(v);
 *   no level below 0, and L_v(0) = the sources equal to v;
 *   every arc (v, u): u is reached iff v is, and L_v(t) lies within
 *   L_u(t-1) | L_u(t) | L_u(t+1) (|delta_i(u) - delta_i(v)| <= 1);
 *   every t > 0: L_v(t) lies within the union over neighbours u of L_u(t-1)
 *   (each source has a neighbour one level closer).
 * Returns the number of (vertex, condition, word) violations. */
typedef struct {
    int64_t n;
    const int32_t *row_ptr, *col;
    int32_t k;
    const int32_t *src_v, *src_i;  /* the sources sorted by vertex, and their indices */
    int32_t R, W;
    int64_t P;
    const uint32_t *dist;
    const uint64_t *masks;
    uint64_t *scratch;             /* per thread: P * W parent words + W source words */
    int64_t *bad;
} certw_ctx;

static uint64_t certw_level(const certw_ctx *c, int64_t v, int64_t t, int32_t w)
{
    const uint32_t dv = c->dist[v];
    if (dv == UINT32_MAX) return 0;
    const int64_t p = t - (int64_t)dv + c->R;
    if (p < 0 || p >= c->P) return 0;
    return c->masks[((size_t)p * c->n + (size_t)v) * c->W + (size_t)w];
}

static void certw_body(int64_t lo, int64_t hi, int tid, void *p)
{
    certw_ctx *c = (certw_ctx *)p;
    const int64_t n = c->n, P = c->P;
    const int32_t W = c->W, R = c->R;
    uint64_t *par = c->scratch + (size_t)tid * (size_t)(P + 1) * W;
    uint64_t *srcw = par + (size_t)P * W;
    int64_t bad = 0;
    for (int64_t v = lo; v < hi; v++) {
        const uint32_t dv = c->dist[v];
        /* sources equal to v */
        for (int32_t w = 0; w < W; w++) srcw[w] = 0;
        {
            int32_t a = 0, b = c->k;
            while (a < b) {
                const int32_t m = (a + b) / 2;
                if (c->src_v[m] < v) a = m + 1;
                else b = m;
            }
            for (int32_t j = a; j < c->k && c->src_v[j] == v; j++)
                srcw[c->src_i[j] / 64] |= 1ull << (c->src_i[j] % 64);
        }
        if (dv == UINT32_MAX) {
            for (int64_t pl = 0; pl < P; pl++)
                for (int32_t w = 0; w < W; w++)
                    if (c->masks[((size_t)pl * n + (size_t)v) * W + (size_t)w]) bad++;
            for (int32_t w = 0; w < W; w++)
                if (srcw[w]) bad++;
            for (int32_t e = c->row_ptr[v]; e < c->row_ptr[v + 1]; e++)
                if (c->dist[c->col[e]] != UINT32_MAX) bad++;
            continue;
        }
        for (int32_t w = 0; w < W; w++) {
            uint64_t acc = 0;
            for (int64_t pl = 0; pl < P; pl++) {
                const uint64_t x = c->masks[((size_t)pl * n + (size_t)v) * W + (size_t)w];
                if (acc & x) bad++;
                acc |= x;
                if ((int64_t)dv + pl - R < 0 && x) bad++;
            }
            const int32_t lo_i = 64 * w;
            uint64_t fullw = 0;
            if (c->k >= lo_i + 64) fullw = ~0ull;
            else if (c->k > lo_i) fullw = (1ull << (c->k - lo_i)) - 1;
            if (acc != fullw) bad++;
            if (certw_level(c, v, 0, w) != srcw[w]) bad++;
        }
        if (!(c->masks[((size_t)R * n + (size_t)v) * W] & 1ull)) bad++;
        for (int64_t i = 0; i < P * W; i++) par[i] = 0;
        for (int32_t e = c->row_ptr[v]; e < c->row_ptr[v + 1]; e++) {
            const int64_t u = c->col[e];
            const uint32_t du = c->dist[u];
            if (du == UINT32_MAX) {
                bad++;
                continue;
            }
            /* level t of v is plane t - du + R of u: shift = dv - du */
            const int64_t shift = (int64_t)dv - (int64_t)du;
            for (int64_t pl = 0; pl < P; pl++) {
                for (int32_t w = 0; w < W; w++) {
                    const uint64_t x = c->masks[((size_t)pl * n + (size_t)v) * W + (size_t)w];
                    uint64_t lu[3];  /* u at levels t - 1, t, t + 1 */
                    for (int q = 0; q < 3; q++) {
                        const int64_t pu = pl + shift + q - 1;
                        lu[q] = (pu >= 0 && pu < P) ? c->masks[((size_t)pu * n + (size_t)u) * W + (size_t)w] : 0;
                    }
                    if (x & ~(lu[0] | lu[1] | lu[2])) bad++;
                    par[pl * W + w] |= lu[0];
                }
            }
        }
        for (int64_t pl = 0; pl < P; pl++) {
            if ((int64_t)dv + pl - R <= 0) continue;
            for (int32_t w = 0; w < W; w++)
                if (c->masks[((size_t)pl * n + (size_t)v) * W + (size_t)w] & ~par[pl * W + w]) bad++;
        }
    }
    c->bad[tid] += bad;
}

typedef struct {
    int32_t v, i;
} src_pair;

static int cmp_src_pair(const void *a, const void *b)
{
    const src_pair *x = (const src_pair *)a, *y = (const src_pair *)b;
    if (x->v != y->v) return (x->v > y->v) - (x->v < y->v);
    return (x->i > y->i) - (x->i < y->i);
}

int64_t oracle_certificate_words(int64_t n, const int32_t *row_ptr, const int32_t *col, int32_t k,
                                 const int32_t *S, int32_t R, int32_t W, const uint32_t *dist,
                                 const uint64_t *masks, int32_t nthreads)
{
    if (n <= 0 || k < 1 || k > 64 * W || R < 0) return OR_E_ARG;
    int nt = nthreads_or_default(nthreads);
    const int64_t P = 2 * (int64_t)R + 1;
    src_pair *sp = (src_pair *)malloc(sizeof(src_pair) * (size_t)k);
    int32_t *sv = (int32_t *)malloc(sizeof(int32_t) * (size_t)k);
    int32_t *si = (int32_t *)malloc(sizeof(int32_t) * (size_t)k);
    uint64_t *scratch = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)MAX_THREADS * (size_t)(P + 1) * (size_t)W);
    if (!sp || !sv || !si || !scratch) {
        free(sp);
        free(sv);
        free(si);
        free(scratch);
        return OR_E_NOMEM;
    }
    for (int32_t i = 0; i < k; i++) {
        sp[i].v = S[i];
        sp[i].i = i;
    }
    qsort(sp, (size_t)k, sizeof(src_pair), cmp_src_pair);
    for (int32_t i = 0; i < k; i++) {
        sv[i] = sp[i].v;
        si[i] = sp[i].i;
    }
    int64_t bad_by_thread[MAX_THREADS] = {0};
    certw_ctx cc = {n, row_ptr, col, k, sv, si, R, W, P, dist, masks, scratch, bad_by_thread};
    parallel_for(n, 1024, nt, certw_body, &cc);
    int64_t bad = 0;
    for (int t = 0; t < nt; t++) bad += bad_by_thread[t];
    free(sp);
    free(sv);
    free(si);
    free(scratch);
    return bad;
}

/* ---------------------------------------------------------------------------
 * Graph cleanup.  flags: 1 symmetrize, 2 dedup, 4 drop self-loops, 8 keep the
 * largest connected component (ties: the component holding the smallest
 * original id).  Kept vertices are relabelled 0..n-1 in ascending original-id
 * order; each output row is sorted ascending.  The CSR is returned in buffers
 * allocated here (release with oracle_free).
 * ------------------------------------------------------------------------- */
static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

static int64_t uf_find(int64_t *parent, int64_t x)
{
    while (parent[x] != x) {
        parent[x] = parent[parent[x]];
        x = parent[x];
    }
    return x;
}

void oracle_free(void *p) { free(p); }

typedef struct {
    const int64_t *off;
    int32_t *adj;
    int64_t *fill;
    int dedup;
} sort_rows_ctx;

static void sort_rows_body(int64_t lo, int64_t hi, int tid, void *p)
{
    (void)tid;
    sort_rows_ctx *c = (sort_rows_ctx *)p;
    for (int64_t v = lo; v < hi; v++) {
        int32_t *row = c->adj + c->off[v];
        int64_t len = c->off[v + 1] - c->off[v];
        qsort(row, (size_t)len, sizeof(int32_t), cmp_i32);
        if (c->dedup && len > 1) {
            int64_t w = 1;
            for (int64_t j = 1; j < len; j++)
                if (row[j] != row[w - 1]) row[w++] = row[j];
            len = w;
        }
        c->fill[v] = len;
    }
}

int oracle_clean_csr(int64_t n_in, int64_t num_edges, const int64_t *src, const int64_t *dst,
                     uint32_t flags, int64_t *old_to_new, int64_t *n_out, int64_t *m_out,
                     int32_t **row_ptr_out, int32_t **col_out)
{
    if (n_in <= 0 || n_in > INT32_MAX || num_edges < 0) return OR_E_ARG;
    for (int64_t e = 0; e < num_edges; e++)
        if (src[e] < 0 || src[e] >= n_in || dst[e] < 0 || dst[e] >= n_in) return OR_E_ARG;
    const int sym = (flags & 1) != 0, dedup = (flags & 2) != 0, noloop = (flags & 4) != 0,
              lcc = (flags & 8) != 0;

    /* bucket the arcs by tail */
    int64_t *off = (int64_t *)calloc((size_t)n_in + 1, sizeof(int64_t));
    if (!off) return OR_E_NOMEM;
    for (int64_t e = 0; e < num_edges; e++) {
        if (noloop && src[e] == dst[e]) continue;
        off[src[e] + 1]++;
        if (sym) off[dst[e] + 1]++;
    }
    for (int64_t v = 0; v < n_in; v++) off[v + 1] += off[v];
    const int64_t A = off[n_in];
    int32_t *adj = (int32_t *)malloc(sizeof(int32_t) * (size_t)(A > 0 ? A : 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)n_in);
    if (!adj || !fill) {
        free(off);
        free(adj);
        free(fill);
        return OR_E_NOMEM;
    }
    memcpy(fill, off, sizeof(int64_t) * (size_t)n_in);
    for (int64_t e = 0; e < num_edges; e++) {
        if (noloop && src[e] == dst[e]) continue;
        adj[fill[src[e]]++] = (int32_t)dst[e];
        if (sym) adj[fill[dst[e]]++] = (int32_t)src[e];
    }
    /* sort (and dedup) every row; fill[v] becomes the row's kept length */
    sort_rows_ctx sc = {off, adj, fill, dedup};
    parallel_for(n_in, 4096, nthreads_or_default(0), sort_rows_body, &sc);
    /* components (union-find over arcs, arcs taken as undirected) */
    char *keep = (char *)malloc((size_t)n_in);
    if (!keep) {
        free(off);
        free(adj);
        free(fill);
        return OR_E_NOMEM;
    }
    if (lcc) {
        int64_t *parent = (int64_t *)malloc(sizeof(int64_t) * (size_t)n_in);
        int64_t *size = (int64_t *)calloc((size_t)n_in, sizeof(int64_t));
        if (!parent || !size) {
            free(parent);
            free(size);
            free(off);
            free(adj);
            free(fill);
            free(keep);
            return OR_E_NOMEM;
        }
        for (int64_t v = 0; v < n_in; v++) parent[v] = v;
        for (int64_t v = 0; v < n_in; v++)
            for (int64_t j = 0; j < fill[v]; j++) {
                int64_t a = uf_find(parent, v), b = uf_find(parent, adj[off[v] + j]);
                if (a != b) {
                    if (a < b) parent[b] = a;
                    else parent[a] = b;
                }
            }
        for (int64_t v = 0; v < n_in; v++) size[uf_find(parent, v)]++;
        /* roots are the smallest id of their component (union keeps the smaller
         * root), so scanning ids upward meets components by smallest id */
        int64_t best = -1;
        for (int64_t v = 0; v < n_in; v++)
            if (parent[v] == v && (best < 0 || size[v] > size[best])) best = v;
        for (int64_t v = 0; v < n_in; v++) keep[v] = uf_find(parent, v) == best;
        free(parent);
        free(size);
    } else {
        memset(keep, 1, (size_t)n_in);
    }
    int64_t n = 0;
    for (int64_t v = 0; v < n_in; v++) old_to_new[v] = keep[v] ? n++ : -1;
    int64_t m = 0;
    for (int64_t v = 0; v < n_in; v++)
        if (keep[v])
            for (int64_t j = 0; j < fill[v]; j++) m += keep[adj[off[v] + j]] ? 1 : 0;
    if (m > INT32_MAX) {
        free(off);
        free(adj);
        free(fill);
        free(keep);
        return OR_E_ARG;
    }
    int32_t *rp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1));
    int32_t *cl = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    if (!rp || !cl) {
        free(rp);
        free(cl);
        free(off);
        free(adj);
        free(fill);
        free(keep);
        return OR_E_NOMEM;
    }
    int64_t pos = 0, r = 0;
    rp[0] = 0;
    for (int64_t v = 0; v < n_in; v++) {
        if (!keep[v]) continue;
        for (int64_t j = 0; j < fill[v]; j++) {
            int32_t u = adj[off[v] + j];
            if (keep[u]) cl[pos++] = (int32_t)old_to_new[u];
        }
        rp[++r] = (int32_t)pos;
    }
    free(off);
    free(adj);
    free(fill);
    free(keep);
    *n_out = n;
    *m_out = m;
    *row_ptr_out = rp;
    *col_out = cl;
    return OR_OK;
}
