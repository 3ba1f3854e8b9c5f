/*
 * Fast seeded raw-edge generators for the large synthetic workloads.
 * Random draws only: no cleanup, no Cluster-BFS arithmetic.
 *
 * Random numbers: SplitMix64 (Steele, Lea, Flood, OOPSLA 2014) used as a
 * counter-based generator.  Stream (seed, key) starts from
 *     base = mix(mix(seed) ^ key)
 * and its draw number i is mix(base + (i + 1) * 0x9E3779B97F4A7C15), where mix is
 * the SplitMix64 output function.  A uniform double is the top 53 bits * 2^-53.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <unistd.h>

/* Split [0, n) into one contiguous range per thread (OMP_NUM_THREADS, else
 * the online CPUs) and run fn on each; draws are indexed by position, so the
 * split does not change any output. */
typedef void (*range_fn)(int64_t lo, int64_t hi, void *ctx);
typedef struct {
    range_fn fn;
    void *ctx;
    int64_t lo, hi;
} range_arg;

static void *range_worker(void *p)
{
    range_arg *a = (range_arg *)p;
    a->fn(a->lo, a->hi, a->ctx);
    return NULL;
}

static void parallel_ranges(int64_t n, range_fn fn, void *ctx)
{
    const char *env = getenv("OMP_NUM_THREADS");
    int nt = env ? atoi(env) : 0;
    if (nt <= 0) nt = (int)sysconf(_SC_NPROCESSORS_ONLN);
    if (nt < 1) nt = 1;
    if (nt > 64) nt = 64;
    if (n < 65536) nt = 1;
    pthread_t th[64];
    range_arg args[64];
    int started = 0;
    for (int t = 0; t < nt; t++) {
        args[t].fn = fn;
        args[t].ctx = ctx;
        args[t].lo = n * t / nt;
        args[t].hi = n * (t + 1) / nt;
    }
    for (int t = 1; t < nt; t++) {
        if (pthread_create(&th[t], NULL, range_worker, &args[t]) != 0) {
            fn(args[t].lo, args[t].hi, ctx);
            continue;
        }
        th[started++] = th[t];
    }
    fn(args[0].lo, args[0].hi, ctx);
    for (int t = 0; t < started; t++) pthread_join(th[t], NULL);
}

static inline uint64_t mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static inline uint64_t draw(uint64_t base, uint64_t i)
{
    return mix(base + (i + 1) * 0x9E3779B97F4A7C15ULL);
}

static inline double unit(uint64_t x) { return (double)(x >> 11) * (1.0 / 9007199254740992.0); }

uint64_t synth_stream_base(uint64_t seed, uint64_t key) { return mix(mix(seed) ^ key); }

uint64_t synth_draw(uint64_t base, uint64_t i) { return draw(base, i); }

/* R-MAT: edge e uses draws e*scale + l for levels l = 0..scale-1 (most
 * significant bit first).  Quadrant c or d sets the row bit, b or d the column bit. */
typedef struct {
    int32_t scale;
    double a, ab, abc;
    uint64_t base;
    int64_t *src, *dst;
} rmat_ctx;

static void rmat_range(int64_t lo, int64_t hi, void *p)
{
    rmat_ctx *c = (rmat_ctx *)p;
    for (int64_t e = lo; e < hi; e++) {
        int64_t s = 0, t = 0;
        for (int32_t l = 0; l < c->scale; l++) {
            double r = unit(draw(c->base, (uint64_t)e * (uint64_t)c->scale + (uint64_t)l));
            int row = r >= c->ab;
            int colb = (r >= c->a && r < c->ab) || r >= c->abc;
            s = (s << 1) | row;
            t = (t << 1) | colb;
        }
        c->src[e] = s;
        c->dst[e] = t;
    }
}

void synth_rmat(int32_t scale, int64_t n_edges, double a, double b, double c, uint64_t base,
                int64_t *src, int64_t *dst)
{
    rmat_ctx ctx = {scale, a, a + b, a + b + c, base, src, dst};
    parallel_ranges(n_edges, rmat_range, &ctx);
}

/* Walker/Vose alias table for the distribution proportional to w[0..n). */
int synth_alias_build(int64_t n, const double *w, double *prob, int64_t *alias)
{
    double total = 0.0;
    for (int64_t i = 0; i < n; i++) total += w[i];
    int64_t *small = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *large = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    double *p = (double *)malloc(sizeof(double) * (size_t)n);
    if (!small || !large || !p) {
        free(small);
        free(large);
        free(p);
        return -1;
    }
    int64_t ns = 0, nl = 0;
    for (int64_t i = 0; i < n; i++) {
        p[i] = w[i] * (double)n / total;
        if (p[i] < 1.0) small[ns++] = i;
        else large[nl++] = i;
    }
    while (ns > 0 && nl > 0) {
        int64_t s = small[--ns], l = large[--nl];
        prob[s] = p[s];
        alias[s] = l;
        p[l] = (p[l] + p[s]) - 1.0;
        if (p[l] < 1.0) small[ns++] = l;
        else large[nl++] = l;
    }
    while (nl > 0) {
        int64_t l = large[--nl];
        prob[l] = 1.0;
        alias[l] = l;
    }
    while (ns > 0) {
        int64_t s = small[--ns];
        prob[s] = 1.0;
        alias[s] = s;
    }
    free(small);
    free(large);
    free(p);
    return 0;
}

/* Endpoint j in [0, 2*n_edges) uses draws 2j (column) and 2j+1 (coin);
 * endpoint 2e is the src of edge e and 2e+1 its dst. */
typedef struct {
    int64_t n;
    const double *prob;
    const int64_t *alias;
    uint64_t base;
    int64_t *src, *dst;
} alias_ctx;

static void alias_range(int64_t lo, int64_t hi, void *p)
{
    alias_ctx *c = (alias_ctx *)p;
    for (int64_t e = lo; e < hi; e++) {
        int64_t ends[2];
        for (int h = 0; h < 2; h++) {
            uint64_t j = 2 * (uint64_t)e + (uint64_t)h;
            uint64_t x = draw(c->base, 2 * j);
            int64_t col = (int64_t)(((unsigned __int128)x * (unsigned __int128)(uint64_t)c->n) >> 64);
            double coin = unit(draw(c->base, 2 * j + 1));
            ends[h] = coin < c->prob[col] ? col : c->alias[col];
        }
        c->src[e] = ends[0];
        c->dst[e] = ends[1];
    }
}

void synth_alias_pairs(int64_t n, const double *prob, const int64_t *alias, int64_t n_edges,
                       uint64_t base, int64_t *src, int64_t *dst)
{
    alias_ctx ctx = {n, prob, alias, base, src, dst};
    parallel_ranges(n_edges, alias_range, &ctx);
}
