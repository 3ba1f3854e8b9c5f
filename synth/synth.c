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
#include <stdint.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

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
void synth_rmat(int32_t scale, int64_t n_edges, double a, double b, double c, uint64_t base,
                int64_t *src, int64_t *dst)
{
    const double ab = a + b, abc = a + b + c;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < n_edges; e++) {
        int64_t s = 0, t = 0;
        for (int32_t l = 0; l < scale; l++) {
            double r = unit(draw(base, (uint64_t)e * (uint64_t)scale + (uint64_t)l));
            int row = r >= ab;
            int colb = (r >= a && r < ab) || r >= abc;
            s = (s << 1) | row;
            t = (t << 1) | colb;
        }
        src[e] = s;
        dst[e] = t;
    }
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
void synth_alias_pairs(int64_t n, const double *prob, const int64_t *alias, int64_t n_edges,
                       uint64_t base, int64_t *src, int64_t *dst)
{
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < n_edges; e++) {
        int64_t ends[2];
        for (int h = 0; h < 2; h++) {
            uint64_t j = 2 * (uint64_t)e + (uint64_t)h;
            uint64_t x = draw(base, 2 * j);
            int64_t col = (int64_t)(((unsigned __int128)x * (unsigned __int128)(uint64_t)n) >> 64);
            double coin = unit(draw(base, 2 * j + 1));
            ends[h] = coin < prob[col] ? col : alias[col];
        }
        src[e] = ends[0];
        dst[e] = ends[1];
    }
}
