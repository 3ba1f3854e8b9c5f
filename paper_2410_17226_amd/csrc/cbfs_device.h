// Device-side building blocks of the Cluster-BFS level loop (gfx950, wave64).
//
// State of one cluster group (several clusters packed into W 64-bit words per
// vertex; cluster j of the group owns words [j*WC, (j+1)*WC), or, for
// clusters of at most 32 sources, a field of 2^flog bits: clusters
// j*F .. j*F + F-1 share word j, F = 64 >> flog, cluster j*F + f at bits
// [f << flog, (f + 1) << flog) with its center at the field's bit 0):
//   A, B   [n][W]  the paper's S_next / "seen so far" arrays, double-buffered:
//                  in round i, cur = (i even ? A : B) holds Seen_i(v), the set
//                  of sources within distance i of v, complete for every v, and
//                  nxt (the other buffer) accumulates Seen_{i+1}(v).
//   seen   [n][W]  Seen_{i-1}(v): lets the vertex phase form the new bits
//                  Seen_i \ Seen_{i-1} while other threads already OR round-i
//                  contributions into nxt.
//   queue  3 x [cap] int64 frontier entries (piece << 32 | vertex); a vertex of
//                  degree deg occupies max(1, ceil(deg / PIECE)) pieces so that
//                  no work item carries more than PIECE arcs.  Round i reads
//                  queue[i%3] (F_i), fills queue[(i+1)%3] and may use
//                  queue[(i+2)%3] (F_{i-1}) to clear F_{i-1}'s bitmap words.
//   bits   3 x [ceil(n/64)] frontier membership bitmaps; round i reads bits[i%3],
//                  fills bits[(i+1)%3] and clears bits[(i+2)%3] (F_{i-1}).
//   ctr    4 x 4 counters per rotation: pieces, vertices, degree sum, spare.
//                  Round i reads ctr[i%4] and ctr[(i-1)%4], fills ctr[(i+1)%4]
//                  and clears ctr[(i+2)%4].
//
// Invariant (Algorithm "Cluster-BFS search from S", Section 3.2): after the
// vertex phase of round i, Seen_i(u) = {s : d(s,u) <= i}; the edge phase makes
// nxt(v) = Seen_i(v) | OR_{u in N(v)} Seen_i(u) = Seen_{i+1}(v), and v joins
// F_{i+1} iff that adds a bit.  A vertex whose set is full (all sources) is
// finished: it can receive nothing more.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace cbfs {

constexpr int BLOCK = 256;          // threads per block (4 waves of 64)
constexpr int WAVES = BLOCK / 64;
constexpr int PIECE = 256;          // max arcs per frontier work item (push)
constexpr int TILE_ITEMS = 6144;    // merge-path items (rows + arcs) per pull block (LDS for 5 blocks per CU)
constexpr int IPT = TILE_ITEMS / BLOCK;
static_assert(TILE_ITEMS + 2 <= 65535, "pull tiles stage row ends as 16-bit offsets");
constexpr int PULL_CLAIM_WORDS = TILE_ITEMS / 64 + 2;  // bitmap words spanned by a tile's rows
constexpr int PULL_ROW_WORDS = (TILE_ITEMS + 1 + 63) / 64;  // one bit per row of a tile
static_assert(PULL_CLAIM_WORDS <= BLOCK, "one claimed word per thread at a pull tile's flush");
enum { PULL_WALK = 0, PULL_WAVE = 1 };  // forms of the pull round
constexpr int HUB_MAX = 256;        // frontier vertices of a range-owned push round at most
constexpr int HUB_RANGE = 256;      // target vertices owned by one range-owned push block
constexpr int HUB_RANGE_LOG = 8;
static_assert(HUB_RANGE == 1 << HUB_RANGE_LOG, "HUB_RANGE_LOG is log2 of HUB_RANGE");
constexpr int HB_CHUNK = 4096;      // arcs per block of the slice-bounds pass
// row length of the range-owned push's slice-bounds table: one entry per owned
// range and one past the last
__host__ __device__ inline int64_t hub_bounds_stride(int64_t n) { return (n + HUB_RANGE - 1) / HUB_RANGE + 1; }
constexpr int STAGE_CAP = 1024;     // LDS frontier staging capacity per push/seed block
constexpr int SEED_PER_BLOCK = 64;  // sources per block of a seed launch
// arcs per pass when each push thread walks its own entry (wide groups hold
// fewer neighbour sets in registers)
template <int W>
constexpr int push_direct_batch() { return W <= 2 ? 4 : 2; }
static_assert(BLOCK * 4 <= STAGE_CAP, "one direct push pass fits the LDS stager");
constexpr int MAX_W = 16;           // max words per vertex in a group
constexpr uint32_t UNREACHED = 0xFFFFFFFFu;
constexpr int32_t E_RADIUS = -5;
constexpr int32_t E_HIP = -7;

struct GraphArgs {
    int64_t n, m;
    const int32_t *row_ptr;
    const int32_t *col;
    const int32_t *tile_row;   // [ntiles+1] merge-path row coordinate of each pull tile
    const int32_t *tile_edge;  // [ntiles+1] merge-path arc coordinate of each pull tile
    int32_t ntiles;
};

struct SlotArgs {
    uint64_t *A, *B, *seen;
    int64_t *q0, *q1, *q2;
    uint64_t *bits0, *bits1, *bits2;
    unsigned long long *ctr;  // [4][4]
    int64_t nwords;           // bitmap words
};

struct GroupDesc {
    int32_t c0;               // global index of the group's first cluster
    int32_t nc;               // clusters in the group
    int32_t flog;             // log2 of a cluster's field width: 6 = whole words, 3..5 = 8..32 bits
    int32_t pad;
    uint64_t full[MAX_W];     // per word: bits of sources present
};

// Units of a group: WC words each; a unit of one word holds fields_per_word
// clusters (1 unless fields are narrower than a word).
__device__ __forceinline__ int32_t fields_per_word(const GroupDesc &g) { return 1 << (6 - g.flog); }
__device__ __forceinline__ uint64_t field_mask(const GroupDesc &g)
{
    return g.flog >= 6 ? ~0ull : ((1ull << (1 << g.flog)) - 1ull);
}
template <int WC>
__device__ __forceinline__ int32_t units_of(const GroupDesc &g)
{
    if constexpr (WC > 1) return g.nc;
    else return (g.nc + fields_per_word(g) - 1) >> (6 - g.flog);
}

struct OutArgs {
    uint32_t *dist;           // [C][n]
    uint64_t *masks;          // [C][P][n][WC]
    int32_t *status;          // [C]
    int32_t R;                // center-relative: the offset radius; min-relative: the diameter d
    int32_t minrel;           // 1: min-relative encode (P = d + 1), 0: center-relative (P = 2R + 1)
    const int32_t *center;    // [C] each cluster's center vertex (the encode's radius check)
};

// Center-relative with R = 1: the encode needs no earlier round from dist.
// A source's offset at any vertex is bounded by its distance to the center
// (Section 3.1, Fact), so an offset outside [-1, 1] anywhere implies one at
// the center itself, and the radius check is made there: bits reaching the
// center after round 1 (finalize adds the sources that never reach it).
__device__ __forceinline__ bool dist_free(const OutArgs &o) { return o.R == 1 && !o.minrel; }

__host__ __device__ inline int64_t planes_of(const OutArgs &o)
{
    return o.minrel ? (int64_t)o.R + 1 : 2 * (int64_t)o.R + 1;
}

__device__ __forceinline__ uint64_t *cur_buf(const SlotArgs &s, int round) { return (round & 1) ? s.B : s.A; }
__device__ __forceinline__ uint64_t *nxt_buf(const SlotArgs &s, int round) { return (round & 1) ? s.A : s.B; }
__device__ __forceinline__ int64_t *q_buf(const SlotArgs &s, int round)
{
    const int r = round % 3;
    return r == 0 ? s.q0 : (r == 1 ? s.q1 : s.q2);
}
__device__ __forceinline__ uint64_t *bits_buf(const SlotArgs &s, int r3)
{
    return r3 == 0 ? s.bits0 : (r3 == 1 ? s.bits1 : s.bits2);
}
__device__ __forceinline__ unsigned long long *ctr_buf(const SlotArgs &s, int round) { return s.ctr + 4 * (round & 3); }

__device__ __forceinline__ unsigned long long or64(uint64_t *p, uint64_t v)
{
    return atomicOr(reinterpret_cast<unsigned long long *>(p), static_cast<unsigned long long>(v));
}

template <int W>
__device__ __forceinline__ void load_words(const uint64_t *p, uint64_t (&x)[W])
{
    if constexpr (W % 2 == 1) {
#pragma unroll
        for (int w = 0; w < W; w++) x[w] = p[w];
    } else {
#pragma unroll
        for (int w = 0; w < W; w += 2) {
            ulonglong2 t = *reinterpret_cast<const ulonglong2 *>(p + w);
            x[w] = t.x;
            x[w + 1] = t.y;
        }
    }
}

template <int W>
__device__ __forceinline__ void store_words(uint64_t *p, const uint64_t (&x)[W])
{
    if constexpr (W % 2 == 1) {
#pragma unroll
        for (int w = 0; w < W; w++) p[w] = x[w];
    } else {
#pragma unroll
        for (int w = 0; w < W; w += 2) {
            ulonglong2 t;
            t.x = x[w];
            t.y = x[w + 1];
            *reinterpret_cast<ulonglong2 *>(p + w) = t;
        }
    }
}

__device__ __forceinline__ int pieces_of(int deg) { return deg > PIECE ? (deg + PIECE - 1) / PIECE : 1; }

// Queue entries per push block: about PUSH_BLOCK_ARCS arcs per block, so that
// a frontier of a few hub vertices (pieces of PIECE arcs) still spreads over
// many blocks; a power of two in [8, BLOCK].
constexpr int64_t PUSH_BLOCK_ARCS = 4096;
__host__ __device__ inline int32_t push_entries_per_block(int64_t pieces, int64_t degsum)
{
    if (pieces <= 0 || degsum <= 0) return BLOCK;
    int64_t want = PUSH_BLOCK_ARCS * pieces / degsum;
    int32_t e = BLOCK;
    while (e > 8 && e > want) e >>= 1;
    return e;
}

// ---------------------------------------------------------------------------
// Output encoding for one cluster at vertex v, round i (the vertex phase's
// "S_u[i - Delta_u] <- S_new" of Algorithm "Cluster-BFS search from S",
// re-based on the center).  prev = cluster bits seen before round i, nw =
// bits new in round i.  The center is bit 0 of the cluster's first word.
//   - center already seen (its round d is in dist): new bits sit at offset i-d.
//   - center new now: d = i; bits seen earlier sit at negative offsets.  For
//     R = 1 all of them are at -1 and the still-missing bits must arrive at
//     +1, so all three planes are written now; for R >= 2 the pre-center
//     rounds were stashed in planes 0..R-1 (min-relative) and are shifted
//     into place, and the positive planes are cleared for later rounds.
//   - center not yet seen: dist holds the first round Delta_c any bit of the
//     cluster arrived; for R >= 2 the bits are stashed at plane i - Delta_c.
// Any bit whose offset leaves [-R, R] marks the cluster CBFS_E_RADIUS.  For
// R = 1 (dist_free) no earlier round is needed: the check is made at the
// center (bits after round 1) and where bits come while earlier ones wait for
// the center; dist is written once, when the center arrives.
// dold is dist[c][v] as it stood before this call (the caller loads it with
// the state words; only this call writes it in this round; 0 and unused when
// dist_free).
// ---------------------------------------------------------------------------
template <int WC>
__device__ __forceinline__ void emit_cluster(const OutArgs &o, int64_t n, int32_t c, int32_t v,
                                             int32_t i, const uint64_t *prev, const uint64_t *nw,
                                             const uint64_t *full, uint32_t dold)
{
    uint64_t any_new = 0, any_prev = 0;
#pragma unroll
    for (int x = 0; x < WC; x++) {
        any_new |= nw[x];
        any_prev |= prev[x];
    }
    if (!any_new) return;
    const int32_t R = o.R;
    const int64_t P = planes_of(o);
    uint32_t *dslot = o.dist + (size_t)c * (size_t)n + (size_t)v;
    auto plane = [&](int64_t p) { return o.masks + (((size_t)c * P + (size_t)p) * (size_t)n + (size_t)v) * WC; };
    auto put = [&](int64_t p, const uint64_t *val) {
        uint64_t *dst = plane(p);
#pragma unroll
        for (int x = 0; x < WC; x++) dst[x] = val[x];
    };
    auto put_zero = [&](int64_t p) {
        uint64_t *dst = plane(p);
#pragma unroll
        for (int x = 0; x < WC; x++) dst[x] = 0;
    };
    auto violate = [&]() { atomicExch(o.status + c, E_RADIUS); };

    if (o.minrel) {
        // the paper's own form (Section 3.1): Delta_v is the round the first
        // bit arrives, and the bits of round i go to subset i - Delta_v <= d
        if (!any_prev) {
            *dslot = (uint32_t)i;
            put(0, nw);
            for (int32_t p = 1; p <= R; p++) put_zero(p);
        } else {
            const int32_t j = i - (int32_t)dold;
            if (j > R) violate();
            else put(j, nw);
        }
        return;
    }
    if (prev[0] & 1ull) {
        if (R == 1) {
            // the rest arrives one round after the center (plane 2 holds it)
            if (i > 1 && v == o.center[c]) violate();
            return;
        }
        const int32_t k = i - (int32_t)dold;
        if (k < 1 || k > R) {
            violate();
        } else if (R > 1) {
            put(R + k, nw);
        }
        return;
    }
    if (nw[0] & 1ull) {
        const int32_t jc = any_prev && R != 1 ? i - (int32_t)dold : 0;
        if (jc < 0 || jc > R) {
            violate();
            return;
        }
        *dslot = (uint32_t)i;
        if (R == 1) {
            uint64_t rest[WC];
#pragma unroll
            for (int x = 0; x < WC; x++) rest[x] = full[x] & ~(prev[x] | nw[x]);
            put(0, prev);
            put(1, nw);
            put(2, rest);
        } else {
            const int32_t s = R - jc;
            for (int32_t j = jc - 1; j >= 0; j--) {
                uint64_t tmp[WC];
                const uint64_t *src = plane(j);
#pragma unroll
                for (int x = 0; x < WC; x++) tmp[x] = src[x];
                put(j + s, tmp);
            }
            for (int32_t p = 0; p < s; p++) put_zero(p);
            put(R, nw);
            for (int32_t p = R + 1; p <= 2 * R; p++) put_zero(p);
        }
        return;
    }
    // center not reached yet
    if (R == 1) {
        // bits seen in an earlier round are then two or more rounds ahead
        // of the center; the first round itself is not needed
        if (any_prev) violate();
        return;
    }
    int32_t j = 0;
    if (!any_prev) {
        *dslot = (uint32_t)i;
    } else {
        j = i - (int32_t)dold;
    }
    if (j < 0 || j >= R) {
        violate();
        return;
    }
    if (R > 1) {
        put(j, nw);
        if (j == 0)
            for (int32_t p = 1; p < R; p++) put_zero(p);
    }
}

// Vertex phase for u in F_i (lines computing S_new, Delta_u, the subset write
// and the seen update) for cluster j of the group: new = Seen_i(u) \
// Seen_{i-1}(u) from cur and seen.  With NXT_OR, nxt(u) receives the new bits
// by atomic OR so that nxt(u) covers Seen_i(u) by the end of the round;
// without it the caller stores nxt(u) itself (it owns u's row in this round).
// With active false the words are still read (so a caller can request them
// before it knows u is in F_i) and nothing is written.
//
// j is a unit of the group (units_of): a cluster of WC words, or one word
// holding several clusters in fields; the unit's thread owns its words, so the
// seen update stays one plain store.
template <int W, int WC, bool NXT_OR>
__device__ __forceinline__ void vertex_phase_cluster(const SlotArgs &s, const GroupDesc &g, const OutArgs &o,
                                                     int64_t n, int32_t round, int32_t u, int32_t j,
                                                     bool active = true, bool copy_nxt = false)
{
    const uint64_t *cp = cur_buf(s, round) + (size_t)u * W + j * WC;
    uint64_t *sp = s.seen + (size_t)u * W + j * WC;
    const bool fields = WC == 1 && g.flog < 6;
    // a whole-word cluster's distance word is requested with the state words,
    // so the encode does not wait for a second round trip
    const uint32_t dold = fields || dist_free(o) ? 0u : o.dist[(size_t)(g.c0 + j) * (size_t)n + (size_t)u];
    uint64_t cu[WC], sv[WC], nw[WC];
    uint64_t any = 0;
    const uint64_t am = active ? ~0ull : 0ull;  // a value mask, so the loads stay ahead of the test
#pragma unroll
    for (int x = 0; x < WC; x++) {
        cu[x] = cp[x];
        sv[x] = sp[x];
        nw[x] = cu[x] & ~sv[x] & am;
        any |= nw[x];
    }
    if (copy_nxt) {
        // nxt(u) = Seen_i(u) for a row of F_i whose arc phase found nothing new
        uint64_t *np = nxt_buf(s, round) + (size_t)u * W + j * WC;
#pragma unroll
        for (int x = 0; x < WC; x++) np[x] = cu[x];
    }
    if (!any) return;
#pragma unroll
    for (int x = 0; x < WC; x++) {
        sp[x] = cu[x];
        if constexpr (NXT_OR)
            if (nw[x]) or64(nxt_buf(s, round) + (size_t)u * W + j * WC + x, nw[x]);
    }
    if (!fields) {
        emit_cluster<WC>(o, n, g.c0 + j, u, round, sv, nw, g.full + j * WC, dold);
        return;
    }
    const int32_t F = fields_per_word(g);
    const uint64_t fm = field_mask(g);
    for (int32_t f = 0; f < F; f++) {
        const int32_t c = g.c0 + j * F + f;
        if (c >= g.c0 + g.nc) break;
        const int sh = f << g.flog;
        const uint64_t nf = (nw[0] >> sh) & fm;
        if (!nf) continue;
        const uint64_t pf = (sv[0] >> sh) & fm, ff = (g.full[j] >> sh) & fm;
        emit_cluster<1>(o, n, c, u, round, &pf, &nf, &ff,
                        dist_free(o) ? 0u : o.dist[(size_t)c * (size_t)n + (size_t)u]);
    }
}

// The vertex phase of u for every cluster of the group, one after another.
template <int W, int WC, bool NXT_OR = true>
__device__ __forceinline__ void vertex_phase(const SlotArgs &s, const GroupDesc &g, const OutArgs &o,
                                             int64_t n, int32_t round, int32_t u)
{
    const int32_t units = units_of<WC>(g);
#pragma unroll 1
    for (int j = 0; j < W / WC; j++) {
        if (j >= units) break;
        vertex_phase_cluster<W, WC, NXT_OR>(s, g, o, n, round, u, j);
    }
}

// Exclusive block scan of one int per thread; *total receives the sum.
__device__ __forceinline__ int block_exclusive_scan(int x, int *tmp /*[WAVES+1]*/, int *total)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int v = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int y = __shfl_up(v, d, 64);
        if (lane >= d) v += y;
    }
    if (lane == 63) tmp[wid] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int w = 0; w < WAVES; w++) {
            int t = tmp[w];
            tmp[w] = acc;
            acc += t;
        }
        tmp[WAVES] = acc;
    }
    __syncthreads();
    *total = tmp[WAVES];
    const int r = v - x + tmp[wid];
    __syncthreads();
    return r;
}

// Exclusive block max-scan of one non-negative int per thread (0 for the
// first thread).
__device__ __forceinline__ int block_exclusive_max(int x, int *tmp /*[WAVES+1]*/)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int v = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int y = __shfl_up(v, d, 64);
        if (lane >= d) v = v > y ? v : y;
    }
    if (lane == 63) tmp[wid] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int w = 0; w < WAVES; w++) {
            int t = tmp[w];
            tmp[w] = acc;
            acc = acc > t ? acc : t;
        }
    }
    __syncthreads();
    int prev = __shfl_up(v, 1, 64);
    if (lane == 0) prev = 0;
    const int r = prev > tmp[wid] ? prev : tmp[wid];
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------------------
// LDS-staged frontier queue: claimed vertices are collected in LDS and
// appended to the global queue with one atomic per flush, expanded into their
// PIECE-sized work items (offsets from a block scan at flush time).
// ---------------------------------------------------------------------------
// Queue entries of vertices with many pieces (hubs) are written by the whole
// block rather than by the one thread that holds the vertex: such a vertex
// goes to this LDS list (BIG_CAP at most per flush, the rest its thread
// writes), and big_write spreads its pieces over the threads.
constexpr int BIG_PIECES = 8;  // more pieces than this: written by the block
constexpr int BIG_CAP = 32;
struct BigList {
    int32_t v[BIG_CAP], pc[BIG_CAP];
    long long at[BIG_CAP];
    int n;
};

// Entries (p << 32 | v), p < pc, at q[at ..]: by this thread, or listed for
// the block.  big.n must have been zeroed before a barrier that precedes this.
__device__ __forceinline__ void put_pieces(BigList &big, int64_t *q, long long at, int32_t v, int pc)
{
    if (pc > BIG_PIECES) {
        const int slot = atomicAdd(&big.n, 1);
        if (slot < BIG_CAP) {
            big.v[slot] = v;
            big.pc[slot] = pc;
            big.at[slot] = at;
            return;
        }
    }
    for (int p = 0; p < pc; p++) q[at + p] = ((int64_t)p << 32) | (int64_t)(uint32_t)v;
}

// Block-uniform: the listed vertices' entries, every thread taking a share;
// leaves the list empty (the trailing barrier orders the reset before reuse).
__device__ __forceinline__ void big_write(BigList &big, int64_t *q)
{
    __syncthreads();
    const int nb = big.n < BIG_CAP ? big.n : BIG_CAP;
    for (int i = 0; i < nb; i++) {
        const int32_t v = big.v[i];
        const long long at = big.at[i];
        for (int p = threadIdx.x; p < big.pc[i]; p += BLOCK) q[at + p] = ((int64_t)p << 32) | (int64_t)(uint32_t)v;
    }
    __syncthreads();
    if (threadIdx.x == 0) big.n = 0;
    __syncthreads();
}

template <int CAP>
struct Stager {
    int32_t v[CAP];
    int32_t count;
    unsigned long long degsum;
    long long base;
    int tmp[WAVES + 1];
    BigList big;
};

template <int CAP>
__device__ __forceinline__ void stager_init(Stager<CAP> &st)
{
    if (threadIdx.x == 0) {
        st.count = 0;
        st.degsum = 0;
        st.big.n = 0;
    }
}

template <int CAP>
__device__ __forceinline__ void stager_push(Stager<CAP> &st, int32_t v, int32_t deg)
{
    const int slot = atomicAdd(&st.count, 1);
    st.v[slot] = v;
    atomicAdd(&st.degsum, (unsigned long long)deg);
}

// Block-uniform call (every thread).  With sort, the staged vertices are
// first ordered by id (bitonic sort in LDS), so a later chunk of the queue
// covers nearby vertices whose state, distance and plane words share cache
// lines (worth it for low-degree frontiers, where those words dominate).
template <int CAP>
__device__ __forceinline__ void stager_flush(Stager<CAP> &st, const int32_t *row_ptr, int64_t *q_next,
                                             unsigned long long *ctr_next, bool sort = false)
{
    static_assert((CAP & (CAP - 1)) == 0, "the stager sorts a power-of-two array");
    __syncthreads();
    const int cnt = st.count;
    if (cnt == 0) return;
    if (sort) {
        int np2 = 1;
        while (np2 < cnt) np2 <<= 1;
        for (int k = cnt + threadIdx.x; k < np2; k += BLOCK) st.v[k] = INT32_MAX;
        __syncthreads();
        for (int k = 2; k <= np2; k <<= 1)
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int i = threadIdx.x; i < np2; i += BLOCK) {
                    const int ixj = i ^ j;
                    if (ixj > i) {
                        const int32_t x = st.v[i], y = st.v[ixj];
                        if (((i & k) == 0) ? (x > y) : (x < y)) {
                            st.v[i] = y;
                            st.v[ixj] = x;
                        }
                    }
                }
                __syncthreads();
            }
    }
    const int per = (cnt + BLOCK - 1) / BLOCK;
    const int lo = threadIdx.x * per < cnt ? threadIdx.x * per : cnt;
    const int hi = lo + per < cnt ? lo + per : cnt;
    int mine = 0;
    for (int k = lo; k < hi; k++) {
        const int32_t v = st.v[k];
        mine += pieces_of(row_ptr[v + 1] - row_ptr[v]);
    }
    int total;
    const int off = block_exclusive_scan(mine, st.tmp, &total);
    if (threadIdx.x == 0) {
        st.base = (long long)atomicAdd(ctr_next + 0, (unsigned long long)total);
        atomicAdd(ctr_next + 1, (unsigned long long)cnt);
        atomicAdd(ctr_next + 2, st.degsum);
    }
    __syncthreads();
    long long at = st.base + off;
    for (int k = lo; k < hi; k++) {
        const int32_t v = st.v[k];
        const int pc = pieces_of(row_ptr[v + 1] - row_ptr[v]);
        put_pieces(st.big, q_next, at, v, pc);
        at += pc;
    }
    big_write(st.big, q_next);
    if (threadIdx.x == 0) {
        st.count = 0;
        st.degsum = 0;
    }
    __syncthreads();
}

// Claim v for F_{i+1} (the compare-and-swap on r[v] of Algorithm "Cluster-BFS
// search from S", here an atomic OR on a membership bitmap: first setter
// wins).  Bits only go from 0 to 1 within a round, so a plain load that
// already shows v's bit saves the atomic.
template <int CAP>
__device__ __forceinline__ void claim(Stager<CAP> &st, uint64_t *bits_next, int32_t v, int32_t deg)
{
    const unsigned long long bit = 1ull << (v & 63);
    unsigned long long *w = reinterpret_cast<unsigned long long *>(bits_next + (v >> 6));
    if (*w & bit) return;
    const unsigned long long old = atomicOr(w, bit);
    if (!(old & bit)) stager_push(st, v, deg);
}

// Contribute x = Seen_i(u) \ Seen_i(v), non-empty, to v: OR it into nxt(v)
// (atomics whose old value is not needed) and claim v.  v joins F_{i+1}
// whoever's OR lands first: x holds bits v did not have in round i.
template <int W, int CAP>
__device__ __forceinline__ void contribute(Stager<CAP> &st, uint64_t *nxt, uint64_t *bits_next,
                                          const int32_t *row_ptr, int32_t v, const uint64_t (&x)[W])
{
    uint64_t *p = nxt + (size_t)v * W;
#pragma unroll
    for (int w = 0; w < W; w++)
        if (x[w]) or64(p + w, x[w]);
    claim(st, bits_next, v, row_ptr[v + 1] - row_ptr[v]);
}

}  // namespace cbfs
