// Round work of the Cluster-BFS level loop as block-level device functions,
// shared by the one-launch-per-round kernels and the persistent kernel.
//
// Every function below that contains a barrier is block-uniform: all threads
// of the block call it with the same arguments.
#pragma once
#include "cbfs_device.h"

namespace cbfs {

template <int W>
struct PushSmem {
    int scan[BLOCK + 1];
    int32_t estart[BLOCK];
    uint64_t cu[BLOCK * W];
    int tmp[WAVES + 1];
    Stager<STAGE_CAP> st;
};

// Lanes per vertex in the pull: a state of W >= 16 words is split over
// H = W / 8 lanes of 8 words each (register pressure), the lanes of a vertex
// lying 64 / H apart in the wave (one half-wave per half for H = 2).
template <int W>
constexpr int pull_split()
{
    return W >= 16 ? W / 8 : 1;
}

template <int W>
struct PullSmem {
    uint16_t rend[TILE_ITEMS + 2];           // row_end of the tile's rows minus tile_edge (clamped)
    uint64_t claimed[PULL_CLAIM_WORDS];      // F_{i+1} bits of the tile's rows, from word tile_row >> 6
    BigList big;                             // claimed hub rows whose queue entries the block writes
    uint64_t fin[PULL_ROW_WORDS];            // rows whose set is complete (bit: row - tile_row)
    uint64_t stored[PULL_ROW_WORDS];         // local rows whose nxt the arc phase stored
    int tmp[WAVES + 1];
    unsigned long long degsum;
    long long base;
    union {
        uint64_t part[BLOCK / pull_split<W>()][W];  // walk: partial sets of rows shared by walkers, by first walker
        struct {
            uint16_t arow[TILE_ITEMS];       // row of each of the tile's arcs, minus tile_row
            uint64_t out_acc[WAVES][W];      // a wave's share of the row still open at its range end
            uint64_t pend_acc[WAVES][W];     // a wave's share of a row it closes that began earlier
            uint64_t cacc[WAVES][W];         // the OR so far of the row a wave carries between steps
            int32_t out_row[WAVES], pend_row[WAVES];
        } wv;                                // wave form
    };
};

// The wave form's arc -> row map: per arc of the tile its row (minus the
// tile's first row) and three flags.
constexpr int AROW_ROW = 0x1fff;
constexpr int AROW_LAST = 0x2000;   // the row's last arc in the tile
constexpr int AROW_FIRST = 0x4000;  // the row's first arc
constexpr int AROW_DONE = 0x8000;   // the row's set was complete when the round began
static_assert(TILE_ITEMS <= AROW_ROW, "a tile's row offsets fit the arc -> row map's row field");

// lanes 0..al of a word of lane bits
__device__ __forceinline__ uint64_t lane_mask_upto(int al) { return al >= 63 ? ~0ull : (2ull << al) - 1ull; }

template <int W>
union RoundSmem {
    PushSmem<W> push;
    PullSmem<W> pull;
};

// Init (Algorithm "Cluster-BFS search from S", initialization): clear one
// group slot; the group's cluster statuses to CBFS_OK.  Grid-stride part
// [tid, .., stride).
template <int W>
__device__ __forceinline__ void init_part(const SlotArgs &s, int64_t n, const GroupDesc &g, const OutArgs &o,
                                          int64_t tid, int64_t stride)
{
    // 16-byte stores (the arrays start 256-byte aligned in the workspace)
    const int64_t words = n * W;
    const ulonglong2 z = make_ulonglong2(0ull, 0ull);
    for (int64_t k = tid; k < (words >> 1); k += stride) {
        reinterpret_cast<ulonglong2 *>(s.A)[k] = z;
        reinterpret_cast<ulonglong2 *>(s.B)[k] = z;
        reinterpret_cast<ulonglong2 *>(s.seen)[k] = z;
    }
    if ((words & 1) && tid == 0) {
        s.A[words - 1] = 0;
        s.B[words - 1] = 0;
        s.seen[words - 1] = 0;
    }
    for (int64_t k = tid; k < s.nwords; k += stride) {
        s.bits0[k] = 0;
        s.bits1[k] = 0;
        s.bits2[k] = 0;
    }
    if (tid < 16) s.ctr[tid] = 0;
    if (tid < g.nc) o.status[g.c0 + tid] = 0;
}

// Clear the bitmap of F_{i-1} (bits[(i+2)%3]) densely and the counters of
// round i+2 (they last served round i-2).
__device__ __forceinline__ void clear_ahead_part(const SlotArgs &s, int32_t round, int64_t tid, int64_t stride)
{
    uint64_t *clr = bits_buf(s, (round + 2) % 3);
    for (int64_t k = tid; k < s.nwords; k += stride) clr[k] = 0;
    if (tid < 4) ctr_buf(s, round + 2)[tid] = 0;
}

// One clear item of round i for a slot.  Sparse: zero the bitmap words of the
// F_{i-1} entries [item*BLOCK, (item+1)*BLOCK) of queue[(i+2)%3] (a word of
// that bitmap only holds F_{i-1} bits, so the whole word is zeroed).  Dense:
// zero words [item*CLEAR_WORDS, (item+1)*CLEAR_WORDS) of the bitmap.  Item 0
// also clears the counters of round i+2.
constexpr int CLEAR_WORDS = BLOCK * 16;

__device__ __forceinline__ void clear_item(const SlotArgs &s, int32_t round, bool sparse, int64_t nprev, int64_t item)
{
    uint64_t *clr = bits_buf(s, (round + 2) % 3);
    if (sparse) {
        const int64_t idx = item * BLOCK + threadIdx.x;
        if (idx < nprev) {
            const int32_t v = (int32_t)(q_buf(s, round + 2)[idx] & 0xffffffff);
            clr[v >> 6] = 0;
        }
    } else {
        const int64_t hi = (item + 1) * CLEAR_WORDS < s.nwords ? (item + 1) * CLEAR_WORDS : s.nwords;
        for (int64_t k = item * CLEAR_WORDS + threadIdx.x; k < hi; k += BLOCK) clr[k] = 0;
    }
    if (item == 0 && threadIdx.x < 4) ctr_buf(s, round + 2)[threadIdx.x] = 0;
}

// Seed (one block): bit i of cluster j at its source s_i, i.e. Seen_0; and
// F_0 = the sources.  sources/cluster_ptr are the batch arrays on the device.
template <int W, int WC>
__device__ void seed_block(Stager<STAGE_CAP> &st, const SlotArgs &s, const GraphArgs &gr, const GroupDesc &g,
                           const int32_t *sources, const int32_t *cluster_ptr, int32_t part = 0, int32_t parts = 1,
                           int32_t per = BLOCK)
{
    __syncthreads();
    stager_init(st);
    __syncthreads();
    const int32_t first = cluster_ptr[g.c0];
    const int32_t total = cluster_ptr[g.c0 + g.nc] - first;
    // block `part` of `parts` takes every parts-th run of `per` sources (the
    // whole block then writes the pieces of the hubs among them); a source in
    // several clusters is claimed, and queued, once: by the bitmap
    for (int32_t k = part * per + (int32_t)threadIdx.x; (int32_t)threadIdx.x < per && k < total; k += parts * per) {
        const int32_t idx = first + k;
        // the cluster j holding source idx (clusters are non-empty, so the
        // group's cluster_ptr entries increase strictly)
        int32_t j = 0, jh = g.nc - 1;
        while (j < jh) {
            const int32_t mid = (j + jh + 1) >> 1;
            if (cluster_ptr[g.c0 + mid] <= idx) j = mid;
            else jh = mid - 1;
        }
        const int32_t i = idx - cluster_ptr[g.c0 + j];
        const int32_t v = sources[idx];
        if (WC == 1 && g.flog < 6) {  // cluster j in field j % F of word j / F
            const int32_t F = fields_per_word(g);
            or64(s.A + (size_t)v * W + j / F, 1ull << (((j % F) << g.flog) + i));
        } else {
            or64(s.A + (size_t)v * W + j * WC + (i >> 6), 1ull << (i & 63));
        }
        claim(st, s.bits0, v, gr.row_ptr[v + 1] - gr.row_ptr[v]);
    }
    stager_flush(st, gr.row_ptr, s.q0, s.ctr + 0);
}

// ---------------------------------------------------------------------------
// Round i, push direction (EdgeMap-Sparse), one chunk of epb <= BLOCK queue
// entries (pieces of <= PIECE arcs; epb from push_entries_per_block, so a
// chunk holds about PUSH_BLOCK_ARCS arcs): the vertex phase for first pieces, then the
// chunk's arcs spread evenly over the block (block scan + binary search of
// each arc's owner), or, when every entry has at most a few arcs, each thread
// walks its own entry's arcs.  Per arc (u, v): x = Seen_i(u) \ Seen_i(v); if not empty,
// 64-bit atomic OR into nxt(v) and claim v (the Fetch_And_Or and
// compare_and_swap of the paper's edge phase).
// ---------------------------------------------------------------------------
template <int W, int WC>
__device__ void push_chunk(PushSmem<W> &sm, const SlotArgs &s, const GraphArgs &gr, const GroupDesc &g,
                           const OutArgs &o, int32_t round, int64_t nq, int64_t chunk, int32_t epb)
{
    const int64_t first = chunk * epb;
    if (first >= nq) return;  // block-uniform
    __syncthreads();
    stager_init(sm.st);
    const uint64_t *cur = cur_buf(s, round);
    uint64_t *nxt = nxt_buf(s, round);
    uint64_t *bits_next = bits_buf(s, (round + 1) % 3);
    int64_t *q_next = q_buf(s, round + 1);
    unsigned long long *ctr_next = ctr_buf(s, round + 1);

    int cnt = 0;
    int32_t lo = 0;
    uint64_t cu[W];
#pragma unroll
    for (int w = 0; w < W; w++) cu[w] = 0;
    const int64_t idx = first + threadIdx.x;
    if ((int32_t)threadIdx.x < epb && idx < nq) {
        const int64_t e = q_buf(s, round)[idx];
        const int32_t u = (int32_t)(e & 0xffffffff);
        const int32_t p = (int32_t)(e >> 32);
        const int32_t rs = gr.row_ptr[u], re = gr.row_ptr[u + 1];
        lo = rs + p * PIECE;
        const int32_t hi = re < lo + PIECE ? re : lo + PIECE;
        cnt = hi > lo ? hi - lo : 0;
        load_words<W>(cur + (size_t)u * W, cu);
        if (p == 0) vertex_phase<W, WC>(s, g, o, gr.n, round, u);
    }
    // every entry short (a low-degree frontier): each thread pushes its own
    // arcs, DB at a time, with no block scan or owner search
    constexpr int DB = push_direct_batch<W>();
    if (__syncthreads_and(cnt <= 2 * DB)) {
        const int iters = __syncthreads_or(cnt > DB) ? 2 : 1;
        for (int it = 0; it < iters; it++) {
            const int32_t j0 = it * DB;
            int32_t v[DB];
#pragma unroll
            for (int j = 0; j < DB; j++) v[j] = j0 + j < cnt ? gr.col[lo + j0 + j] : -1;
            uint64_t cv[DB][W];
#pragma unroll
            for (int j = 0; j < DB; j++) load_words<W>(cur + (size_t)(v[j] >= 0 ? v[j] : 0) * W, cv[j]);
#pragma unroll
            for (int j = 0; j < DB; j++) {
                if (v[j] < 0) continue;
                uint64_t x[W];
                bool any = false;
#pragma unroll
                for (int w = 0; w < W; w++) {
                    x[w] = cu[w] & ~cv[j][w];
                    any |= x[w] != 0;
                }
                if (any) contribute<W>(sm.st, nxt, bits_next, gr.row_ptr, v[j], x);
            }
            // at most BLOCK * DB <= STAGE_CAP claims per pass
            stager_flush(sm.st, gr.row_ptr, q_next, ctr_next, true);
        }
        return;
    }
    if ((int32_t)threadIdx.x < epb && idx < nq) {
        sm.estart[threadIdx.x] = lo;
#pragma unroll
        for (int w = 0; w < W; w++) sm.cu[threadIdx.x * W + w] = cu[w];
    }
    int total;
    const int off = block_exclusive_scan(cnt, sm.tmp, &total);
    sm.scan[threadIdx.x] = off;
    if (threadIdx.x == 0) sm.scan[BLOCK] = total;
    __syncthreads();

    for (int base = 0; base < total; base += BLOCK) {
        const int e = base + threadIdx.x;
        if (e < total) {
            // owner: last j with scan[j] <= e (entries with no arcs share offsets)
            int lo = 0, hi = BLOCK;
            while (hi - lo > 1) {
                int mid = (lo + hi) >> 1;
                if (sm.scan[mid] <= e) lo = mid;
                else hi = mid;
            }
            const int32_t v = gr.col[sm.estart[lo] + (e - sm.scan[lo])];
            uint64_t cv[W], x[W];
            load_words<W>(cur + (size_t)v * W, cv);
            bool any = false;
#pragma unroll
            for (int w = 0; w < W; w++) {
                x[w] = sm.cu[lo * W + w] & ~cv[w];
                any |= x[w] != 0;
            }
            if (any) contribute<W>(sm.st, nxt, bits_next, gr.row_ptr, v, x);
        }
        __syncthreads();
        if (sm.st.count > STAGE_CAP - BLOCK) stager_flush(sm.st, gr.row_ptr, q_next, ctr_next);
    }
    stager_flush(sm.st, gr.row_ptr, q_next, ctr_next);
}

// ---------------------------------------------------------------------------
// Round i, push direction, for a frontier of at most HUB_MAX vertices whose
// arcs are many (on skewed graphs the sources of round 0 are hubs whose
// neighbour lists overlap).  Each block owns HUB_RANGE consecutive target
// vertices.  For every frontier vertex u it reads the slice of u's sorted
// neighbour list inside its range (from the table of hub_bounds_block, built
// by a pass over the frontier's arcs just before), ORs Seen_i(u) into
// LDS sets of its targets, and then writes nxt(v) once per target with a plain
// store: the global set-union atomics of the arc-parallel push become LDS
// atomics, and a target hit by many frontier vertices is written once.  A
// target's claim is a bit of a frontier-bitmap word the block owns; the
// F_{i+1} queue is built from the bitmap afterwards (bits_to_queue_block), so
// the many short blocks do not contend for the queue counters.  The vertex
// phase of the frontier vertices in the range runs here as well.
// hubs[0 .. hubs[HUB_MAX]) lists the frontier's vertices.
// ---------------------------------------------------------------------------
static_assert(WAVES * 4 + 4 <= 64, "the merges after a wave-form pass run in wave 0");
static_assert(HUB_RANGE == BLOCK && HUB_MAX <= BLOCK, "one owned target and one frontier vertex per thread");
static_assert(HUB_RANGE % 64 == 0, "a block owns whole frontier-bitmap words");

// Slice starts for the range-owned push.  For frontier vertex h (hubs[h])
// and each owned range b up to the range of its last arc, bounds[h * stride +
// b] is the first arc of h's sorted neighbour list whose target is >= b *
// HUB_RANGE.  One thread per arc of the concatenated lists: an arc whose range
// differs from its predecessor's writes the entries of the ranges from the
// one after the predecessor's up to its own (every entry has one writer); the
// push takes ranges past the last arc as starting at the list's end.  Blocks
// stride over chunks of HB_CHUNK arcs, so any grid covers every arc.
struct HubBoundsSmem {
    int32_t rs[HUB_MAX], pre[HUB_MAX + 1];
    int tmp[WAVES + 1];
};

__device__ void hub_bounds_block(HubBoundsSmem &sm, const GraphArgs &gr, const int32_t *hubs, int32_t *bounds,
                                 int64_t stride)
{
    const int32_t nh = hubs[HUB_MAX] < HUB_MAX ? hubs[HUB_MAX] : HUB_MAX;
    int32_t d = 0;
    if ((int)threadIdx.x < nh) {
        const int32_t u = hubs[threadIdx.x];
        const int32_t rs = gr.row_ptr[u];
        d = gr.row_ptr[u + 1] - rs;
        sm.rs[threadIdx.x] = rs;
    }
    int total;
    const int off = block_exclusive_scan(d, sm.tmp, &total);
    if ((int)threadIdx.x < nh) sm.pre[threadIdx.x] = off;
    __syncthreads();
    for (int64_t c0 = (int64_t)blockIdx.x * HB_CHUNK; c0 < total; c0 += (int64_t)gridDim.x * HB_CHUNK) {
        const int32_t c1 = (int32_t)(c0 + HB_CHUNK < total ? c0 + HB_CHUNK : total);
        for (int32_t q = (int32_t)c0 + (int32_t)threadIdx.x; q < c1; q += BLOCK) {
            // the list holding arc q: the last h with pre[h] <= q (an empty
            // list shares its start with the next one, which wins)
            int lo = 0, hi = nh;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (sm.pre[mid] <= q) lo = mid;
                else hi = mid;
            }
            const int32_t e = sm.rs[lo] + (q - sm.pre[lo]);
            const int32_t r = gr.col[e] >> HUB_RANGE_LOG;
            const int32_t prev = q == sm.pre[lo] ? -1 : (gr.col[e - 1] >> HUB_RANGE_LOG);
            int32_t *bh = bounds + (size_t)lo * (size_t)stride;
            for (int32_t b = prev + 1; b <= r; b++) bh[b] = e;
        }
    }
}

template <int W>
struct HubSmem {
    uint64_t acc[HUB_RANGE * W];  // OR of the frontier sets arriving at each owned target
    int32_t hub[HUB_MAX], hlo[HUB_MAX], hoff[HUB_MAX + 1];
    int tmp[WAVES + 1];
};

template <int W, int WC>
__device__ void push_hub_block(HubSmem<W> &sm, const SlotArgs &s, const GraphArgs &gr, const GroupDesc &g,
                               const OutArgs &o, int32_t round, const int32_t *hubs, const int32_t *bounds,
                               int64_t stride, int64_t b)
{
    const int64_t v0 = b * HUB_RANGE;
    if (v0 >= gr.n) return;  // block-uniform
    const int32_t v1 = (int32_t)(v0 + HUB_RANGE < gr.n ? v0 + HUB_RANGE : gr.n);
    const uint64_t *cur = cur_buf(s, round);
    uint64_t *nxt = nxt_buf(s, round);
    const uint64_t *bits_cur = bits_buf(s, round % 3);
    uint64_t *bits_next = bits_buf(s, (round + 1) % 3);
    const int32_t nh = hubs[HUB_MAX] < HUB_MAX ? hubs[HUB_MAX] : HUB_MAX;
    for (int k = threadIdx.x; k < HUB_RANGE * W; k += BLOCK) sm.acc[k] = 0;
    // the slice of each frontier vertex's neighbour list inside [v0, v1)
    int len = 0;
    if ((int)threadIdx.x < nh) {
        const int32_t u = hubs[threadIdx.x];
        const int32_t rs = gr.row_ptr[u], re = gr.row_ptr[u + 1];
        // the slice [first arc >= v0, first arc >= v1) from the bounds table
        // (hub_bounds_block); ranges past the list's last arc have no entry
        // there and start at re
        const int32_t last = re > rs ? (gr.col[re - 1] >> HUB_RANGE_LOG) : -1;
        const int32_t *bh = bounds + (size_t)threadIdx.x * (size_t)stride;
        const int32_t lo0 = b <= last ? bh[b] : re;
        const int32_t lo1 = b + 1 <= last ? bh[b + 1] : re;
        len = lo1 - lo0;
        sm.hub[threadIdx.x] = u;
        sm.hlo[threadIdx.x] = lo0;
    }
    int total;
    const int off = block_exclusive_scan(len, sm.tmp, &total);
    if ((int)threadIdx.x < nh) sm.hoff[threadIdx.x] = off;
    __syncthreads();
    // the slices' arcs spread over the threads; a slice's arcs are consecutive
    for (int idx = threadIdx.x; idx < total; idx += BLOCK) {
        int lo = 0, hi = nh;  // the last frontier vertex whose slice starts at or before idx
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (sm.hoff[mid] <= idx) lo = mid;
            else hi = mid;
        }
        const int32_t v = gr.col[sm.hlo[lo] + (idx - sm.hoff[lo])];
        uint64_t x[W];
        load_words<W>(cur + (size_t)sm.hub[lo] * W, x);
        unsigned long long *a = reinterpret_cast<unsigned long long *>(sm.acc + (size_t)(v - v0) * W);
#pragma unroll
        for (int w = 0; w < W; w++)
            if (x[w]) atomicOr(a + w, x[w]);
    }
    __syncthreads();
    // one owned target per thread: nxt(v) = Seen_i(v) | arrivals, stored once;
    // v joins F_{i+1} when the arrivals hold bits it lacked
    const int32_t v = (int32_t)v0 + (int32_t)threadIdx.x;
    bool claimed = false, in_f = false;
    if (v < v1) {
        uint64_t a[W];
        bool any = false;
#pragma unroll
        for (int w = 0; w < W; w++) {
            a[w] = sm.acc[threadIdx.x * W + w];
            any |= a[w] != 0;
        }
        in_f = (bits_cur[v >> 6] >> (v & 63)) & 1ull;
        if (any || in_f) {
            uint64_t cv[W];
            load_words<W>(cur + (size_t)v * W, cv);
            bool gained = false;
#pragma unroll
            for (int w = 0; w < W; w++) {
                gained |= (a[w] & ~cv[w]) != 0;
                cv[w] |= a[w];
            }
            if (gained || in_f) store_words<W>(nxt + (size_t)v * W, cv);
            claimed = gained;
        }
    }
    const uint64_t word = __ballot(claimed);
    if ((threadIdx.x & 63) == 0 && word)
        atomicOr(reinterpret_cast<unsigned long long *>(bits_next + ((v0 >> 6) + (threadIdx.x >> 6))), word);
    if (in_f) vertex_phase<W, WC, false>(s, g, o, gr.n, round, v);
}

// From a frontier bitmap: its counters, or its queue.  After a round that
// set only bitmap bits (a pull tile or a range-owned push block that does not
// build the queue), BITS_COUNT adds F_{i+1}'s pieces, vertices and degree sum
// to its counters (no returned values: nothing waits on the contended
// counters).  A push round needs the queue: BITS_QUEUE writes the entries of
// F_i (bitmap bits[i % 3]) into queue[i % 3], taking block offsets from the
// spare counter ctr(i)[3], and leaves the other counters alone.  Each thread
// takes BQ_VPT consecutive vertices (a slice of one bitmap word and their
// row_ptr entries, loaded together); a block's entries are contiguous and in
// vertex order, and are written with consecutive threads on consecutive
// entries.
constexpr int BQ_VPT = 16;
static_assert(64 % BQ_VPT == 0, "a thread's vertices lie in one bitmap word");
enum { BITS_COUNT = 0, BITS_QUEUE = 1 };
struct BitsQueueSmem {
    int32_t v[BLOCK * BQ_VPT];       // claimed vertices of the block, in order
    int32_t start[BLOCK * BQ_VPT];   // their first entry, from the block's base
    int tmp[WAVES + 1];
    unsigned long long degsum;
    long long base;
};

__device__ void bits_to_queue_block(BitsQueueSmem &sm, const SlotArgs &s, const GraphArgs &gr, int32_t fround,
                                    int32_t what)
{
    const int64_t v0 = ((int64_t)blockIdx.x * BLOCK + threadIdx.x) * BQ_VPT;
    uint32_t m = 0;  // this thread's frontier vertices, bit k for v0 + k
    if (v0 < gr.n) m = (uint32_t)(bits_buf(s, fround % 3)[v0 >> 6] >> (v0 & 63)) & ((1u << BQ_VPT) - 1);
    int32_t rp[BQ_VPT + 1];
    int pieces = 0;
    unsigned long long degs = 0;
    if (m) {
        // frontier vertices are < n, so row_ptr is read up to row_ptr[n]
#pragma unroll
        for (int k = 0; k <= BQ_VPT; k++) rp[k] = v0 + k <= gr.n ? gr.row_ptr[v0 + k] : 0;
#pragma unroll
        for (int k = 0; k < BQ_VPT; k++)
            if ((m >> k) & 1u) {
                const int32_t d = rp[k + 1] - rp[k];
                pieces += pieces_of(d);
                degs += (unsigned long long)d;
            }
    }
    if (threadIdx.x == 0) sm.degsum = 0;
    int total, nv;
    const int off = block_exclusive_scan(pieces, sm.tmp, &total);  // its barriers order the clear above
    const int vix = block_exclusive_scan(__popc(m), sm.tmp, &nv);
    if (total == 0) return;  // block-uniform
    unsigned long long *ctr = ctr_buf(s, fround);
    if (what == BITS_COUNT) {
        if (m) atomicAdd(&sm.degsum, degs);
        __syncthreads();
        if (threadIdx.x == 0) {
            atomicAdd(ctr + 0, (unsigned long long)total);
            atomicAdd(ctr + 1, (unsigned long long)nv);
            atomicAdd(ctr + 2, sm.degsum);
        }
        return;
    }
    if (m) {
        int at = off, x = vix;
#pragma unroll
        for (int k = 0; k < BQ_VPT; k++)
            if ((m >> k) & 1u) {
                sm.v[x] = (int32_t)(v0 + k);
                sm.start[x] = at;
                at += pieces_of(rp[k + 1] - rp[k]);
                x++;
            }
    }
    if (threadIdx.x == 0) sm.base = (long long)atomicAdd(ctr + 3, (unsigned long long)total);
    __syncthreads();
    int64_t *q = q_buf(s, fround) + sm.base;
    for (int e = threadIdx.x; e < total; e += BLOCK) {
        int lo = 0, hi = nv;  // the last vertex whose entries start at or before e
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (sm.start[mid] <= e) lo = mid;
            else hi = mid;
        }
        q[e] = ((int64_t)(e - sm.start[lo]) << 32) | (int64_t)(uint32_t)sm.v[lo];
    }
}

// ---------------------------------------------------------------------------
// Round i, pull direction (EdgeMap-Dense), one merge-path tile of TILE_ITEMS
// items (arcs and row ends) of the CSR: rows [tile_row, next tile_row) end in
// the tile, and its arcs are [tile_edge, next tile_edge).  The tile's row ends
// are staged in LDS (offsets from its first arc).
//
// Every row has one owner in the tile that holds its end item.  A row whose
// arcs and end all lie in this tile (a local row) gets nxt(v) = Seen_i(v) |
// new by a plain store and its claim in an LDS bitmap of the tile's rows; the
// (at most two) rows that cross the tile's edges merge into nxt and the
// frontier bitmap with global atomics.  After the arc phase the vertex phase
// runs for the rows whose end item is in the tile and that are in F_i, one
// row per thread (coalesced).  Finally the claimed words go to the frontier
// bitmap (plain stores where a word only holds local rows) and the claimed
// rows, expanded into their pieces, to the F_{i+1} queue at offsets from one
// block scan.
//
// Two forms of the arc phase, chosen per round:
//   PULL_WALK  each thread walks IPT consecutive items row segment by row
//              segment; per row it skips a complete set (EdgeMap's Cond_F),
//              gathers Seen_i(u) only for neighbours u in F_i (a neighbour
//              outside F_i has Seen_i(u) = Seen_{i-1}(u), already inside
//              Seen_i(v)) and stops once the set is complete (EdgeMap-Dense's
//              break).  Neighbour ids and frontier words are fetched one and
//              two batches ahead.  Partial sets of rows that span threads meet
//              in LDS.  Best when many rows are complete or F_i is small.
//   PULL_WAVE  each wave takes a contiguous quarter of the tile's arcs, 64
//              consecutive arcs per step (coalesced ids; a row's sorted
//              neighbours share cache lines) and gathers Seen_i(u) for every
//              neighbour of an incomplete row; a segmented OR-scan combines
//              each row's lanes.  Best when F_i holds most arcs and few rows
//              are complete (the first dense rounds).
// ---------------------------------------------------------------------------
struct PullTile {
    int32_t r0, e0, r1, e1;      // first row / arc of this tile and of the next
    int32_t tile_rows, tile_edges, tile_items;
    int32_t start_r0, end_r1;    // row_ptr[r0] (may lie before e0), row_end of r1
    int32_t loc_lo;              // local rows: [loc_lo, r1)
    int32_t wbase, nclaim;       // claimed bitmap words [wbase, wbase + nclaim)
};

__device__ __forceinline__ PullTile pull_coords(const GraphArgs &gr, int32_t t)
{
    PullTile T;
    T.r0 = gr.tile_row[t];
    T.e0 = gr.tile_edge[t];
    T.r1 = gr.tile_row[t + 1];
    T.e1 = gr.tile_edge[t + 1];
    T.tile_rows = T.r1 - T.r0;
    T.tile_edges = T.e1 - T.e0;
    T.tile_items = T.tile_rows + T.tile_edges;
    T.start_r0 = gr.row_ptr[T.r0];
    T.end_r1 = (int64_t)T.r1 < gr.n ? gr.row_ptr[T.r1 + 1] : T.e1;
    T.loc_lo = T.start_r0 >= T.e0 ? T.r0 : T.r0 + 1;
    T.wbase = T.r0 >> 6;
    T.nclaim = (T.r1 >> 6) - T.wbase + 1;
    return T;
}

// OR x (non-empty, bits v lacked in round i) into words [hw, hw + WL) of
// nxt(v) (W words per vertex) for a row whose arcs span several tiles; true
// if this call won v's claim in the frontier bitmap.
template <int WL, int W>
__device__ __forceinline__ bool merge_global(uint64_t *nxt, uint64_t *bits_next, int32_t v, int hw,
                                             const uint64_t (&x)[WL])
{
    uint64_t *p = nxt + (size_t)v * W + hw;
#pragma unroll
    for (int w = 0; w < WL; w++)
        if (x[w]) or64(p + w, x[w]);
    const unsigned long long bit = 1ull << (v & 63);
    const unsigned long long old = atomicOr(reinterpret_cast<unsigned long long *>(bits_next + (v >> 6)), bit);
    return !(old & bit);
}

template <int W>
__device__ __forceinline__ void pull_claim(PullSmem<W> &sm, const PullTile &T, int32_t v)
{
    atomicOr(reinterpret_cast<unsigned long long *>(&sm.claimed[(v >> 6) - T.wbase]), 1ull << (v & 63));
}

// A 64-bit DPP move: lanes whose source is outside the row, and rows left out
// of ROW_MASK, read 0.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint64_t dpp64(uint64_t x)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)x, CTRL, ROW_MASK, 0xF, true);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(x >> 32), CTRL, ROW_MASK, 0xF, true);
    return ((uint64_t)hi << 32) | lo;
}

// Inclusive segmented OR-scan over the wave: afterwards lane i holds the OR of
// lanes [first, i], where first <= i is the first lane of i's segment and
// segments are runs of consecutive lanes.  Shifts by 1, 2, 4, 8 inside each
// row of 16 lanes (DPP row_shr), then the ends of rows 0 and 2 into rows 1 and
// 3 (row_bcast:15), then the end of row 1 into rows 2 and 3 (row_bcast:31):
// all in VALU, no LDS permutes.
template <int W, int AL = 64>
__device__ __forceinline__ void seg_or_scan(uint64_t (&x)[W], int lane, int first)
{
    static_assert(AL == 64 || AL == 32 || AL == 16, "segments of 16, 32 or 64 lanes");
    // one AND-OR per dword: the lane's mask (all ones when the shifted lane
    // lies in its segment) is formed once per level
    auto level = [&](auto ctrl, auto rmask, bool take) {
        if (__ballot(take) == 0) return;  // no lane's segment reaches this far: the level is a no-op
        uint32_t m = take ? 0xFFFFFFFFu : 0u;
        asm("" : "+v"(m));  // an opaque mask: keeps AND-OR from being turned back into selects
#pragma unroll
        for (int w = 0; w < W; w++) {
            const uint32_t lo = (uint32_t)x[w], hi = (uint32_t)(x[w] >> 32);
            const uint32_t ylo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)lo, decltype(ctrl)::value,
                                                                       decltype(rmask)::value, 0xF, true);
            const uint32_t yhi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)hi, decltype(ctrl)::value,
                                                                       decltype(rmask)::value, 0xF, true);
            x[w] = ((uint64_t)((yhi & m) | hi) << 32) | (uint64_t)((ylo & m) | lo);
        }
    };
    using c1 = std::integral_constant<int, 0x111>;
    using c2 = std::integral_constant<int, 0x112>;
    using c4 = std::integral_constant<int, 0x114>;
    using c8 = std::integral_constant<int, 0x118>;
    using b15 = std::integral_constant<int, 0x142>;
    using b31 = std::integral_constant<int, 0x143>;
    using all = std::integral_constant<int, 0xF>;
    level(c1{}, all{}, lane - 1 >= first);
    level(c2{}, all{}, lane - 2 >= first);
    level(c4{}, all{}, lane - 4 >= first);
    level(c8{}, all{}, lane - 8 >= first);
    // with AL < 64 the wave holds 64 / AL independent scans of AL lanes each
    // (lane is the index inside its scan): the cross-row levels stop there
    if constexpr (AL >= 32)
        level(b15{}, std::integral_constant<int, 0xA>{}, (lane & 16) != 0 && (lane & ~15) - 1 >= first);
    if constexpr (AL == 64) level(b31{}, std::integral_constant<int, 0xC>{}, lane >= 32 && 31 >= first);
}

// Decisions shared by the H lanes of one vertex (the lanes in grp, all
// active): any / all of their predicates.
template <int H>
__device__ __forceinline__ bool group_any(bool p, uint64_t grp)
{
    if constexpr (H == 1) return p;
    else return (__ballot(p) & grp) != 0;
}
template <int H>
__device__ __forceinline__ bool group_all(bool p, uint64_t grp)
{
    if constexpr (H == 1) return p;
    else return (__ballot(p) & grp) == grp;
}

// True when a | b (this lane's share of a set: words [hw, hw + WL) for the
// lane's share index hw / WL) equals the complete set on every lane of the
// lane's group grp (all of them active).  For H > 1 each share's words are
// compared as scalars, one ballot per word, so no vector register holds a
// per-lane copy of the complete set.
template <int H, int WL>
__device__ __forceinline__ bool share_complete(const uint64_t (&a)[WL], const uint64_t (&b)[WL],
                                               const uint64_t *gfull, uint64_t grp)
{
    if constexpr (H == 1) {
        bool f = true;
#pragma unroll
        for (int w = 0; w < WL; w++) f &= (a[w] | b[w]) == gfull[w];
        return f;
    } else {
        constexpr int AL = 64 / H;
        uint64_t all = 0;  // lanes whose share equals the complete set's
#pragma unroll
        for (int j = 0; j < H; j++) {
            uint64_t m = ((AL == 64 ? 0ull : (1ull << AL)) - 1ull) << (j * AL);
#pragma unroll
            for (int w = 0; w < WL; w++) m &= __ballot((a[w] | b[w]) == gfull[j * WL + w]);
            all |= m;
        }
        return (all & grp) == grp;
    }
}

// Lanes al, al + AL, al + 2 AL, ... of a wave (the H lanes of one vertex).
template <int H>
__device__ __forceinline__ uint64_t lane_group(int al)
{
    constexpr int AL = 64 / H;
    uint64_t m = 0;
#pragma unroll
    for (int j = 0; j < H; j++) m |= 1ull << (al + AL * j);
    return m;
}

__device__ __forceinline__ uint64_t readlane64(uint64_t x, int src)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, src);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

template <int W>
constexpr int pull_batch()
{
    return W <= 2 ? 8 : (W <= 4 ? 4 : 1);
}

// PULL_WALK arc phase and vertex phase (see above).  With H = pull_split<W>()
// lanes per vertex, lanes al, al + AL, ... (AL = 64 / H) of a wave form one
// walker: they walk the same items with the same control flow, each with its
// WL = W / H words of every set, and take shared decisions (set complete,
// anything new) together.
template <int W, int WC>
__device__ void pull_walk(PullSmem<W> &sm, const SlotArgs &s, const GraphArgs &gr, const GroupDesc &g,
                          const OutArgs &o, int32_t round, const PullTile &T)
{
    constexpr int H = pull_split<W>();
    constexpr int WL = W / H;
    constexpr int AL = 64 / H;
    constexpr int WALKERS = BLOCK / H;
    constexpr int IPW = IPT * H;  // items per walker
    constexpr int NB = pull_batch<WL>();
    const uint64_t *cur = cur_buf(s, round);
    uint64_t *nxt = nxt_buf(s, round);
    const uint64_t *bits_cur = bits_buf(s, round % 3);
    uint64_t *bits_next = bits_buf(s, (round + 1) % 3);
    const int32_t r0 = T.r0, e0 = T.e0, r1 = T.r1;
    const int lane = threadIdx.x & 63, al = lane % AL;
    const int hw = (lane / AL) * WL;  // this lane's first word of a set
    const int walker = (int)(threadIdx.x >> 6) * AL + al;
    const uint64_t grp = lane_group<H>(al);
    for (int i = threadIdx.x; i < WALKERS * W; i += BLOCK) (&sm.part[0][0])[i] = 0;
    __syncthreads();
    // row_end[r] for a row of the tile (exact for r < r1; past e1 for r1)
    auto rend_of = [&](int32_t r) { return e0 + (int32_t)sm.rend[r - r0]; };
    auto rstart_of = [&](int32_t r) { return r == r0 ? T.start_r0 : e0 + (int32_t)sm.rend[r - 1 - r0]; };

    // this walker's merge-path start inside the tile
    int32_t rel = walker * IPW;
    if (rel > T.tile_items) rel = T.tile_items;
    int32_t my_end = (walker + 1) * IPW;
    if (my_end > T.tile_items) my_end = T.tile_items;
    const int32_t my_start = rel;
    int32_t row, edge;
    {
        int32_t lo = rel > T.tile_edges ? rel - T.tile_edges : 0;
        int32_t hi = rel < T.tile_rows ? rel : T.tile_rows;
        while (lo < hi) {
            int32_t mid = (lo + hi) >> 1;
            if ((int32_t)sm.rend[mid] <= rel - mid - 1) lo = mid + 1;
            else hi = mid;
        }
        row = r0 + lo;
        edge = e0 + (rel - lo);
    }


    // a local row with new bits stores nxt(v) here; a row of F_i without any
    // gets nxt(v) = Seen_i(v) in the vertex pass
    auto finish_local = [&](int32_t v, const uint64_t (&cv)[WL], const uint64_t (&acc)[WL]) {
        bool any = false;
#pragma unroll
        for (int w = 0; w < WL; w++) any |= acc[w] != 0;
        if (!group_any<H>(any, grp)) return;
        uint64_t nv[WL];
#pragma unroll
        for (int w = 0; w < WL; w++) nv[w] = cv[w] | acc[w];
        store_words<WL>(nxt + (size_t)v * W + hw, nv);
        if (hw == 0) {
            const int32_t k = v - r0;
            atomicOr(reinterpret_cast<unsigned long long *>(&sm.stored[k >> 6]), 1ull << (k & 63));
            pull_claim(sm, T, v);
        }
    };

    // a local row owned here whose first arcs other walkers scanned: its own
    // partial set joins theirs in LDS and the row is finished after the barrier
    int32_t pend = -1;
    int32_t rstart = rel < my_end ? rstart_of(row) : 0;
    while (rel < my_end) {
        const int32_t rend = rend_of(row);
        const int32_t budget = my_end - rel;
        const int32_t seg_end = rend < edge + budget ? rend : edge + budget;
        if ((sm.fin[(row - r0) >> 6] >> ((row - r0) & 63)) & 1ull) {
            // complete when the round began: nothing to gather, nothing new
            rel += seg_end - edge;
            edge = seg_end;
            if (!(edge == rend && rel < my_end)) break;
            rel++;
            row++;
            rstart = rend;
            continue;
        }
        uint64_t cv[WL], acc[WL];
        // software pipeline: the row's own set, the first two batches'
        // neighbour ids and the first batch's frontier words are requested
        // together; in the loop, batch k's Seen_i(u) gathers go out with
        // batch k+1's frontier words and batch k+2's ids, so each batch waits
        // for its own gathers only
        load_words<WL>(cur + (size_t)row * W + hw, cv);
        int32_t u0[NB], u1[NB];
        uint64_t b0[NB];
#pragma unroll
        for (int j = 0; j < NB; j++) {
            u0[j] = (edge + j < seg_end) ? gr.col[edge + j] : row;
            u1[j] = (edge + NB + j < seg_end) ? gr.col[edge + NB + j] : row;
        }
#pragma unroll
        for (int j = 0; j < NB; j++) b0[j] = bits_cur[u0[j] >> 6];
#pragma unroll
        for (int w = 0; w < WL; w++) acc[w] = 0;
        bool fin = share_complete<H, WL>(cv, acc, g.full, grp);
        for (int32_t e = edge; e < seg_end && !fin; e += NB) {
            int32_t u[NB];
            uint64_t hm[NB];  // all ones for a neighbour whose set counts
#pragma unroll
            for (int j = 0; j < NB; j++) {
                const bool hit = (((b0[j] >> (u0[j] & 63)) & 1ull) != 0) && e + j < seg_end;
                hm[j] = hit ? ~0ull : 0ull;
                u[j] = hit ? u0[j] : row;  // keep the load in place, its value is masked off
            }
            uint64_t cu[NB][WL];
#pragma unroll
            for (int j = 0; j < NB; j++) load_words<WL>(cur + (size_t)u[j] * W + hw, cu[j]);
#pragma unroll
            for (int j = 0; j < NB; j++) b0[j] = bits_cur[u1[j] >> 6];
#pragma unroll
            for (int j = 0; j < NB; j++) {
                u0[j] = u1[j];
                u1[j] = (e + 2 * NB + j < seg_end) ? gr.col[e + 2 * NB + j] : row;
            }
#pragma unroll
            for (int w = 0; w < WL; w++) {
#pragma unroll
                for (int j = 0; j < NB; j++) acc[w] |= cu[j][w] & hm[j];
                acc[w] &= ~cv[w];
            }
            fin = share_complete<H, WL>(acc, cv, g.full, grp);
        }
        rel += seg_end - edge;
        edge = seg_end;
        const bool owns_end = edge == rend && rel < my_end;
        const int32_t first_item = (row - r0) + (rstart - e0);
        const bool local = first_item >= 0 && row < r1;
        if (!local) {
            // crosses a tile edge: merge by global atomics (each lane its words)
            bool any = false;
#pragma unroll
            for (int w = 0; w < WL; w++) any |= acc[w] != 0;
            if (any && merge_global<WL, W>(nxt, bits_next, row, hw, acc)) pull_claim(sm, T, row);
        } else if (!owns_end || first_item < my_start) {
            // a local row other walkers share: into the slot of its first walker
            uint64_t *slot = sm.part[first_item / IPW] + hw;
#pragma unroll
            for (int w = 0; w < WL; w++)
                if (acc[w]) atomicOr(reinterpret_cast<unsigned long long *>(slot + w), acc[w]);
            if (owns_end) pend = row;
        } else {
            finish_local(row, cv, acc);
        }
        if (!owns_end) break;  // items exhausted inside this row
        rel++;
        row++;
        rstart = rend;
    }
    __syncthreads();
    if (pend >= 0) {
        const int32_t first_item = (pend - r0) + (rstart_of(pend) - e0);
        const uint64_t *slot = sm.part[first_item / IPW] + hw;
        uint64_t cv[WL], acc[WL];
        load_words<WL>(cur + (size_t)pend * W + hw, cv);
#pragma unroll
        for (int w = 0; w < WL; w++) acc[w] = slot[w];
        finish_local(pend, cv, acc);
    }
    __syncthreads();
    // vertex phase of the rows whose end item is in this tile, one thread per
    // (row, cluster): the threads of a row read its words together, with the
    // frontier word (membership only gates the writes); a local row of F_i
    // the arc phase did not store gets nxt(v) = Seen_i(v)
    constexpr int CPV = W / WC;
    const int32_t units = units_of<WC>(g);
    for (int32_t idx = threadIdx.x; idx < (r1 - r0) * CPV; idx += BLOCK) {
        const int32_t v = r0 + idx / CPV, j = idx % CPV;
        if (j >= units) continue;
        const bool in_f = (bits_cur[v >> 6] >> (v & 63)) & 1ull;
        const int32_t k = v - r0;
        if (v < T.loc_lo) {
            vertex_phase_cluster<W, WC, true>(s, g, o, gr.n, round, v, j, in_f);  // tile-crossing row
        } else {
            const bool copy = in_f && !((sm.stored[k >> 6] >> (k & 63)) & 1ull);
            vertex_phase_cluster<W, WC, false>(s, g, o, gr.n, round, v, j, in_f, copy);
        }
    }
    __syncthreads();
}

// PULL_WAVE arc phase and vertex phase (see above).  With H = pull_split<W>()
// lanes per vertex a step covers AL = 64 / H arcs: arc k of the step on lanes
// k, k + AL, ..., each lane with its WL = W / H words of every set; the
// segmented scan runs within each group of AL lanes, and the lanes of one arc
// take shared decisions (anything new, set complete) together.
template <int W, int WC>
__device__ void pull_wave(PullSmem<W> &sm, const SlotArgs &s, const GraphArgs &gr, const GroupDesc &g,
                          const OutArgs &o, int32_t round, const PullTile &T)
{
    constexpr int H = pull_split<W>();
    constexpr int WL = W / H;
    constexpr int AL = 64 / H;
    const uint64_t *cur = cur_buf(s, round);
    uint64_t *nxt = nxt_buf(s, round);
    const uint64_t *bits_cur = bits_buf(s, round % 3);
    uint64_t *bits_next = bits_buf(s, (round + 1) % 3);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int al = lane % AL, h = lane / AL, hw = h * WL;
    const uint64_t grp = lane_group<H>(al);
    const int32_t r0 = T.r0, e0 = T.e0, r1 = T.r1, tile_rows = T.tile_rows, tile_edges = T.tile_edges;

    for (int32_t k = threadIdx.x; k < tile_edges; k += BLOCK) sm.wv.arow[k] = 0;
    if (threadIdx.x < WAVES) {
        sm.wv.out_row[threadIdx.x] = -1;
        sm.wv.pend_row[threadIdx.x] = -1;
    }
    __syncthreads();
    // row start offset of row r0 + k (negative for a row begun before the tile)
    auto rstart_off = [&](int32_t k) { return k == 0 ? T.start_r0 - e0 : (int32_t)sm.rend[k - 1]; };
    // row starts scattered for the arc -> row map
    for (int32_t k = threadIdx.x; k <= tile_rows; k += BLOCK) {
        const int32_t r = r0 + k;
        if ((int64_t)r >= gr.n) continue;
        const int32_t so = rstart_off(k);
        const int32_t a = so > 0 ? so : 0;
        const int32_t b = (int32_t)sm.rend[k] < tile_edges ? (int32_t)sm.rend[k] : tile_edges;
        if (a < b) sm.wv.arow[a] = (uint16_t)k;
    }
    __syncthreads();
    {
        // arc -> row: running max of the scattered row starts
        const int32_t per = (tile_edges + BLOCK - 1) / BLOCK;
        const int32_t lo = (int32_t)threadIdx.x * per < tile_edges ? (int32_t)threadIdx.x * per : tile_edges;
        const int32_t hi = lo + per < tile_edges ? lo + per : tile_edges;
        int m = 0;
        for (int32_t k = lo; k < hi; k++) {
            const int x = sm.wv.arow[k];
            m = x > m ? x : m;
            sm.wv.arow[k] = (uint16_t)m;
        }
        const int before = block_exclusive_max(m, sm.tmp);
        // the final row of each arc, with the facts a step needs about it
        for (int32_t k = lo; k < hi; k++) {
            int r = sm.wv.arow[k];
            r = r > before ? r : before;
            int a = r;
            if (k + 1 == (int32_t)sm.rend[r]) a |= AROW_LAST;
            if (k == rstart_off(r)) a |= AROW_FIRST;
            if ((sm.fin[r >> 6] >> (r & 63)) & 1ull) a |= AROW_DONE;
            sm.wv.arow[k] = (uint16_t)a;
        }
    }
    __syncthreads();

    const int32_t wa = (int32_t)(((int64_t)tile_edges * wv) / WAVES);
    const int32_t wb = (int32_t)(((int64_t)tile_edges * (wv + 1)) / WAVES);
    // a row whose every contribution from this tile is in x (words
    // [hx, hx + WL) of each set; the lanes of gx hold the other words); cv
    // holds those words of cur(v)
    auto finish_row_cv = [&](int32_t k, const uint64_t (&x)[WL], uint64_t (&cv)[WL], int hx, uint64_t gx) {
        const int32_t v = r0 + k;
        uint64_t acc[WL];
        bool any = false;
#pragma unroll
        for (int w = 0; w < WL; w++) {
            acc[w] = x[w] & ~cv[w];
            any |= acc[w] != 0;
        }
        if (v >= T.loc_lo && v < r1) {
            if (!group_any<H>(any, gx)) return;
#pragma unroll
            for (int w = 0; w < WL; w++) cv[w] |= acc[w];
            store_words<WL>(nxt + (size_t)v * W + hx, cv);
            if (hx == 0) {
                atomicOr(reinterpret_cast<unsigned long long *>(&sm.stored[k >> 6]), 1ull << (k & 63));
                pull_claim(sm, T, v);
            }
        } else if (any && merge_global<WL, W>(nxt, bits_next, v, hx, acc)) {
            pull_claim(sm, T, v);
        }
    };
    auto finish_row = [&](int32_t k, const uint64_t (&x)[WL], int hx, uint64_t gx) {
        bool nz = false;
#pragma unroll
        for (int w = 0; w < WL; w++) nz |= x[w] != 0;
        if (!group_any<H>(nz, gx)) return;
        uint64_t cv[WL];
        load_words<WL>(cur + (size_t)(r0 + k) * W + hx, cv);
        finish_row_cv(k, x, cv, hx, gx);
    };
    // a row's share of this wave's range ends with x: finished here, or left
    // for the merge below (begun in an earlier wave's range, or open past it)
    auto close_row = [&](int32_t k, const uint64_t (&x)[WL]) {
        if (rstart_off(k) >= wa) {
            finish_row(k, x, hw, grp);
        } else {
            sm.wv.pend_row[wv] = k;
#pragma unroll
            for (int w = 0; w < WL; w++) sm.wv.pend_acc[wv][hw + w] = x[w];
        }
    };
    auto leave_row = [&](int32_t k, const uint64_t (&x)[WL]) {
        sm.wv.out_row[wv] = k;
#pragma unroll
        for (int w = 0; w < WL; w++) sm.wv.out_acc[wv][hw + w] = x[w];
    };

    int32_t crow = -1;  // row carried from the wave's previous step (wave-uniform)
    uint64_t ccv[WL];   // its cur words (this lane's share); its OR so far is in sm.wv.cacc[wv]
#pragma unroll
    for (int w = 0; w < WL; w++) ccv[w] = 0;
    for (int32_t base = wa; base < wb;) {
        int32_t next = base + AL;
        const int32_t k = base + al;
        const bool in = k < wb;
        const int32_t a = in ? (int32_t)sm.wv.arow[k] : 0;
        const int32_t rk = a & AROW_ROW;  // a valid row index on every lane
        const bool active = in && !(a & AROW_DONE);
        const bool last = in && (a & AROW_LAST);  // the row's last arc in the tile
        // a row that will carry out of this step and was not carried into it:
        // its words go out with this step's gathers, so the completeness test
        // at the step's end already covers its first AL arcs
        {
            const int32_t rl = __builtin_amdgcn_readlane(rk, AL - 1);
            const int32_t ll = __builtin_amdgcn_readlane((int)last, AL - 1);
            if (base + AL < wb && !ll && rl != crow)
                load_words<WL>(cur + (size_t)(r0 + rl) * W + hw, ccv);
        }
        uint64_t x[WL];
#pragma unroll
        for (int w = 0; w < WL; w++) x[w] = 0;
        if (__ballot(active)) {
            const int32_t u = active ? gr.col[e0 + k] : r0;
            const uint64_t hm = active ? ~0ull : 0ull;
            // the lane where this row's arcs begin in this step (lanes of one
            // row are consecutive: the nearest first arc at or below this
            // lane, else lane 0); a lane past the range is its own segment
            const uint64_t fb = (__ballot(in && (a & AROW_FIRST)) >> (h * AL)) & lane_mask_upto(al);
            const int first = in ? (fb ? 63 - __builtin_clzll(fb) : 0) : al;
            load_words<WL>(cur + (size_t)u * W + hw, x);
#pragma unroll
            for (int w = 0; w < WL; w++) x[w] &= hm;
            seg_or_scan<WL, AL>(x, al, first);
        }
        // the last lane of a row's run in this step
        const bool tail = in && (al == AL - 1 || k + 1 == wb || last);
        if (tail && rk == crow) {
#pragma unroll
            for (int w = 0; w < WL; w++) x[w] |= sm.wv.cacc[wv][hw + w];
        }
        const bool closes = tail && last;                   // the row's last arc in the tile
        const bool leaves = tail && !closes && k + 1 == wb;  // open past this wave's range
        const bool carries = tail && !closes && !leaves;     // only the step's last arc
        if (closes) close_row(rk, x);
        else if (leaves) leave_row(rk, x);
        // carry into the next step: the carrying lanes (the step's last arc,
        // one per share of the words) keep the row's OR so far in LDS; a
        // carried row found complete adds nothing more, so the wave closes it
        // now and jumps past its remaining arcs
        if (__builtin_amdgcn_readlane((int)carries, AL - 1)) {
            crow = __builtin_amdgcn_readlane(rk, AL - 1);
            bool f = false;
            if (al == AL - 1) {
#pragma unroll
                for (int w = 0; w < WL; w++) sm.wv.cacc[wv][hw + w] = x[w];
                f = share_complete<H, WL>(x, ccv, g.full, grp);
            }
            if (__builtin_amdgcn_readlane((int)f, AL - 1)) {
                const int32_t cre = (int32_t)sm.rend[crow];
                if (al == AL - 1) {
                    if (cre > wb) {
                        leave_row(crow, x);
                    } else if (rstart_off(crow) >= wa) {
                        uint64_t cv[WL];
#pragma unroll
                        for (int w = 0; w < WL; w++) cv[w] = ccv[w];
                        finish_row_cv(crow, x, cv, hw, grp);
                    } else {
                        close_row(crow, x);  // pending: merged after the loop
                    }
                }
                next = cre <= wb ? cre : wb;
                crow = -1;
            }
        } else {
            crow = -1;
        }
        base = next;
    }
    __syncthreads();
    // rows split between waves: the closing wave's share plus the earlier ones
    // (H threads per wave, one per share of the words); the row continuing
    // past the tile merges globally (H threads after those)
    if ((int)threadIdx.x < WAVES * H) {
        const int w0 = threadIdx.x / H, hx = (threadIdx.x % H) * WL;
        const uint64_t gx = ((1ull << H) - 1ull) << (w0 * H);
        const int32_t rk = sm.wv.pend_row[w0];
        if (rk >= 0) {
            uint64_t x[WL];
#pragma unroll
            for (int w = 0; w < WL; w++) x[w] = sm.wv.pend_acc[w0][hx + w];
            for (int w1 = 0; w1 < w0; w1++)
                if (sm.wv.out_row[w1] == rk) {
#pragma unroll
                    for (int w = 0; w < WL; w++) x[w] |= sm.wv.out_acc[w1][hx + w];
                }
            finish_row(rk, x, hx, gx);
        }
    } else if ((int)threadIdx.x < WAVES * H + H) {
        const int hx = ((int)threadIdx.x - WAVES * H) * WL;
        const uint64_t gx = ((1ull << H) - 1ull) << (WAVES * H);
        int32_t rk = -1;
        for (int w1 = 0; w1 < WAVES; w1++)
            if (sm.wv.out_row[w1] >= 0 && (int32_t)sm.rend[sm.wv.out_row[w1]] > tile_edges) rk = sm.wv.out_row[w1];
        if (rk >= 0) {
            uint64_t x[WL];
#pragma unroll
            for (int w = 0; w < WL; w++) x[w] = 0;
            for (int w1 = 0; w1 < WAVES; w1++)
                if (sm.wv.out_row[w1] == rk) {
#pragma unroll
                    for (int w = 0; w < WL; w++) x[w] |= sm.wv.out_acc[w1][hx + w];
                }
            finish_row(rk, x, hx, gx);
        }
    }
    __syncthreads();
    // vertex phase of the rows whose end item is in this tile, one thread per
    // (row, cluster); a local row the arc phase did not store gets nxt(v) =
    // Seen_i(v) here, each thread its cluster's words
    constexpr int CPV = W / WC;
    const int32_t units = units_of<WC>(g);
    for (int32_t idx = threadIdx.x; idx < (r1 - r0) * CPV; idx += BLOCK) {
        const int32_t v = r0 + idx / CPV, j = idx % CPV;
        if (j >= units || !((bits_cur[v >> 6] >> (v & 63)) & 1ull)) continue;
        const int32_t k = v - r0;
        if (v < T.loc_lo) {
            vertex_phase_cluster<W, WC, true>(s, g, o, gr.n, round, v, j);  // tile-crossing row
        } else {
            const bool copy = !((sm.stored[k >> 6] >> (k & 63)) & 1ull);
            vertex_phase_cluster<W, WC, false>(s, g, o, gr.n, round, v, j, true, copy);
        }
    }
    __syncthreads();
}

// queue = false: the tile writes F_{i+1}'s bitmap words and adds to its
// counters without waiting on them; the queue, if a push round needs it, is
// built from the bitmap afterwards (bits_to_queue_block).
template <int W, int WC>
__device__ void pull_tile(PullSmem<W> &sm, const SlotArgs &s, const GraphArgs &gr, const GroupDesc &g,
                          const OutArgs &o, int32_t round, int32_t t, int32_t form, bool queue = true)
{
    const PullTile T = pull_coords(gr, t);
    __syncthreads();
    for (int32_t k = threadIdx.x; k <= T.tile_rows; k += BLOCK) {
        const int32_t r = T.r0 + k;
        int32_t x = ((int64_t)r < gr.n ? gr.row_ptr[r + 1] : T.e1) - T.e0;
        sm.rend[k] = (uint16_t)(x > T.tile_edges + 1 ? T.tile_edges + 1 : x);
    }
    for (int32_t k = threadIdx.x; k < T.nclaim; k += BLOCK) sm.claimed[k] = 0;
    if (threadIdx.x == 0) {
        sm.degsum = 0;
        sm.big.n = 0;
    }
    // rows whose set is already complete gather nothing: each wave tests 64
    // consecutive rows (coalesced row words) and writes their bitmap word
    {
        const uint64_t *cur = cur_buf(s, round);
        const int lane = threadIdx.x & 63;
        for (int32_t kb = (int32_t)(threadIdx.x >> 6) * 64; kb <= T.tile_rows; kb += WAVES * 64) {
            const int32_t k = kb + lane;
            bool f = false;
            if (k <= T.tile_rows && (int64_t)(T.r0 + k) < gr.n) {
                uint64_t cv[W];
                load_words<W>(cur + (size_t)(T.r0 + k) * W, cv);
                f = true;
#pragma unroll
                for (int w = 0; w < W; w++) f &= cv[w] == g.full[w];
            }
            const uint64_t word = __ballot(f);
            if (lane == 0) {
                sm.fin[kb >> 6] = word;
                sm.stored[kb >> 6] = 0;
            }
        }
    }
    if (form == PULL_WAVE) pull_wave<W, WC>(sm, s, gr, g, o, round, T);
    else pull_walk<W, WC>(sm, s, gr, g, o, round, T);

    // frontier flush: one claimed word per thread (nclaim <= BLOCK)
    const int32_t r0 = T.r0, r1 = T.r1, e0 = T.e0;
    uint64_t *bits_next = bits_buf(s, (round + 1) % 3);
    auto deg_of = [&](int32_t v) {
        const int32_t k = v - r0;
        const int32_t st = k == 0 ? T.start_r0 : e0 + (int32_t)sm.rend[k - 1];
        return (v == r1 ? T.end_r1 : e0 + (int32_t)sm.rend[k]) - st;
    };
    uint64_t word = 0;
    int pieces = 0;
    if ((int32_t)threadIdx.x < T.nclaim) {
        word = sm.claimed[threadIdx.x];
        if (word) {
            const int64_t wi = (int64_t)T.wbase + threadIdx.x;
            if (wi * 64 >= T.loc_lo && wi * 64 + 63 < r1) bits_next[wi] = word;
            else atomicOr(reinterpret_cast<unsigned long long *>(bits_next + wi), word);
            unsigned long long dsum = 0;
            for (uint64_t x = word; x; x &= x - 1) {
                const int32_t v = (int32_t)(wi * 64 + __builtin_ctzll(x));
                const int32_t d = deg_of(v);
                pieces += pieces_of(d);
                dsum += (unsigned long long)d;
            }
            atomicAdd(&sm.degsum, dsum);
        }
    }
    int total;
    const int off = block_exclusive_scan(pieces, sm.tmp, &total);
    int cnt_total;
    block_exclusive_scan(__popcll(word), sm.tmp, &cnt_total);
    if (total == 0) return;  // block-uniform
    unsigned long long *ctr_next = ctr_buf(s, round + 1);
    if (!queue) {
        if (threadIdx.x == 0) {
            atomicAdd(ctr_next + 0, (unsigned long long)total);
            atomicAdd(ctr_next + 1, (unsigned long long)cnt_total);
            atomicAdd(ctr_next + 2, sm.degsum);
        }
        return;
    }
    if (threadIdx.x == 0) {
        sm.base = (long long)atomicAdd(ctr_next + 0, (unsigned long long)total);
        atomicAdd(ctr_next + 1, (unsigned long long)cnt_total);
        atomicAdd(ctr_next + 2, sm.degsum);
    }
    __syncthreads();
    int64_t *q = q_buf(s, round + 1);
    long long at = sm.base + off;
    const int64_t wi = (int64_t)T.wbase + threadIdx.x;
    for (uint64_t x = word; x; x &= x - 1) {
        const int32_t v = (int32_t)(wi * 64 + __builtin_ctzll(x));
        const int pc = pieces_of(deg_of(v));
        put_pieces(sm.big, q, at, v, pc);
        at += pc;
    }
    big_write(sm.big, q);
}

// ---------------------------------------------------------------------------
// Finalize: a vertex never reached by the center (center-relative) or by any
// source (min-relative) gets CBFS_UNREACHED and zero masks (a cluster source
// reaching it is a radius violation); a vertex reached but not by every
// source of the cluster is a violation too.
// ---------------------------------------------------------------------------
template <int W, int WC>
__device__ __forceinline__ void finalize_part(const SlotArgs &s, int64_t n, const GroupDesc &g, const OutArgs &o,
                                              int64_t tid, int64_t stride)
{
    const int64_t P = planes_of(o);
    const bool fields = WC == 1 && g.flog < 6;
    const int32_t F = fields ? fields_per_word(g) : 1;
    const uint64_t fm = fields ? field_mask(g) : ~0ull;
    for (int64_t v = tid; v < n; v += stride) {
        uint64_t sv[W];
        load_words<W>(s.seen + (size_t)v * W, sv);
#pragma unroll
        for (int j = 0; j < W / WC; j++) {
            for (int32_t f = 0; f < F; f++) {
                const int32_t cj = j * F + f;  // cluster index in the group
                if (cj >= g.nc) break;
                const int32_t c = g.c0 + cj;
                uint64_t sc[WC], fl[WC];
#pragma unroll
                for (int x = 0; x < WC; x++) {
                    sc[x] = fields ? (sv[j] >> (f << g.flog)) & fm : sv[j * WC + x];
                    fl[x] = fields ? (g.full[j] >> (f << g.flog)) & fm : g.full[j * WC + x];
                }
                bool any = false, full = true;
#pragma unroll
                for (int x = 0; x < WC; x++) {
                    any |= sc[x] != 0;
                    full &= sc[x] == fl[x];
                }
                // unreached: by the center (center-relative), or by every source
                // (min-relative, where Delta_v needs only one)
                if (o.minrel ? !any : !(sc[0] & 1ull)) {
                    if (any) atomicExch(o.status + c, E_RADIUS);
                    o.dist[(size_t)c * n + v] = UNREACHED;
                    for (int64_t p = 0; p < P; p++) {
                        uint64_t *dst = o.masks + (((size_t)c * P + p) * (size_t)n + (size_t)v) * WC;
#pragma unroll
                        for (int x = 0; x < WC; x++) dst[x] = 0;
                    }
                } else if (!full) {
                    atomicExch(o.status + c, E_RADIUS);
                }
            }
        }
    }
}

}  // namespace cbfs
