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

template <int W>
struct PullSmem {
    uint64_t part[BLOCK][W];                 // partial sets of rows shared by threads, by first thread
    uint64_t claimed[PULL_CLAIM_WORDS];      // F_{i+1} bits of the tile's rows, from word tile_row >> 6
    uint16_t rend[TILE_ITEMS + 2];           // row_end of the tile's rows minus tile_edge (clamped)
    int tmp[WAVES + 1];
    unsigned long long degsum;
    long long base;
};

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
    const int64_t words = n * W;
    for (int64_t k = tid; k < words; k += stride) {
        s.A[k] = 0;
        s.B[k] = 0;
        s.seen[k] = 0;
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
                           const int32_t *sources, const int32_t *cluster_ptr)
{
    __syncthreads();
    stager_init(st);
    __syncthreads();
    const int32_t first = cluster_ptr[g.c0];
    const int32_t total = cluster_ptr[g.c0 + g.nc] - first;
    for (int32_t k = threadIdx.x; k < total; k += BLOCK) {
        const int32_t idx = first + k;
        int32_t j = 0;
        while (cluster_ptr[g.c0 + j + 1] <= idx) j++;
        const int32_t i = idx - cluster_ptr[g.c0 + j];
        const int32_t v = sources[idx];
        or64(s.A + (size_t)v * W + j * WC + (i >> 6), 1ull << (i & 63));
        claim(st, s.bits0, v, gr.row_ptr[v + 1] - gr.row_ptr[v]);
    }
    stager_flush(st, gr.row_ptr, s.q0, s.ctr + 0);
}

// ---------------------------------------------------------------------------
// Round i, push direction (EdgeMap-Sparse), one chunk of epb <= BLOCK queue
// entries (pieces of <= PIECE arcs; epb from push_entries_per_block, so a
// chunk holds about PUSH_BLOCK_ARCS arcs): the vertex phase for first pieces, then the
// chunk's arcs spread evenly over the block (block scan + binary search of
// each arc's owner).  Per arc (u, v): x = Seen_i(u) \ Seen_i(v); if not empty,
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
    const int64_t idx = first + threadIdx.x;
    if ((int32_t)threadIdx.x < epb && idx < nq) {
        const int64_t e = q_buf(s, round)[idx];
        const int32_t u = (int32_t)(e & 0xffffffff);
        const int32_t p = (int32_t)(e >> 32);
        const int32_t rs = gr.row_ptr[u], re = gr.row_ptr[u + 1];
        const int32_t lo = rs + p * PIECE;
        const int32_t hi = re < lo + PIECE ? re : lo + PIECE;
        cnt = hi > lo ? hi - lo : 0;
        uint64_t cu[W];
        load_words<W>(cur + (size_t)u * W, cu);
        if (p == 0) vertex_phase<W, WC>(s, g, o, gr.n, round, u);
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
// Round i, pull direction (EdgeMap-Dense), one merge-path tile of TILE_ITEMS
// items (arcs and row ends) of the CSR.  The tile's row ends are first staged
// in LDS (as offsets from the tile's first arc), so that each thread finds its
// merge-path start and walks its rows without global row-pointer loads.  Each
// thread then walks IPT consecutive items row segment by row segment.  For a
// row v it loads Seen_i(v) once (a finished row, holding every source, is
// skipped: EdgeMap's Cond_F), then processes its arcs in batches: the frontier
// bits of all neighbours in the batch, then Seen_i(u) of all of them, are
// requested together (unconditional loads with a select, so the loads
// overlap), and the new bits are OR-ed into a register accumulator; the row
// stops once the accumulator completes the set (EdgeMap-Dense's break).
// Without test_frontier every neighbour's set is OR-ed: a neighbour outside
// F_i has Seen_i(u) = Seen_{i-1}(u), already inside Seen_i(v), so this only
// saves the bitmap lookups when F_i holds most of the arcs.
//
// Every row has one owner, the thread that consumes its end item.  For a row
// whose arcs and end all lie in this tile (a local row) the partial sets of
// the threads on it meet in LDS (slot of the row's first thread), and the
// owner writes nxt(v) = Seen_i(v) | new with a plain store and claims v in an
// LDS bitmap of the tile's rows.  Only the (at most two) rows that cross the
// tile's edges merge into nxt and the frontier bitmap with global atomics; a
// claim they win joins the LDS bitmap.  Then the vertex phase runs for the
// rows whose end item is in the tile and that are in F_i, one row per thread,
// so its loads and stores are coalesced.  Finally the claimed words go to the
// frontier bitmap (plain stores where a word only holds local rows of this
// tile) and the claimed rows, expanded into their pieces, to the F_{i+1}
// queue at offsets from one block scan.
// ---------------------------------------------------------------------------
template <int W>
constexpr int pull_batch()
{
    return W <= 2 ? 8 : (W <= 4 ? 4 : 1);
}

// OR x (non-empty, bits v lacked in round i) into nxt(v) for a row whose arcs
// span several tiles; true if this call won v's claim in the frontier bitmap.
template <int W>
__device__ __forceinline__ bool merge_global(uint64_t *nxt, uint64_t *bits_next, int32_t v, const uint64_t (&x)[W])
{
    uint64_t *p = nxt + (size_t)v * W;
#pragma unroll
    for (int w = 0; w < W; w++)
        if (x[w]) or64(p + w, x[w]);
    const unsigned long long bit = 1ull << (v & 63);
    const unsigned long long old = atomicOr(reinterpret_cast<unsigned long long *>(bits_next + (v >> 6)), bit);
    return !(old & bit);
}

template <int W, int WC>
__device__ void pull_tile(PullSmem<W> &sm, const SlotArgs &s, const GraphArgs &gr, const GroupDesc &g,
                          const OutArgs &o, int32_t round, int32_t t, bool test_frontier)
{
    constexpr int NB = pull_batch<W>();
    const uint64_t *cur = cur_buf(s, round);
    uint64_t *nxt = nxt_buf(s, round);
    const uint64_t *bits_cur = bits_buf(s, round % 3);
    uint64_t *bits_next = bits_buf(s, (round + 1) % 3);

    const int32_t r0 = gr.tile_row[t], e0 = gr.tile_edge[t];
    const int32_t r1 = gr.tile_row[t + 1], e1 = gr.tile_edge[t + 1];
    // merge-path coordinates inside the tile: arc e of row r is item
    // (r - r0) + (e - e0); the end item of row r is (r - r0) + (row_end[r] - e0).
    // Rows r0 .. r1 - 1 end in this tile; row r1 (if it exists) may have arcs
    // here and end in a later tile.
    const int32_t tile_rows = r1 - r0, tile_edges = e1 - e0;
    const int32_t tile_items = tile_rows + tile_edges;
    const int32_t start_r0 = gr.row_ptr[r0];  // may lie before e0
    const int32_t end_r1 = (int64_t)r1 < gr.n ? gr.row_ptr[r1 + 1] : e1;
    // local rows: [loc_lo, r1), those whose first arc is in this tile
    const int32_t loc_lo = start_r0 >= e0 ? r0 : r0 + 1;
    const int32_t wbase = r0 >> 6;
    const int32_t nclaim = (r1 >> 6) - wbase + 1;
    __syncthreads();
#pragma unroll
    for (int w = 0; w < W; w++) sm.part[threadIdx.x][w] = 0;
    for (int32_t k = threadIdx.x; k < nclaim; k += BLOCK) sm.claimed[k] = 0;
    for (int32_t k = threadIdx.x; k <= tile_rows; k += BLOCK) {
        const int32_t r = r0 + k;
        int32_t x = ((int64_t)r < gr.n ? gr.row_ptr[r + 1] : e1) - e0;
        sm.rend[k] = (uint16_t)(x > tile_edges + 1 ? tile_edges + 1 : x);
    }
    if (threadIdx.x == 0) sm.degsum = 0;
    __syncthreads();
    // row_end[r] for a row of the tile (exact for r < r1; past e1 for r1)
    auto rend_of = [&](int32_t r) { return e0 + (int32_t)sm.rend[r - r0]; };
    auto rstart_of = [&](int32_t r) { return r == r0 ? start_r0 : e0 + (int32_t)sm.rend[r - 1 - r0]; };

    // this thread's merge-path start inside the tile
    int32_t rel = (int32_t)threadIdx.x * IPT;
    if (rel > tile_items) rel = tile_items;
    int32_t my_end = ((int32_t)threadIdx.x + 1) * IPT;
    if (my_end > tile_items) my_end = tile_items;
    const int32_t my_start = rel;
    int32_t row, edge;
    {
        int32_t lo = rel > tile_edges ? rel - tile_edges : 0;
        int32_t hi = rel < tile_rows ? rel : tile_rows;
        while (lo < hi) {
            int32_t mid = (lo + hi) >> 1;
            if ((int32_t)sm.rend[mid] <= rel - mid - 1) lo = mid + 1;
            else hi = mid;
        }
        row = r0 + lo;
        edge = e0 + (rel - lo);
    }

    uint64_t full[W];
#pragma unroll
    for (int w = 0; w < W; w++) full[w] = g.full[w];

    auto claim_lds = [&](int32_t v) {
        atomicOr(reinterpret_cast<unsigned long long *>(&sm.claimed[(v >> 6) - wbase]), 1ull << (v & 63));
    };
    auto finish_local = [&](int32_t v, const uint64_t (&cv)[W], const uint64_t (&acc)[W]) {
        bool any = false;
#pragma unroll
        for (int w = 0; w < W; w++) any |= acc[w] != 0;
        const bool in_f = (bits_cur[v >> 6] >> (v & 63)) & 1ull;
        if (in_f || any) {
            uint64_t nv[W];
#pragma unroll
            for (int w = 0; w < W; w++) nv[w] = cv[w] | acc[w];
            store_words<W>(nxt + (size_t)v * W, nv);
        }
        if (any) claim_lds(v);
    };

    // a local row owned here whose first arcs other threads scanned: its own
    // partial set joins theirs in LDS and the row is finished after the barrier
    int32_t pend = -1;
    int32_t rstart = rel < my_end ? rstart_of(row) : 0;
    while (rel < my_end) {
        const int32_t rend = rend_of(row);
        const int32_t budget = my_end - rel;
        const int32_t seg_end = rend < edge + budget ? rend : edge + budget;
        uint64_t cv[W], acc[W];
        load_words<W>(cur + (size_t)row * W, cv);
        bool fin = true;
#pragma unroll
        for (int w = 0; w < W; w++) {
            acc[w] = 0;
            fin &= cv[w] == full[w];
        }
        for (int32_t e = edge; e < seg_end && !fin; e += NB) {
            int32_t u[NB];
            bool hit[NB];
#pragma unroll
            for (int j = 0; j < NB; j++) u[j] = (e + j < seg_end) ? gr.col[e + j] : row;
            if (test_frontier) {
                uint64_t bw[NB];
#pragma unroll
                for (int j = 0; j < NB; j++) bw[j] = bits_cur[u[j] >> 6];
#pragma unroll
                for (int j = 0; j < NB; j++) hit[j] = ((bw[j] >> (u[j] & 63)) & 1ull) && (e + j < seg_end);
            } else {
#pragma unroll
                for (int j = 0; j < NB; j++) hit[j] = e + j < seg_end;
            }
            uint64_t cu[NB][W];
#pragma unroll
            for (int j = 0; j < NB; j++) load_words<W>(cur + (size_t)(hit[j] ? u[j] : row) * W, cu[j]);
            bool f = true;
#pragma unroll
            for (int w = 0; w < W; w++) {
#pragma unroll
                for (int j = 0; j < NB; j++) acc[w] |= hit[j] ? (cu[j][w] & ~cv[w]) : 0ull;
                f &= (acc[w] | cv[w]) == full[w];
            }
            fin = f;
        }
        rel += seg_end - edge;
        edge = seg_end;
        const bool owns_end = edge == rend && rel < my_end;
        const int32_t first_item = (row - r0) + (rstart - e0);
        const bool local = first_item >= 0 && row < r1;
        if (!local) {
            // crosses a tile edge: merge by global atomics
            bool any = false;
#pragma unroll
            for (int w = 0; w < W; w++) any |= acc[w] != 0;
            if (any && merge_global<W>(nxt, bits_next, row, acc)) claim_lds(row);
        } else if (!owns_end || first_item < my_start) {
            // a local row other threads share: into the slot of its first thread
            uint64_t *slot = sm.part[first_item / IPT];
#pragma unroll
            for (int w = 0; w < W; w++)
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
        const uint64_t *slot = sm.part[first_item / IPT];
        uint64_t cv[W], acc[W];
        load_words<W>(cur + (size_t)pend * W, cv);
#pragma unroll
        for (int w = 0; w < W; w++) acc[w] = slot[w];
        finish_local(pend, cv, acc);
    }
    // vertex phase of the rows whose end item is in this tile
    for (int32_t v = r0 + (int32_t)threadIdx.x; v < r1; v += BLOCK) {
        if (!((bits_cur[v >> 6] >> (v & 63)) & 1ull)) continue;
        if (v < loc_lo) vertex_phase<W, WC, true>(s, g, o, gr.n, round, v);  // tile-crossing row
        else vertex_phase<W, WC, false>(s, g, o, gr.n, round, v);
    }
    __syncthreads();

    // frontier flush: one claimed word per thread (nclaim <= BLOCK)
    auto deg_of = [&](int32_t v) { return (v == r1 ? end_r1 : rend_of(v)) - rstart_of(v); };
    uint64_t word = 0;
    int pieces = 0;
    if ((int32_t)threadIdx.x < nclaim) {
        word = sm.claimed[threadIdx.x];
        if (word) {
            const int64_t wi = (int64_t)wbase + threadIdx.x;
            if (wi * 64 >= loc_lo && wi * 64 + 63 < r1) bits_next[wi] = word;
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
    if (threadIdx.x == 0) {
        sm.base = (long long)atomicAdd(ctr_next + 0, (unsigned long long)total);
        atomicAdd(ctr_next + 1, (unsigned long long)cnt_total);
        atomicAdd(ctr_next + 2, sm.degsum);
    }
    __syncthreads();
    int64_t *dst = q_buf(s, round + 1) + sm.base + off;
    const int64_t wi = (int64_t)wbase + threadIdx.x;
    for (uint64_t x = word; x; x &= x - 1) {
        const int32_t v = (int32_t)(wi * 64 + __builtin_ctzll(x));
        const int pc = pieces_of(deg_of(v));
        for (int p = 0; p < pc; p++) *dst++ = ((int64_t)p << 32) | (int64_t)(uint32_t)v;
    }
}

// ---------------------------------------------------------------------------
// Finalize: a vertex never reached by the center gets CBFS_UNREACHED and zero
// masks (a cluster source reaching it is a radius violation); a vertex reached
// by the center but not by every source of the cluster is a violation too.
// ---------------------------------------------------------------------------
template <int W, int WC>
__device__ __forceinline__ void finalize_part(const SlotArgs &s, int64_t n, const GroupDesc &g, const OutArgs &o,
                                              int64_t tid, int64_t stride)
{
    const int64_t P = 2 * (int64_t)o.R + 1;
    for (int64_t v = tid; v < n; v += stride) {
        uint64_t sv[W];
        load_words<W>(s.seen + (size_t)v * W, sv);
#pragma unroll
        for (int j = 0; j < W / WC; j++) {
            if (j >= g.nc) break;
            const int32_t c = g.c0 + j;
            const uint64_t *sc = sv + j * WC;
            bool any = false, full = true;
#pragma unroll
            for (int x = 0; x < WC; x++) {
                any |= sc[x] != 0;
                full &= sc[x] == g.full[j * WC + x];
            }
            if (!(sc[0] & 1ull)) {
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

}  // namespace cbfs
