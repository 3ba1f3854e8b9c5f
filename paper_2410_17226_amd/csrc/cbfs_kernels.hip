// Kernels of the Cluster-BFS level loop (Algorithm "Cluster-BFS search from S",
// with the two EdgeMap directions of Appendix A) for gfx950.
#include <hip/hip_runtime.h>

#include "cbfs_device.h"
#include "cbfs_kernels.h"

namespace cbfs {

// ---------------------------------------------------------------------------
// Merge-path partition of (rows, arcs) into pull tiles of TILE_ITEMS items
// (Merrill & Garland's merge-based decomposition): tile t starts at diagonal
// t*TILE_ITEMS; (row, edge) is the split where row ends row_ptr[1..] merge
// with arc indices 0..m-1.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void merge_path_search(int64_t diag, const int32_t *row_end, int64_t n, int64_t m,
                                                  int32_t *row, int32_t *edge)
{
    int64_t lo = diag > m ? diag - m : 0;
    int64_t hi = diag < n ? diag : n;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if ((int64_t)row_end[mid] <= diag - mid - 1) lo = mid + 1;
        else hi = mid;
    }
    *row = (int32_t)lo;
    *edge = (int32_t)(diag - lo);
}

__global__ void k_tiles(const int32_t *row_ptr, int64_t n, int64_t m, int32_t ntiles, int32_t *tile_row,
                        int32_t *tile_edge)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t > ntiles) return;
    int64_t diag = t * TILE_ITEMS;
    if (diag > n + m) diag = n + m;
    merge_path_search(diag, row_ptr + 1, n, m, tile_row + t, tile_edge + t);
}

// ---------------------------------------------------------------------------
// Init: clear one group slot; cluster statuses of the group to CBFS_OK.
// ---------------------------------------------------------------------------
template <int W>
__global__ void k_init(SlotArgs s, int64_t n, GroupDesc g, OutArgs o)
{
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
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
    if (tid < 12) s.ctr[tid] = 0;
    if (tid < g.nc) o.status[g.c0 + tid] = 0;
}

// Seed: bit i of cluster j at its source s_i (Seen_0), and F_0 = the sources.
// One block; sources/cluster_ptr are the batch's arrays in device memory.
template <int W, int WC>
__global__ void k_seed(SlotArgs s, GraphArgs gr, GroupDesc g, const int32_t *sources,
                       const int32_t *cluster_ptr)
{
    __shared__ Stager st;
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
    stager_flush(st, s.q0, s.ctr + 0);
}

// ---------------------------------------------------------------------------
// Round i, push direction (EdgeMap-Sparse).  Each block takes BLOCK queue
// entries (pieces of <= PIECE arcs), runs the vertex phase for first pieces,
// then spreads the block's arcs evenly over its threads (block scan + binary
// search of the arc's owner).  Per arc (u, v): x = Seen_i(u) \ Seen_i(v); if
// not empty, 64-bit atomic OR into nxt(v) and claim v (Fetch_And_Or + CAS of
// the paper).  Blocks past the queue only clear the round-(i+2) bitmap.
// ---------------------------------------------------------------------------
template <int W, int WC>
__global__ __launch_bounds__(BLOCK) void k_push(SlotArgs s, GraphArgs gr, GroupDesc g, OutArgs o, int32_t round,
                                                int64_t nq)
{
    __shared__ int s_scan[BLOCK + 1];
    __shared__ int32_t s_estart[BLOCK];
    __shared__ uint64_t s_cu[BLOCK * W];
    __shared__ int s_tmp[WAVES + 1];
    __shared__ Stager st;

    // clear the bitmap and counters two rounds ahead (dead since round i-1)
    {
        uint64_t *clr = bits_buf(s, (round + 2) % 3);
        const int64_t tid = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
        for (int64_t k = tid; k < s.nwords; k += (int64_t)gridDim.x * BLOCK) clr[k] = 0;
        if (tid < 4) ctr_buf(s, round + 2)[tid] = 0;
    }
    const int64_t first = (int64_t)blockIdx.x * BLOCK;
    if (first >= nq) return;  // block-uniform

    stager_init(st);
    const uint64_t *cur = cur_buf(s, round);
    uint64_t *nxt = nxt_buf(s, round);
    uint64_t *bits_next = bits_buf(s, (round + 1) % 3);
    int64_t *q_next = q_buf(s, round + 1);
    unsigned long long *ctr_next = ctr_buf(s, round + 1);

    int cnt = 0;
    const int64_t idx = first + threadIdx.x;
    if (idx < nq) {
        const int64_t e = q_buf(s, round)[idx];
        const int32_t u = (int32_t)(e & 0xffffffff);
        const int32_t p = (int32_t)(e >> 32);
        const int32_t rs = gr.row_ptr[u], re = gr.row_ptr[u + 1];
        const int32_t lo = rs + p * PIECE;
        const int32_t hi = re < lo + PIECE ? re : lo + PIECE;
        cnt = hi > lo ? hi - lo : 0;
        uint64_t cu[W];
        load_words<W>(cur + (size_t)u * W, cu);
        if (p == 0) vertex_phase<W, WC>(s, g, o, gr.n, round, u, cu);
        s_estart[threadIdx.x] = lo;
#pragma unroll
        for (int w = 0; w < W; w++) s_cu[threadIdx.x * W + w] = cu[w];
    }
    int total;
    const int off = block_exclusive_scan(cnt, s_tmp, &total);
    s_scan[threadIdx.x] = off;
    if (threadIdx.x == 0) s_scan[BLOCK] = total;
    __syncthreads();

    for (int base = 0; base < total; base += BLOCK) {
        const int e = base + threadIdx.x;
        if (e < total) {
            // owner: last j with s_scan[j] <= e (pieces with zero arcs share offsets)
            int lo = 0, hi = BLOCK;
            while (hi - lo > 1) {
                int mid = (lo + hi) >> 1;
                if (s_scan[mid] <= e) lo = mid;
                else hi = mid;
            }
            const int32_t v = gr.col[s_estart[lo] + (e - s_scan[lo])];
            uint64_t cv[W], x[W];
            load_words<W>(cur + (size_t)v * W, cv);
            bool any = false;
#pragma unroll
            for (int w = 0; w < W; w++) {
                x[w] = s_cu[lo * W + w] & ~cv[w];
                any |= x[w] != 0;
            }
            if (any) contribute<W>(st, nxt, bits_next, gr.row_ptr, v, x);
        }
        __syncthreads();
        if (st.count > STAGE_CAP - BLOCK) stager_flush(st, q_next, ctr_next);
    }
    stager_flush(st, q_next, ctr_next);
}

// ---------------------------------------------------------------------------
// Round i, pull direction (EdgeMap-Dense).  Blocks [0, nvb) run the vertex
// phase over the queue's first pieces; blocks [nvb, nvb + ntiles) each take a
// merge-path tile of the CSR: the tile's arcs are staged in LDS with
// coalesced loads, every thread walks TILE_ITEMS/BLOCK consecutive items
// (arcs or row ends), OR-ing Seen_i(u) of frontier neighbours u into a
// register accumulator that starts from Seen_i(v); a row stops early once the
// accumulator holds every source (the break of EdgeMap-Dense).  At a row end
// (or the thread's last item) the bits not yet in Seen_i(v) are merged into
// nxt(v) with atomics, since a row may span threads and tiles.
// ---------------------------------------------------------------------------
template <int W, int WC>
__global__ __launch_bounds__(BLOCK) void k_pull(SlotArgs s, GraphArgs gr, GroupDesc g, OutArgs o, int32_t round,
                                                int64_t nq, int32_t nvb)
{
    __shared__ int32_t s_col[TILE_ITEMS];
    __shared__ Stager st;

    {
        uint64_t *clr = bits_buf(s, (round + 2) % 3);
        const int64_t tid = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
        for (int64_t k = tid; k < s.nwords; k += (int64_t)gridDim.x * BLOCK) clr[k] = 0;
        if (tid < 4) ctr_buf(s, round + 2)[tid] = 0;
    }
    const uint64_t *cur = cur_buf(s, round);
    if ((int32_t)blockIdx.x < nvb) {
        const int64_t idx = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
        if (idx < nq) {
            const int64_t e = q_buf(s, round)[idx];
            if ((e >> 32) == 0) {
                const int32_t u = (int32_t)(e & 0xffffffff);
                uint64_t cu[W];
                load_words<W>(cur + (size_t)u * W, cu);
                vertex_phase<W, WC>(s, g, o, gr.n, round, u, cu);
            }
        }
        return;
    }
    const int32_t t = (int32_t)blockIdx.x - nvb;
    const int32_t r0 = gr.tile_row[t], e0 = gr.tile_edge[t];
    const int32_t r1 = gr.tile_row[t + 1], e1 = gr.tile_edge[t + 1];
    stager_init(st);
    for (int32_t k = threadIdx.x; k < e1 - e0; k += BLOCK) s_col[k] = gr.col[e0 + k];
    __syncthreads();

    uint64_t *nxt = nxt_buf(s, round);
    const uint64_t *bits_cur = bits_buf(s, round % 3);
    uint64_t *bits_next = bits_buf(s, (round + 1) % 3);
    const int32_t *row_end = gr.row_ptr + 1;

    // this thread's merge-path start inside the tile
    const int32_t tile_rows = r1 - r0, tile_edges = e1 - e0;
    const int32_t tile_items = tile_rows + tile_edges;
    int32_t rel = (int32_t)threadIdx.x * IPT;
    if (rel > tile_items) rel = tile_items;
    int32_t my_end = ((int32_t)threadIdx.x + 1) * IPT;
    if (my_end > tile_items) my_end = tile_items;
    int32_t row, edge;
    {
        int32_t lo = rel > tile_edges ? rel - tile_edges : 0;
        int32_t hi = rel < tile_rows ? rel : tile_rows;
        while (lo < hi) {
            int32_t mid = (lo + hi) >> 1;
            if (row_end[r0 + mid] - e0 <= rel - mid - 1) lo = mid + 1;
            else hi = mid;
        }
        row = r0 + lo;
        edge = e0 + (rel - lo);
    }

    uint64_t full[W];
#pragma unroll
    for (int w = 0; w < W; w++) full[w] = g.full[w];

    uint64_t cv[W], acc[W];
    int32_t rend = 0;
    bool have_row = false, done_row = false;
    for (int it = 0; it < IPT; it++) {
        if (rel < my_end) {
            if (!have_row) {
                load_words<W>(cur + (size_t)row * W, cv);
                rend = row_end[row];
                bool fin = true;
#pragma unroll
                for (int w = 0; w < W; w++) {
                    acc[w] = 0;
                    fin &= cv[w] == full[w];
                }
                done_row = fin;
                have_row = true;
            }
            if (edge < rend) {
                if (!done_row) {
                    const int32_t u = s_col[edge - e0];
                    if ((bits_cur[u >> 6] >> (u & 63)) & 1ull) {
                        uint64_t cu[W];
                        load_words<W>(cur + (size_t)u * W, cu);
                        bool fin = true;
#pragma unroll
                        for (int w = 0; w < W; w++) {
                            acc[w] |= cu[w] & ~cv[w];
                            fin &= (acc[w] | cv[w]) == full[w];
                        }
                        done_row = fin;
                    }
                }
                edge++;
            } else {
                // row end: merge what this thread found for `row`
                bool any = false;
#pragma unroll
                for (int w = 0; w < W; w++) any |= acc[w] != 0;
                if (any) contribute<W>(st, nxt, bits_next, gr.row_ptr, row, acc);
                row++;
                have_row = false;
            }
            rel++;
        }
        // at most one claim per thread per item: keep room for the next one
        __syncthreads();
        if (st.count > STAGE_CAP - BLOCK) stager_flush(st, q_buf(s, round + 1), ctr_buf(s, round + 1));
    }
    // partial row at the thread's end
    if (have_row) {
        bool any = false;
#pragma unroll
        for (int w = 0; w < W; w++) any |= acc[w] != 0;
        if (any) contribute<W>(st, nxt, bits_next, gr.row_ptr, row, acc);
    }
    stager_flush(st, q_buf(s, round + 1), ctr_buf(s, round + 1));
}

// ---------------------------------------------------------------------------
// Finalize: a vertex never reached by the center gets CBFS_UNREACHED and zero
// masks (a cluster source reaching it is a radius violation); a vertex reached
// by the center but not by every source of the cluster is a violation too.
// ---------------------------------------------------------------------------
template <int W, int WC>
__global__ void k_finalize(SlotArgs s, int64_t n, GroupDesc g, OutArgs o)
{
    const int64_t P = 2 * (int64_t)o.R + 1;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
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

// ---------------------------------------------------------------------------
// Host-side launchers (dispatch on the template parameters).
// ---------------------------------------------------------------------------
#define CBFS_DISPATCH(W_, WC_, CALL)                                     \
    do {                                                                 \
        if ((W_) == 1 && (WC_) == 1) { constexpr int W = 1, WC = 1; CALL; } \
        else if ((W_) == 3 && (WC_) == 3) { constexpr int W = 3, WC = 3; CALL; } \
        else if ((W_) == 2 && (WC_) == 1) { constexpr int W = 2, WC = 1; CALL; } \
        else if ((W_) == 2 && (WC_) == 2) { constexpr int W = 2, WC = 2; CALL; } \
        else if ((W_) == 4 && (WC_) == 1) { constexpr int W = 4, WC = 1; CALL; } \
        else if ((W_) == 4 && (WC_) == 2) { constexpr int W = 4, WC = 2; CALL; } \
        else if ((W_) == 4 && (WC_) == 4) { constexpr int W = 4, WC = 4; CALL; } \
        else if ((W_) == 8 && (WC_) == 1) { constexpr int W = 8, WC = 1; CALL; } \
        else if ((W_) == 8 && (WC_) == 2) { constexpr int W = 8, WC = 2; CALL; } \
        else if ((W_) == 8 && (WC_) == 4) { constexpr int W = 8, WC = 4; CALL; } \
        else return hipErrorInvalidValue;                                \
    } while (0)

static int clear_blocks(int64_t nwords) { return (int)((nwords + BLOCK * 16 - 1) / (BLOCK * 16)) + 1; }

hipError_t launch_tiles(const int32_t *row_ptr, int64_t n, int64_t m, int32_t ntiles, int32_t *tile_row,
                        int32_t *tile_edge, hipStream_t st)
{
    k_tiles<<<(ntiles + 1 + BLOCK - 1) / BLOCK, BLOCK, 0, st>>>(row_ptr, n, m, ntiles, tile_row, tile_edge);
    return hipGetLastError();
}

hipError_t launch_init(int W, const SlotArgs &s, int64_t n, const GroupDesc &g, const OutArgs &o, hipStream_t st)
{
    int64_t words = n * W;
    int blocks = (int)std::min<int64_t>(4096, (words + BLOCK - 1) / BLOCK + 1);
    CBFS_DISPATCH(W, (W == 3 ? 3 : 1), ((void)WC, k_init<W><<<blocks, BLOCK, 0, st>>>(s, n, g, o)));
    return hipGetLastError();
}

hipError_t launch_seed(int W, int WC, const SlotArgs &s, const GraphArgs &gr, const GroupDesc &g,
                       const int32_t *sources, const int32_t *cluster_ptr, hipStream_t st)
{
    CBFS_DISPATCH(W, WC, (k_seed<W, WC><<<1, BLOCK, 0, st>>>(s, gr, g, sources, cluster_ptr)));
    return hipGetLastError();
}

hipError_t launch_push(int W, int WC, const SlotArgs &s, const GraphArgs &gr, const GroupDesc &g,
                       const OutArgs &o, int32_t round, int64_t nq, hipStream_t st)
{
    int64_t work = (nq + BLOCK - 1) / BLOCK;
    int64_t blocks = std::max<int64_t>(work, clear_blocks(s.nwords));
    CBFS_DISPATCH(W, WC, (k_push<W, WC><<<(unsigned)blocks, BLOCK, 0, st>>>(s, gr, g, o, round, nq)));
    return hipGetLastError();
}

hipError_t launch_pull(int W, int WC, const SlotArgs &s, const GraphArgs &gr, const GroupDesc &g,
                       const OutArgs &o, int32_t round, int64_t nq, hipStream_t st)
{
    int32_t nvb = (int32_t)((nq + BLOCK - 1) / BLOCK);
    int64_t blocks = (int64_t)nvb + gr.ntiles;
    CBFS_DISPATCH(W, WC, (k_pull<W, WC><<<(unsigned)blocks, BLOCK, 0, st>>>(s, gr, g, o, round, nq, nvb)));
    return hipGetLastError();
}

hipError_t launch_finalize(int W, int WC, const SlotArgs &s, int64_t n, const GroupDesc &g, const OutArgs &o,
                           hipStream_t st)
{
    int blocks = (int)std::min<int64_t>(8192, (n + BLOCK - 1) / BLOCK);
    CBFS_DISPATCH(W, WC, (k_finalize<W, WC><<<blocks, BLOCK, 0, st>>>(s, n, g, o)));
    return hipGetLastError();
}

}  // namespace cbfs
