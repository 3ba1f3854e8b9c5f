// Exact 2-hop distance oracle (the paper's appendix on the exact distance
// oracle: pruned landmark labeling, phase 2 run in batches of growing size).
//
// Phase 1 is a C-BFS batch whose center-relative labels (cbfs_labels_pack)
// answer, for a pair, the shortest path through any of its sources.  Phase 2
// runs a pruned BFS from every remaining vertex in rank order.  Roots are cut
// into batches b_0 = first, b_{i+1} = min(max_batch, floor(b_i * growth)); the
// roots of one batch search side by side and all of them prune against the
// index as it stood when the batch began (phase-1 labels plus the 2-hop labels
// of earlier batches), so the labels do not depend on how a batch is spread
// over the device.  At a vertex u reached at distance d from root h, the index
// answer for (h, u) at most d prunes u (no label, no expansion); otherwise
// (rank(h), d) joins u's label and u's neighbours are visited.
//
// Device layout: labels [n][cap] of (rank << 32) | distance, lab_cnt [n];
// the entries of each vertex stay sorted by rank (a batch appends ranks above
// every earlier one, and its own entries are sorted when it ends).  During a
// batch, searches read only the first cnt0[u] entries (the count at batch
// start) and append past them with an atomic counter.
//
// One block per root: the root's 2-hop label sits in an LDS hash (rank ->
// distance) and its phase-1 labels in LDS; the BFS is level-synchronous with
// one thread per frontier vertex, a visited bitmap and two frontier queues
// per search slot in the workspace.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "cbfs.h"
#include "cbfs_internal.h"
#include "cbfs_labels.h"

namespace cbfs {

constexpr int PLL_BLOCK = 256;
constexpr int32_t PLL_EMPTY = -1;

struct PllArgs {
    int64_t n;
    const int32_t *row_ptr, *col;
    int32_t C, R;              // phase-1 clusters (0: none) and their radius
    const uint32_t *bp_dist;   // [n][C]
    const uint64_t *bp_mask;   // [n][C][2R]
    const int32_t *order;      // [count] roots by rank
    int64_t rank0;             // rank of block 0's root
    int32_t cap;               // label capacity per vertex
    int32_t *cnt;              // [n] label sizes (appended to)
    const int32_t *cnt0;       // [n] label sizes when the batch began
    uint64_t *labels;          // [n][cap]
    uint64_t *visited;         // [slots][nwords]
    int32_t *queue;            // [slots][2][n]
    int64_t nwords;
    int32_t hslots;            // LDS hash slots (a power of two >= 2 cap)
    int32_t *err;              // set to 1 when a label overflows cap
};

__device__ __forceinline__ uint32_t pll_hash(int32_t r, int32_t hslots)
{
    return ((uint32_t)r * 2654435761u) & (uint32_t)(hslots - 1);
}

__global__ __launch_bounds__(PLL_BLOCK) void k_pll_bfs(PllArgs a)
{
    extern __shared__ uint64_t pll_lds[];
    const int32_t H = a.hslots;
    const int32_t CL = a.C * 2 * a.R;  // phase-1 mask words per vertex
    int32_t *hkeys = reinterpret_cast<int32_t *>(pll_lds);
    uint32_t *hvals = reinterpret_cast<uint32_t *>(hkeys + H);
    uint64_t *rmask = reinterpret_cast<uint64_t *>(hvals + H);   // [C][2R], 8-byte aligned: H is even
    uint32_t *rdist = reinterpret_cast<uint32_t *>(rmask + CL);  // [C]
    __shared__ int32_t s_fcnt, s_ncnt;

    const int slot = blockIdx.x;
    const int64_t rank = a.rank0 + blockIdx.x;
    const int32_t h = a.order[rank];
    const int64_t n = a.n;
    uint64_t *vis = a.visited + (size_t)slot * a.nwords;
    int32_t *q0 = a.queue + (size_t)slot * 2 * n;
    int32_t *q1 = q0 + n;

    for (int32_t i = threadIdx.x; i < H; i += PLL_BLOCK) hkeys[i] = PLL_EMPTY;
    for (int64_t w = threadIdx.x; w < a.nwords; w += PLL_BLOCK) vis[w] = 0;
    for (int32_t i = threadIdx.x; i < CL; i += PLL_BLOCK) rmask[i] = a.bp_mask[(size_t)h * CL + i];
    for (int32_t i = threadIdx.x; i < a.C; i += PLL_BLOCK) rdist[i] = a.bp_dist[(size_t)h * a.C + i];
    __syncthreads();
    // the root's 2-hop label (distinct ranks) into the hash
    const uint64_t *lh = a.labels + (size_t)h * a.cap;
    const int32_t nh = a.cnt0[h];
    for (int32_t e = threadIdx.x; e < nh; e += PLL_BLOCK) {
        const uint64_t x = lh[e];
        const int32_t r = (int32_t)(x >> 32);
        uint32_t p = pll_hash(r, H);
        while (atomicCAS(&hkeys[p], PLL_EMPTY, r) != PLL_EMPTY) p = (p + 1) & (uint32_t)(H - 1);
        hvals[p] = (uint32_t)x;
    }
    if (threadIdx.x == 0) {
        q0[0] = h;
        vis[h >> 6] = 1ull << (h & 63);
        s_fcnt = 1;
        s_ncnt = 0;
    }
    __syncthreads();

    // the index's answer for (h, u) is at most d
    auto covered = [&](int32_t u, uint32_t d) -> bool {
        const uint32_t *du = a.bp_dist + (size_t)u * a.C;
        const uint64_t *mu = a.bp_mask + (size_t)u * CL;
        for (int32_t c = 0; c < a.C; c++) {
            const uint32_t v = cluster_pair_value(rdist[c], du[c], rmask + (size_t)c * 2 * a.R,
                                                  mu + (size_t)c * 2 * a.R, a.R);
            if (v <= d) return true;
        }
        const uint64_t *lu = a.labels + (size_t)u * a.cap;
        const int32_t nu = a.cnt0[u];
        for (int32_t e = 0; e < nu; e++) {
            const uint64_t x = lu[e];
            const int32_t r = (int32_t)(x >> 32);
            uint32_t p = pll_hash(r, H);
            while (true) {
                const int32_t k = hkeys[p];
                if (k == r) {
                    if ((uint64_t)hvals[p] + (uint32_t)x <= d) return true;
                    break;
                }
                if (k == PLL_EMPTY) break;
                p = (p + 1) & (uint32_t)(H - 1);
            }
        }
        return false;
    };

    int32_t *cur = q0, *nxt = q1;
    for (uint32_t d = 0;; d++) {
        const int32_t fcnt = s_fcnt;
        if (fcnt == 0) break;  // block-uniform
        for (int32_t i = threadIdx.x; i < fcnt; i += PLL_BLOCK) {
            const int32_t u = cur[i];
            if (covered(u, d)) continue;  // pruned: no label, not expanded
            const int32_t pos = atomicAdd(&a.cnt[u], 1);
            if (pos < a.cap) a.labels[(size_t)u * a.cap + pos] = ((uint64_t)rank << 32) | d;
            else atomicExch(a.err, 1);
            for (int32_t e = a.row_ptr[u]; e < a.row_ptr[u + 1]; e++) {
                const int32_t w = a.col[e];
                const unsigned long long bit = 1ull << (w & 63);
                if (vis[w >> 6] & bit) continue;
                const unsigned long long old = atomicOr(reinterpret_cast<unsigned long long *>(vis + (w >> 6)), bit);
                if (!(old & bit)) nxt[atomicAdd(&s_ncnt, 1)] = w;
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            s_fcnt = s_ncnt;
            s_ncnt = 0;
        }
        __syncthreads();
        int32_t *t = cur;
        cur = nxt;
        nxt = t;
    }
}

__global__ void k_pll_snapshot(const int32_t *cnt, int32_t *cnt0, int64_t n)
{
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
        cnt0[v] = cnt[v];
}

// Sort the entries a batch appended to each label (one thread per vertex; a
// batch adds few entries per vertex) and clamp counts that overflowed.
__global__ void k_pll_sort_new(int32_t *cnt, const int32_t *cnt0, uint64_t *labels, int32_t cap, int64_t n)
{
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        int32_t hi = cnt[v];
        if (hi > cap) {
            hi = cap;
            cnt[v] = cap;
        }
        uint64_t *l = labels + (size_t)v * cap;
        for (int32_t i = cnt0[v] + 1; i < hi; i++) {
            const uint64_t x = l[i];
            int32_t j = i - 1;
            while (j >= cnt0[v] && l[j] > x) {
                l[j + 1] = l[j];
                j--;
            }
            l[j + 1] = x;
        }
    }
}

// One wave per query: the phase-1 answer (lanes over clusters), then each
// lane takes entries of L(s) and finds their rank in L(t) by binary search.
__global__ __launch_bounds__(256) void k_pll_query(int64_t n, int32_t C, int32_t R, const uint32_t *bp_dist,
                                                   const uint64_t *bp_mask, int32_t cap, const int32_t *cnt,
                                                   const uint64_t *labels, int64_t q, const int32_t *qs,
                                                   const int32_t *qt, uint32_t *ans)
{
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (wave >= q) return;  // wave-uniform
    const int32_t s = qs[wave], t = qt[wave];
    const int64_t L = 2 * (int64_t)R;
    uint32_t best = CBFS_UNREACHED;
    for (int32_t c = lane; c < C; c += 64) {
        const uint32_t v = cluster_pair_value(bp_dist[(size_t)s * C + c], bp_dist[(size_t)t * C + c],
                                              bp_mask + ((size_t)s * C + c) * L, bp_mask + ((size_t)t * C + c) * L, R);
        best = v < best ? v : best;
    }
    const uint64_t *ls = labels + (size_t)s * cap, *lt = labels + (size_t)t * cap;
    const int32_t ns = cnt[s], nt = cnt[t];
    for (int32_t i = lane; i < ns; i += 64) {
        const uint64_t x = ls[i];
        const uint32_t r = (uint32_t)(x >> 32);
        int32_t lo = 0, hi = nt;
        while (lo < hi) {
            const int32_t mid = (lo + hi) >> 1;
            if ((uint32_t)(lt[mid] >> 32) < r) lo = mid + 1;
            else hi = mid;
        }
        if (lo < nt && (uint32_t)(lt[lo] >> 32) == r) {
            const uint64_t sum = (uint64_t)(uint32_t)x + (uint32_t)lt[lo];
            if (sum < best) best = (uint32_t)sum;
        }
    }
#pragma unroll
    for (int dd = 32; dd >= 1; dd >>= 1) {
        const uint32_t o = __shfl_xor(best, dd, 64);
        best = o < best ? o : best;
    }
    if (lane == 0) ans[wave] = best;
}

struct PllPlan {
    int32_t first, max_batch, slots;
    double growth;
    int64_t nwords;
    size_t off_visited, off_queue, off_cnt0, off_err, bytes;
};

static cbfs_status pll_plan(int64_t n, const cbfs_pll_params *p, PllPlan *out)
{
    PllPlan P;
    P.first = p && p->first ? p->first : 200;
    P.growth = p && p->growth != 0.0f ? (double)p->growth : 1.5;
    P.max_batch = p && p->max_batch ? p->max_batch : 1000;
    P.slots = p && p->slots ? p->slots : (P.max_batch < 1024 ? P.max_batch : 1024);
    if (n < 1 || P.first < 1 || !(P.growth >= 1.0) || P.max_batch < 1 || P.slots < 1 || P.slots > 65535)
        return fail(CBFS_E_ARG, "cbfs_pll: bad batch parameters");
    P.nwords = (n + 63) / 64;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += (bytes + 255) / 256 * 256;
        return at;
    };
    P.off_visited = take(sizeof(uint64_t) * (size_t)P.nwords * P.slots);
    P.off_queue = take(sizeof(int32_t) * 2 * (size_t)n * P.slots);
    P.off_cnt0 = take(sizeof(int32_t) * (size_t)n);
    P.off_err = take(sizeof(int32_t));
    P.bytes = off;
    *out = P;
    return CBFS_OK;
}

}  // namespace cbfs

using namespace cbfs;

extern "C" size_t cbfs_pll_workspace_size(int64_t n, const cbfs_pll_params *params)
{
    PllPlan P;
    if (pll_plan(n, params, &P) != CBFS_OK) return 0;
    return P.bytes;
}

extern "C" cbfs_status cbfs_pll_build(const cbfs_csr *g, const cbfs_labels *bp, const int32_t *order, int64_t count,
                                      const cbfs_pll_params *params, int32_t label_cap, int32_t *lab_cnt,
                                      uint64_t *labels, void *workspace, size_t workspace_bytes, void *stream)
{
    if (!g || !g->row_ptr || !g->col || g->n < 1 || count < 0 || count > g->n || (count > 0 && !order) ||
        label_cap < 1 || label_cap > CBFS_PLL_LABEL_CAP_MAX || !lab_cnt || !labels || !workspace)
        return fail(CBFS_E_ARG, "cbfs_pll_build: bad argument");
    int32_t C = 0, R = 0;
    if (bp) {
        if (bp->n != g->n || bp->num_clusters < 1 || bp->radius < 0 || !bp->dist_vm ||
            (bp->radius > 0 && !bp->mask_vm))
            return fail(CBFS_E_ARG, "cbfs_pll_build: bad phase-1 labels");
        C = bp->num_clusters;
        R = bp->radius;
        if ((int64_t)C * 2 * R > CBFS_PLL_PHASE1_WORDS_MAX)
            return fail(CBFS_E_ARG, "cbfs_pll_build: phase-1 labels exceed the on-chip budget");
    }
    PllPlan P;
    cbfs_status rc = pll_plan(g->n, params, &P);
    if (rc != CBFS_OK) return rc;
    if (workspace_bytes < P.bytes) return fail(CBFS_E_WORKSPACE, "cbfs_pll_build: workspace too small");
    const hipStream_t st = (hipStream_t)stream;
    char *ws = (char *)workspace;
    int32_t hslots = 2;
    while (hslots < 2 * label_cap) hslots *= 2;
    PllArgs a;
    a.n = g->n;
    a.row_ptr = g->row_ptr;
    a.col = g->col;
    a.C = C;
    a.R = R;
    a.bp_dist = bp ? bp->dist_vm : nullptr;
    a.bp_mask = bp ? bp->mask_vm : nullptr;
    a.order = order;
    a.cap = label_cap;
    a.cnt = lab_cnt;
    a.cnt0 = (const int32_t *)(ws + P.off_cnt0);
    a.labels = labels;
    a.visited = (uint64_t *)(ws + P.off_visited);
    a.queue = (int32_t *)(ws + P.off_queue);
    a.nwords = P.nwords;
    a.hslots = hslots;
    a.err = (int32_t *)(ws + P.off_err);
    const size_t lds = (size_t)hslots * 8 + (size_t)C * 2 * R * 8 + (size_t)C * 4;
    const int vblocks = (int)((g->n + 255) / 256 < 4096 ? (g->n + 255) / 256 : 4096);
    hipError_t e;
    if ((e = hipMemsetAsync(lab_cnt, 0, sizeof(int32_t) * (size_t)g->n, st)) != hipSuccess ||
        (e = hipMemsetAsync(a.err, 0, sizeof(int32_t), st)) != hipSuccess)
        return hip_fail("pll clear", e);
    void *tok;
    prof_begin(CBFS_KERNEL_PLL, st, &tok);
    int64_t b = P.first;
    for (int64_t lo = 0; lo < count;) {
        const int64_t size = b < count - lo ? b : count - lo;
        k_pll_snapshot<<<vblocks, 256, 0, st>>>(lab_cnt, (int32_t *)(ws + P.off_cnt0), g->n);
        for (int64_t c0 = 0; c0 < size; c0 += P.slots) {
            a.rank0 = lo + c0;
            const int64_t blocks = size - c0 < P.slots ? size - c0 : P.slots;
            k_pll_bfs<<<(unsigned)blocks, PLL_BLOCK, lds, st>>>(a);
        }
        k_pll_sort_new<<<vblocks, 256, 0, st>>>(lab_cnt, a.cnt0, labels, label_cap, g->n);
        if ((e = hipGetLastError()) != hipSuccess) {
            prof_end(tok);
            return hip_fail("pll batch", e);
        }
        lo += size;
        const int64_t nb = (int64_t)((double)b * P.growth);
        b = nb < P.max_batch ? nb : P.max_batch;
        if (b < 1) b = 1;
    }
    prof_end(tok);
    int32_t err = 0;
    if ((e = hipMemcpyAsync(&err, a.err, sizeof(int32_t), hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return hip_fail("pll error flag", e);
    if (err) return fail(CBFS_E_WORKSPACE, "cbfs_pll_build: a vertex's label exceeded label_cap");
    return CBFS_OK;
}

extern "C" cbfs_status cbfs_pll_query(const cbfs_labels *bp, int64_t n, int32_t label_cap, const int32_t *lab_cnt,
                                      const uint64_t *labels, int64_t q, const int32_t *s, const int32_t *t,
                                      uint32_t *ans, void *stream)
{
    if (n < 1 || label_cap < 1 || !lab_cnt || !labels || q < 0 || (q > 0 && (!s || !t || !ans)))
        return fail(CBFS_E_ARG, "cbfs_pll_query: bad argument");
    if (bp && (bp->n != n || bp->num_clusters < 1 || bp->radius < 0 || !bp->dist_vm || (bp->radius > 0 && !bp->mask_vm)))
        return fail(CBFS_E_ARG, "cbfs_pll_query: bad phase-1 labels");
    if (q == 0) return CBFS_OK;
    const int64_t blocks = (q * 64 + 255) / 256;
    void *tok;
    prof_begin(CBFS_KERNEL_QUERY, (hipStream_t)stream, &tok);
    k_pll_query<<<(unsigned)blocks, 256, 0, (hipStream_t)stream>>>(
        n, bp ? bp->num_clusters : 0, bp ? bp->radius : 0, bp ? bp->dist_vm : nullptr, bp ? bp->mask_vm : nullptr,
        label_cap, lab_cnt, labels, q, s, t, ans);
    hipError_t e = hipGetLastError();
    prof_end(tok);
    return e == hipSuccess ? CBFS_OK : hip_fail("pll query", e);
}
