// Landmark-labeling queries over cluster labels (Section 4.2, "Answering
// Queries with Clustered Landmarks"; Algorithm "Framework of Landmark
// Labeling", Query).
//
// For one cluster with center-relative labels (dist d(c,.), offset subsets
// M_o(.), o in [-R, R]), every source x has d(x,s) = d(c,s) + o_x(s), so
//   min_x d(x,s) + d(x,t) = d(c,s) + d(c,t) + min_x (o_x(s) + o_x(t)).
// The center has offset 0 at both ends, so the minimum is at most 0, and only
// pairs (a, b) with a + b < 0 can lower it.  Such a pair has a, b <= R - 1
// (the other offset is at least -R), so the +R plane is never needed: the
// labels keep planes -R .. R-1 (2R of them), and the correction is the lowest
// sum a + b < 0 with M_a(s) & M_b(t) non-empty, else 0.  For R = 1 this is
// -2 if M_-1(s) & M_-1(t), else -1 if M_-1(s) & M_0(t) or M_0(s) & M_-1(t),
// else 0.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "cbfs.h"
#include "cbfs_internal.h"
#include "cbfs_labels.h"

namespace cbfs {

// Cluster-major outputs -> vertex-major labels (planes -R .. R-1).  One thread
// per (cluster, vertex) pair, cluster-major order, so the reads of each plane
// are coalesced.
__global__ void k_labels_pack(const uint32_t *dist, const uint64_t *masks, int32_t C, int64_t n, int32_t R,
                              uint32_t *dist_vm, uint64_t *mask_vm)
{
    const int64_t P = 2 * (int64_t)R + 1;
    const int64_t L = 2 * (int64_t)R;
    const int64_t total = (int64_t)C * n;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = k / n, v = k - c * n;
        dist_vm[v * C + c] = dist[k];
        uint64_t *dst = mask_vm + (v * C + c) * L;
        for (int64_t p = 0; p < L; p++) dst[p] = masks[(c * P + p) * n + v];
    }
}

// One wave per query; lanes stride over clusters, then a wave min-reduction.
__global__ __launch_bounds__(256) void k_query(int64_t n, int32_t C, int32_t R, const uint32_t *dist_vm,
                                               const uint64_t *mask_vm, int64_t q, const int32_t *qs,
                                               const int32_t *qt, uint32_t *ans)
{
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (wave >= q) return;  // wave-uniform
    const int64_t L = 2 * (int64_t)R;  // planes kept per cluster: offsets -R .. R-1
    const int64_t s = qs[wave], t = qt[wave];
    const uint32_t *ds_row = dist_vm + s * C, *dt_row = dist_vm + t * C;
    const uint64_t *ms_row = mask_vm + s * C * L, *mt_row = mask_vm + t * C * L;
    uint32_t best = CBFS_UNREACHED;
    for (int32_t c = lane; c < C; c += 64) {
        // ms[a + R] = M_a(s), a in [-R, R-1]
        const uint32_t val = cluster_pair_value(ds_row[c], dt_row[c], ms_row + (int64_t)c * L,
                                                mt_row + (int64_t)c * L, R);
        best = val < best ? val : best;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const uint32_t o = __shfl_xor(best, d, 64);
        best = o < best ? o : best;
    }
    if (lane == 0) ans[wave] = best;
}


// ---------------------------------------------------------------------------
// Compact labels: the storage the paper gives a cluster distance vector under a
// memory budget (Section 5.3, landmark labeling experiments): a one-byte
// distance and the 2R subsets as w-bit words, w in {8, 16, 32, 64} the
// cluster's source count bound; 1 + 2R w / 8 bytes per cluster and vertex.
// Distance 255 means unreached.
__device__ int g_pack_err;  // set by a pack that met a distance >= 255 or a source bit >= w

template <typename M>
__global__ void k_labels_pack_compact(const uint32_t *dist, const uint64_t *masks, int32_t C, int64_t n, int32_t R,
                                      uint8_t *dist8, M *mask_c)
{
    constexpr int WBITS = 8 * sizeof(M);
    const int64_t P = 2 * (int64_t)R + 1;
    const int64_t L = 2 * (int64_t)R;
    const int64_t total = (int64_t)C * n;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = k / n, v = k - c * n;
        const uint32_t d = dist[k];
        if (d != CBFS_UNREACHED && d >= 255) atomicExch(&g_pack_err, 1);
        dist8[v * C + c] = d == CBFS_UNREACHED || d >= 255 ? (uint8_t)255 : (uint8_t)d;
        M *dst = mask_c + (v * C + c) * L;
        for (int64_t p = 0; p < L; p++) {
            const uint64_t m = masks[(c * P + p) * n + v];
            if (WBITS < 64 && (m >> (WBITS % 64)) != 0) atomicExch(&g_pack_err, 1);
            dst[p] = (M)m;
        }
    }
}

template <typename M>
__global__ __launch_bounds__(256) void k_query_compact(int32_t C, int32_t R, const uint8_t *dist8, const M *mask_c,
                                                       int64_t q, const int32_t *qs, const int32_t *qt, uint32_t *ans)
{
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (wave >= q) return;  // wave-uniform
    const int64_t L = 2 * (int64_t)R;
    const int64_t s = qs[wave], t = qt[wave];
    uint32_t best = CBFS_UNREACHED;
    for (int32_t c = lane; c < C; c += 64) {
        const uint8_t ds = dist8[s * C + c], dt = dist8[t * C + c];
        const uint32_t val = cluster_pair_value<M>(ds == 255 ? CBFS_UNREACHED : ds, dt == 255 ? CBFS_UNREACHED : dt,
                                                   mask_c + (s * C + c) * L, mask_c + (t * C + c) * L, R);
        best = val < best ? val : best;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const uint32_t o = __shfl_xor(best, d, 64);
        best = o < best ? o : best;
    }
    if (lane == 0) ans[wave] = best;
}

// ---------------------------------------------------------------------------
// Bidirectional local search of the query path (Appendix B, "Applying
// Bi-Directional Search in the Queries"): from each endpoint, the first tau
// vertices a FIFO BFS discovers (root first, then the neighbours of each
// dequeued vertex in row order), each with its exact distance; the answer is
// the lowest d(s,x) + d(t,x) over the vertices both searches found.
//
// One wave per query (a block of 64 threads), everything in LDS:
//   keys[H], vals[H]  open-addressing set of the vertices one side has seen
//                     (H >= 1.5 (tau + LS_STEP), so it never fills);
//   ls/lsd[tau]       s side's discovery list and distances (kept for the
//                     intersection), lt/ltd[tau] the t side's.
// The search scans the arcs of up to 64 queued vertices as one concatenated
// run, LS_STEP = 64 LS_ARCS consecutive arcs per step (arc 64 r + lane of the
// step on lane `lane`, r < LS_ARCS), numbered in the order the sequential
// search would scan them.  A neighbour seen for
// the first time in a step may occur on several arcs; the earliest arc is its
// discoverer, found with an LDS atomic min of the arc numbers on its slot, and
// discoverers take list positions by ballot rank in arc order, which
// reproduces the sequential discovery order.  Positions >= tau are dropped
// (the sequential search stops there); their keys stay in the set marked
// dropped, so the set holds at most tau + LS_STEP - 1 keys.
//
// vals states: PENDING (inserted in this step, owner not decided), an arc
// number < LS_STEP (owner being decided), KEPT | dist, DROPPED.
constexpr uint32_t LS_PENDING = 0xFFFFFFFFu;
constexpr uint32_t LS_DROPPED = 0xFFFFFFFEu;
constexpr uint32_t LS_KEPT = 0x80000000u;
constexpr int32_t LS_EMPTY = -1;
constexpr int LS_ARCS = 1;                 // arcs per lane per step (4 measured no faster)
constexpr int32_t LS_STEP = 64 * LS_ARCS;  // arcs per step

// Multiplicative hash scaled to [0, H) (H need not be a power of two).
__device__ __forceinline__ uint32_t ls_hash(int32_t v, uint32_t H)
{
    return (uint32_t)(((uint64_t)((uint32_t)v * 2654435761u) * H) >> 32);
}

__device__ __forceinline__ bool ls_kept(uint32_t val) { return (val >> 30) == 2u; }

// Slot of v, inserting v if absent (lanes racing for one empty slot: the CAS
// lets one key in, the others probe on unless they carry the same key).
__device__ __forceinline__ uint32_t ls_insert(int32_t *keys, uint32_t H, int32_t v)
{
    uint32_t slot = ls_hash(v, H);
    while (true) {
        const int32_t k = keys[slot];
        if (k == v) return slot;
        if (k == LS_EMPTY) {
            const int32_t old = atomicCAS(&keys[slot], LS_EMPTY, v);
            if (old == LS_EMPTY || old == v) return slot;
        }
        slot = slot + 1 == H ? 0u : slot + 1;
    }
}

__device__ __forceinline__ uint32_t ls_find(const int32_t *keys, const uint32_t *vals, uint32_t H, int32_t v)
{
    uint32_t slot = ls_hash(v, H);
    while (true) {
        const int32_t k = keys[slot];
        if (k == v) return vals[slot];
        if (k == LS_EMPTY) return LS_DROPPED;
        slot = slot + 1 == H ? 0u : slot + 1;
    }
}

// tau-bounded FIFO BFS from root; leaves its set in keys/vals and its
// discovery list in list/listd; returns the list length.  Wave-uniform.
__device__ int32_t ls_search(const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col, int32_t root,
                             int32_t tau, uint32_t H, int32_t *keys, uint32_t *vals, int32_t *list,
                             uint16_t *listd, int32_t *pre_excl, int32_t *pre_base, int32_t *pre_dist)
{
    const int lane = threadIdx.x;
    for (uint32_t i = lane; i < H; i += 64) {
        keys[i] = LS_EMPTY;
        vals[i] = LS_PENDING;
    }
    __syncthreads();
    if (lane == 0) {
        const uint32_t slot = ls_insert(keys, H, root);
        vals[slot] = LS_KEPT;
        list[0] = root;
        listd[0] = 0;
    }
    __syncthreads();
    int32_t cnt = 1, head = 0;
    while (head < cnt && cnt < tau) {
        const int32_t gend = head + 64 < cnt ? head + 64 : cnt;
        const int32_t gn = gend - head;
        int32_t deg = 0, base = 0, pd = 0;
        if (lane < gn) {
            const int32_t u = list[head + lane];
            base = row_ptr[u];
            deg = row_ptr[u + 1] - base;
            pd = listd[head + lane];
        }
        int32_t incl = deg;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int32_t o = __shfl_up(incl, d, 64);
            if (lane >= d) incl += o;
        }
        const int32_t total = __shfl(incl, 63, 64);
        pre_excl[lane] = incl - deg;
        pre_base[lane] = base;
        pre_dist[lane] = pd + 1;
        __syncthreads();
        for (int32_t a0 = 0; a0 < total && cnt < tau; a0 += LS_STEP) {
            int32_t v[LS_ARCS], dv[LS_ARCS];
            uint32_t slot[LS_ARCS];
            bool fresh[LS_ARCS];
            int32_t lo = 0;
#pragma unroll
            for (int r = 0; r < LS_ARCS; r++) {  // owners, then the column reads, all in flight together
                const int32_t g = a0 + 64 * r + lane;
                v[r] = -1;
                dv[r] = 0;
                if (g < total) {
                    int32_t hi = gn - 1;  // the last queued vertex whose arcs start at or before g
                    while (lo < hi) {
                        const int32_t mid = (lo + hi + 1) >> 1;
                        if (pre_excl[mid] <= g) lo = mid;
                        else hi = mid - 1;
                    }
                    v[r] = col[pre_base[lo] + (g - pre_excl[lo])];
                    dv[r] = pre_dist[lo];
                }
            }
#pragma unroll
            for (int r = 0; r < LS_ARCS; r++) slot[r] = v[r] >= 0 ? ls_insert(keys, H, v[r]) : 0u;
            __syncthreads();
#pragma unroll
            for (int r = 0; r < LS_ARCS; r++) fresh[r] = v[r] >= 0 && vals[slot[r]] == LS_PENDING;
            __syncthreads();
#pragma unroll
            for (int r = 0; r < LS_ARCS; r++)
                if (fresh[r]) atomicMin(&vals[slot[r]], (uint32_t)(64 * r + lane));
            __syncthreads();
            uint64_t won[LS_ARCS];
#pragma unroll
            for (int r = 0; r < LS_ARCS; r++) {
                fresh[r] = fresh[r] && vals[slot[r]] == (uint32_t)(64 * r + lane);  // the earliest arc
                won[r] = __ballot(fresh[r]);
            }
            __syncthreads();
            const uint64_t below = (1ull << lane) - 1ull;
#pragma unroll
            for (int r = 0; r < LS_ARCS; r++) {
                if (fresh[r]) {
                    const int32_t pos = cnt + (int32_t)__popcll(won[r] & below);
                    if (pos < tau) {
                        list[pos] = v[r];
                        listd[pos] = (uint16_t)dv[r];
                        vals[slot[r]] = LS_KEPT | (uint32_t)dv[r];
                    } else {
                        vals[slot[r]] = LS_DROPPED;
                    }
                }
                cnt += (int32_t)__popcll(won[r]);
            }
            cnt = cnt < tau ? cnt : tau;
            __syncthreads();
        }
        head = gend;
    }
    return cnt;
}

__global__ __launch_bounds__(64) void k_local_search(const int32_t *__restrict__ row_ptr,
                                                     const int32_t *__restrict__ col, int64_t q,
                                                     const int32_t *qs, const int32_t *qt, int32_t tau,
                                                     uint32_t H, uint32_t *ans)
{
    extern __shared__ int32_t lds[];
    int32_t *keys = lds;
    uint32_t *vals = (uint32_t *)(keys + H);
    int32_t *pre_excl = (int32_t *)(vals + H);
    int32_t *pre_base = pre_excl + 64;
    int32_t *pre_dist = pre_base + 64;
    int32_t *ls = pre_dist + 64;
    int32_t *lt = ls + tau;
    uint16_t *lsd = (uint16_t *)(lt + tau);
    uint16_t *ltd = lsd + tau;
    const int lane = threadIdx.x;
    for (int64_t j = blockIdx.x; j < q; j += gridDim.x) {
        const int32_t cs = ls_search(row_ptr, col, qs[j], tau, H, keys, vals, ls, lsd, pre_excl, pre_base,
                                     pre_dist);
        ls_search(row_ptr, col, qt[j], tau, H, keys, vals, lt, ltd, pre_excl, pre_base, pre_dist);
        uint32_t best = CBFS_UNREACHED;
        for (int32_t k = lane; k < cs; k += 64) {
            const uint32_t val = ls_find(keys, vals, H, ls[k]);
            if (ls_kept(val)) {
                const uint32_t c = (uint32_t)lsd[k] + (val & ~LS_KEPT);
                best = c < best ? c : best;
            }
        }
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
            const uint32_t o = __shfl_xor(best, d, 64);
            best = o < best ? o : best;
        }
        if (lane == 0 && best < ans[j]) ans[j] = best;
        __syncthreads();
    }
}

// Set slots for a given tau: 1.5 times the most keys one side inserts (tau
// kept + LS_STEP - 1 dropped), rounded up to a multiple of 64; and the LDS
// bytes of one k_local_search block.
static uint32_t local_set_slots(int32_t tau)
{
    const int64_t need = (3 * ((int64_t)tau + LS_STEP) + 1) / 2;
    return (uint32_t)((need + 63) / 64 * 64);
}

static size_t local_lds_bytes(int32_t tau, uint32_t H)
{
    return (size_t)H * 8 + 3 * 64 * 4 + (size_t)tau * 2 * 4 + (size_t)tau * 2 * 2;
}

}  // namespace cbfs

using namespace cbfs;

extern "C" cbfs_status cbfs_labels_pack(const uint32_t *dist, const uint64_t *masks, int32_t num_clusters,
                                        int64_t n, int32_t radius, uint32_t *dist_vm, uint64_t *mask_vm,
                                        void *stream)
{
    if (!dist || !masks || !dist_vm || (radius > 0 && !mask_vm) || num_clusters < 1 || n < 1 || radius < 0 ||
        radius > 1024)
        return fail(CBFS_E_ARG, "cbfs_labels_pack: bad argument");
    const int64_t total = (int64_t)num_clusters * n;
    const int blocks = (int)((total + 255) / 256 < 65536 ? (total + 255) / 256 : 65536);
    void *tok;
    prof_begin(CBFS_KERNEL_LABELS, (hipStream_t)stream, &tok);
    k_labels_pack<<<blocks, 256, 0, (hipStream_t)stream>>>(dist, masks, num_clusters, n, radius, dist_vm, mask_vm);
    hipError_t e = hipGetLastError();
    prof_end(tok);
    return e == hipSuccess ? CBFS_OK : hip_fail("labels_pack", e);
}

extern "C" cbfs_status cbfs_query_batch(const cbfs_labels *L, int64_t q, const int32_t *s, const int32_t *t,
                                        uint32_t *ans, void *stream)
{
    if (!L || !L->dist_vm || (L->radius > 0 && !L->mask_vm) || L->n < 1 || L->num_clusters < 1 || L->radius < 0 ||
        L->radius > 1024 || q < 0 || (q > 0 && (!s || !t || !ans)))
        return fail(CBFS_E_ARG, "cbfs_query_batch: bad argument");
    if (q == 0) return CBFS_OK;
    const int64_t blocks = (q * 64 + 255) / 256;
    void *tok;
    prof_begin(CBFS_KERNEL_QUERY, (hipStream_t)stream, &tok);
    k_query<<<(unsigned)blocks, 256, 0, (hipStream_t)stream>>>(L->n, L->num_clusters, L->radius, L->dist_vm,
                                                                 L->mask_vm, q, s, t, ans);
    hipError_t e = hipGetLastError();
    prof_end(tok);
    return e == hipSuccess ? CBFS_OK : hip_fail("query", e);
}

extern "C" cbfs_status cbfs_query_local(const cbfs_csr *g, int64_t q, const int32_t *s, const int32_t *t,
                                        int32_t tau, uint32_t *ans, void *stream)
{
    if (!g || !g->row_ptr || !g->col || g->n < 1 || g->m < 0 || q < 0 || tau < 1 || tau > CBFS_LOCAL_TAU_MAX ||
        (q > 0 && (!s || !t || !ans)))
        return fail(CBFS_E_ARG, "cbfs_query_local: bad argument");
    if (q == 0) return CBFS_OK;
    const uint32_t H = local_set_slots(tau);
    const size_t lds = local_lds_bytes(tau, H);
    const int64_t blocks = q < (1 << 20) ? q : (1 << 20);
    void *tok;
    prof_begin(CBFS_KERNEL_LOCAL, (hipStream_t)stream, &tok);
    k_local_search<<<(unsigned)blocks, 64, lds, (hipStream_t)stream>>>(g->row_ptr, g->col, q, s, t, tau, H, ans);
    hipError_t e = hipGetLastError();
    prof_end(tok);
    return e == hipSuccess ? CBFS_OK : hip_fail("query_local", e);
}

extern "C" cbfs_status cbfs_labels_pack_compact(const uint32_t *dist, const uint64_t *masks, int32_t num_clusters,
                                                int64_t n, int32_t radius, int32_t w, uint8_t *dist8, void *masks_out,
                                                void *stream)
{
    if (!dist || (radius > 0 && (!masks || !masks_out)) || !dist8 || num_clusters < 1 || n < 1 || radius < 0 ||
        radius > 1024 || (w != 8 && w != 16 && w != 32 && w != 64))
        return fail(CBFS_E_ARG, "cbfs_labels_pack_compact: bad argument");
    const hipStream_t st = (hipStream_t)stream;
    const int zero = 0;
    hipError_t e;
    if ((e = hipMemcpyToSymbolAsync(HIP_SYMBOL(g_pack_err), &zero, sizeof(int), 0, hipMemcpyHostToDevice, st)) !=
        hipSuccess)
        return hip_fail("compact pack flag", e);
    const int64_t total = (int64_t)num_clusters * n;
    const int blocks = (int)((total + 255) / 256 < 65536 ? (total + 255) / 256 : 65536);
    void *tok;
    prof_begin(CBFS_KERNEL_LABELS, st, &tok);
    switch (w) {
    case 8: k_labels_pack_compact<uint8_t><<<blocks, 256, 0, st>>>(dist, masks, num_clusters, n, radius, dist8,
                                                                    (uint8_t *)masks_out); break;
    case 16: k_labels_pack_compact<uint16_t><<<blocks, 256, 0, st>>>(dist, masks, num_clusters, n, radius, dist8,
                                                                      (uint16_t *)masks_out); break;
    case 32: k_labels_pack_compact<uint32_t><<<blocks, 256, 0, st>>>(dist, masks, num_clusters, n, radius, dist8,
                                                                      (uint32_t *)masks_out); break;
    default: k_labels_pack_compact<uint64_t><<<blocks, 256, 0, st>>>(dist, masks, num_clusters, n, radius, dist8,
                                                                      (uint64_t *)masks_out); break;
    }
    e = hipGetLastError();
    prof_end(tok);
    if (e != hipSuccess) return hip_fail("labels_pack_compact", e);
    int err = 0;
    if ((e = hipMemcpyFromSymbolAsync(&err, HIP_SYMBOL(g_pack_err), sizeof(int), 0, hipMemcpyDeviceToHost, st)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return hip_fail("compact pack flag", e);
    if (err) return fail(CBFS_E_RANGE, "cbfs_labels_pack_compact: a distance >= 255 or a source beyond w");
    return CBFS_OK;
}

extern "C" cbfs_status cbfs_query_batch_compact(const cbfs_compact_labels *L, int64_t q, const int32_t *s,
                                                const int32_t *t, uint32_t *ans, void *stream)
{
    if (!L || !L->dist8 || (L->radius > 0 && !L->masks) || L->n < 1 || L->num_clusters < 1 || L->radius < 0 ||
        L->radius > 1024 || (L->w != 8 && L->w != 16 && L->w != 32 && L->w != 64) || q < 0 ||
        (q > 0 && (!s || !t || !ans)))
        return fail(CBFS_E_ARG, "cbfs_query_batch_compact: bad argument");
    if (q == 0) return CBFS_OK;
    const int64_t blocks = (q * 64 + 255) / 256;
    const hipStream_t st = (hipStream_t)stream;
    void *tok;
    prof_begin(CBFS_KERNEL_QUERY, st, &tok);
    switch (L->w) {
    case 8: k_query_compact<uint8_t><<<(unsigned)blocks, 256, 0, st>>>(L->num_clusters, L->radius, L->dist8,
                                                                        (const uint8_t *)L->masks, q, s, t, ans); break;
    case 16: k_query_compact<uint16_t><<<(unsigned)blocks, 256, 0, st>>>(L->num_clusters, L->radius, L->dist8,
                                                                          (const uint16_t *)L->masks, q, s, t, ans); break;
    case 32: k_query_compact<uint32_t><<<(unsigned)blocks, 256, 0, st>>>(L->num_clusters, L->radius, L->dist8,
                                                                          (const uint32_t *)L->masks, q, s, t, ans); break;
    default: k_query_compact<uint64_t><<<(unsigned)blocks, 256, 0, st>>>(L->num_clusters, L->radius, L->dist8,
                                                                          (const uint64_t *)L->masks, q, s, t, ans); break;
    }
    hipError_t e = hipGetLastError();
    prof_end(tok);
    return e == hipSuccess ? CBFS_OK : hip_fail("query_compact", e);
}
