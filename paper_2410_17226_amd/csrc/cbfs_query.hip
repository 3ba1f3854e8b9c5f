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
        const uint32_t ds = ds_row[c], dt = dt_row[c];
        if (ds == CBFS_UNREACHED || dt == CBFS_UNREACHED) continue;
        const uint64_t *ms = ms_row + (int64_t)c * L;  // ms[a + R] = M_a(s), a in [-R, R-1]
        const uint64_t *mt = mt_row + (int64_t)c * L;
        int32_t corr = 0;
        for (int32_t sum = -2 * R; sum < 0 && corr == 0; sum++) {
            const int32_t alo = sum - (R - 1) > -R ? sum - (R - 1) : -R;  // b = sum - a <= R - 1
            const int32_t ahi = sum + R < R - 1 ? sum + R : R - 1;        // b >= -R
            for (int32_t a = alo; a <= ahi; a++) {
                if (ms[a + R] & mt[sum - a + R]) {
                    corr = sum;
                    break;
                }
            }
        }
        const uint32_t val = (uint32_t)((int64_t)ds + (int64_t)dt + corr);
        best = val < best ? val : best;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const uint32_t o = __shfl_xor(best, d, 64);
        best = o < best ? o : best;
    }
    if (lane == 0) ans[wave] = best;
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
