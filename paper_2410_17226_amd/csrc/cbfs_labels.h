// Device helper shared by the label queries (landmark labeling, Section 4.2,
// and the exact oracle's phase-1 labels).
#pragma once
#include <cstdint>

#include <hip/hip_runtime.h>

#include "cbfs.h"

namespace cbfs {

// One cluster's answer for (s, t) from center-relative labels: ds = d(c, s),
// dt = d(c, t), ms[a + R] = M_a(s) and mt[b + R] = M_b(t) for offsets
// a, b in [-R, R-1].  Every source x of the cluster has d(x, v) = d(c, v) +
// o_x(v), so the minimum over x of d(x, s) + d(x, t) is ds + dt plus the lowest
// offset sum a + b < 0 whose subsets intersect, else plus 0 (the center).
// CBFS_UNREACHED when either end is unreached.
// Masks of any width (w-bit subsets of a cluster of w sources).
template <typename M>
__device__ __forceinline__ uint32_t cluster_pair_value(uint32_t ds, uint32_t dt, const M *ms, const M *mt, int32_t R)
{
    if (ds == CBFS_UNREACHED || dt == CBFS_UNREACHED) return CBFS_UNREACHED;
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
    return (uint32_t)((int64_t)ds + (int64_t)dt + corr);
}

}  // namespace cbfs
