// Launchers of the Cluster-BFS kernels (host side of cbfs_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "cbfs_device.h"

namespace cbfs {

hipError_t launch_tiles(const int32_t *row_ptr, int64_t n, int64_t m, int32_t ntiles, int32_t *tile_row,
                        int32_t *tile_edge, hipStream_t st);
hipError_t launch_init(int W, const SlotArgs &s, int64_t n, const GroupDesc &g, const OutArgs &o, hipStream_t st);
hipError_t launch_seed(int W, int WC, const SlotArgs &s, const GraphArgs &gr, const GroupDesc &g,
                       const int32_t *sources, const int32_t *cluster_ptr, hipStream_t st);
hipError_t launch_push(int W, int WC, const SlotArgs &s, const GraphArgs &gr, const GroupDesc &g,
                       const OutArgs &o, int32_t round, int64_t nq, hipStream_t st);
hipError_t launch_pull(int W, int WC, const SlotArgs &s, const GraphArgs &gr, const GroupDesc &g,
                       const OutArgs &o, int32_t round, int64_t nq, hipStream_t st);
hipError_t launch_finalize(int W, int WC, const SlotArgs &s, int64_t n, const GroupDesc &g, const OutArgs &o,
                           hipStream_t st);

}  // namespace cbfs
