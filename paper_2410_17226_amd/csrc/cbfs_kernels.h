// Launchers of the Cluster-BFS kernels (host side of cbfs_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "cbfs_device.h"

namespace cbfs {

constexpr int MAX_SLOTS = 64;  // group slots searched side by side in one persistent launch
constexpr int GRAB = 4;        // work items a persistent block takes per counter update
constexpr int DIES = 8;        // accelerator dies (XCDs), each with its own L2
// Barrier control words, one 128-byte line each: generation, die-leader
// arrivals, then per die: arrivals, registered blocks, die generation.
constexpr int CTL_LINE = 32;   // words per line
constexpr int CTL_GEN = 0, CTL_COUNT = 1, CTL_DIE_COUNT = 2, CTL_DIE_TOTAL = 2 + DIES,
              CTL_DIE_GEN = 2 + 2 * DIES;
constexpr int CTL_WORDS = CTL_LINE * (2 + 3 * DIES);

// Per-group statistics the persistent kernel keeps: rounds, push rounds,
// pull rounds, sum |F_i|, sum deg(F_i), sum |F_i| over pull rounds.
constexpr int STAT_WORDS = 6;

// Arguments of the persistent batch kernel (all pointers are device memory).
struct PersistArgs {
    GraphArgs gr;
    OutArgs o;
    const SlotArgs *slots;      // [num_slots]
    const GroupDesc *groups;    // [num_groups]
    int32_t num_groups, num_slots;
    const int32_t *sources;     // batch sources
    const int32_t *cluster_ptr; // batch cluster_ptr
    unsigned int *ctl;          // [CTL_WORDS] barrier state, work counters (zeroed before launch)
    unsigned long long *work;   // [3 * DIES] per-round work counters of each die
    int32_t *err;               // 0 ok, 1 barrier timeout, 2 round limit
    long long *stats;           // [num_groups][STAT_WORDS]
    float alpha, beta, gamma;
    int32_t force_pull;
    int32_t schedule;           // 0 fixed stride, 1 shared work counter
    int64_t max_rounds;
};

hipError_t launch_tiles(const int32_t *row_ptr, int64_t n, int64_t m, int32_t ntiles, int32_t *tile_row,
                        int32_t *tile_edge, hipStream_t st);
hipError_t launch_init(int W, const SlotArgs &s, int64_t n, const GroupDesc &g, const OutArgs &o, hipStream_t st);
hipError_t launch_seed(int W, int WC, const SlotArgs &s, const GraphArgs &gr, const GroupDesc &g,
                       const int32_t *sources, const int32_t *cluster_ptr, int32_t num_sources, hipStream_t st);
hipError_t launch_push(int W, int WC, const SlotArgs &s, const GraphArgs &gr, const GroupDesc &g,
                       const OutArgs &o, int32_t round, int64_t nq, int64_t degsum, hipStream_t st);
// Push round for a frontier of at most HUB_MAX vertices (nq queue entries):
// lists them into hubs[0 .. hubs[HUB_MAX]) (HUB_MAX + 1 ints of device
// memory), then one block per HUB_RANGE target vertices.
hipError_t launch_push_hub(int W, int WC, const SlotArgs &s, const GraphArgs &gr, const GroupDesc &g,
                           const OutArgs &o, int32_t round, int64_t nq, int64_t degsum, int32_t *hubs,
                           int32_t *bounds, hipStream_t st);
hipError_t launch_pull(int W, int WC, const SlotArgs &s, const GraphArgs &gr, const GroupDesc &g,
                       const OutArgs &o, int32_t round, int32_t form, bool queue, hipStream_t st);
// The queue of F_round from its bitmap (after rounds that left only the
// bitmap and the counters).
hipError_t launch_build_queue(const SlotArgs &s, const GraphArgs &gr, int32_t round, hipStream_t st);
hipError_t launch_finalize(int W, int WC, const SlotArgs &s, int64_t n, const GroupDesc &g, const OutArgs &o,
                           hipStream_t st);
// Status clean-up after a batch: every cluster whose status is not CBFS_OK
// gets dist = CBFS_UNREACHED and zero masks; with *abort_flag != 0 (nullable)
// every cluster first gets CBFS_E_HIP.
hipError_t launch_scrub(const OutArgs &o, int64_t n, int32_t C, int32_t WC, const int32_t *abort_flag,
                        hipStream_t st);
// Blocks of the persistent kernel on the current device: per_cu per compute
// unit (0 = as many as can be resident), capped at what can be resident.
hipError_t persistent_grid(int W, int WC, int per_cu, int *blocks);
hipError_t launch_persistent(int W, int WC, const PersistArgs &a, int blocks, hipStream_t st);

}  // namespace cbfs
