// Kernels of the Cluster-BFS level loop (Algorithm "Cluster-BFS search from S",
// with the two EdgeMap directions of Appendix A) for gfx950:
//   - one launch per step (init / seed / round / finalize), driven by the host;
//   - one persistent cooperative launch that runs the whole batch, with the
//     level loop and the direction choice on the device and grid barriers
//     between rounds.
#include <hip/hip_runtime.h>

#include "cbfs_kernels.h"
#include "cbfs_round.h"

namespace cbfs {

// ---------------------------------------------------------------------------
// Merge-path partition of (rows, arcs) into pull tiles of TILE_ITEMS items
// (Merrill & Garland's merge-based decomposition): tile t starts at diagonal
// t*TILE_ITEMS; (row, edge) is the split where row ends row_ptr[1..] merge
// with arc indices 0..m-1.
// ---------------------------------------------------------------------------
__global__ void k_tiles(const int32_t *row_ptr, int64_t n, int64_t m, int32_t ntiles, int32_t *tile_row,
                        int32_t *tile_edge)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t > ntiles) return;
    int64_t diag = t * TILE_ITEMS;
    if (diag > n + m) diag = n + m;
    const int32_t *row_end = row_ptr + 1;
    int64_t lo = diag > m ? diag - m : 0;
    int64_t hi = diag < n ? diag : n;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if ((int64_t)row_end[mid] <= diag - mid - 1) lo = mid + 1;
        else hi = mid;
    }
    tile_row[t] = (int32_t)lo;
    tile_edge[t] = (int32_t)(diag - lo);
}

// ---------------------------------------------------------------------------
// One launch per step.
// ---------------------------------------------------------------------------
template <int W>
__global__ void k_init(SlotArgs s, int64_t n, GroupDesc g, OutArgs o)
{
    init_part<W>(s, n, g, o, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, (int64_t)gridDim.x * blockDim.x);
}

template <int W, int WC>
__global__ __launch_bounds__(BLOCK) void k_seed(SlotArgs s, GraphArgs gr, GroupDesc g, const int32_t *sources,
                                                const int32_t *cluster_ptr)
{
    __shared__ Stager<STAGE_CAP> st;
    seed_block<W, WC>(st, s, gr, g, sources, cluster_ptr, blockIdx.x, gridDim.x, SEED_PER_BLOCK);
}

template <int W, int WC>
__global__ __launch_bounds__(BLOCK) void k_push(SlotArgs s, GraphArgs gr, GroupDesc g, OutArgs o, int32_t round,
                                                int64_t nq, int32_t epb)
{
    __shared__ PushSmem<W> sm;
    clear_ahead_part(s, round, (int64_t)blockIdx.x * BLOCK + threadIdx.x, (int64_t)gridDim.x * BLOCK);
    push_chunk<W, WC>(sm, s, gr, g, o, round, nq, blockIdx.x, epb);
}

// The frontier's vertices (entries of piece 0) listed for the range-owned
// push: hubs[0 .. hubs[HUB_MAX]), in no particular order (the push does not
// depend on it); hubs[HUB_MAX] starts at zero and counts the slots.
__global__ __launch_bounds__(BLOCK) void k_hub_list(SlotArgs s, int32_t round, int64_t nq, int32_t *hubs)
{
    const int64_t k = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (k >= nq) return;
    const int64_t e = q_buf(s, round)[k];
    if ((e >> 32) != 0) return;
    const int slot = atomicAdd(hubs + HUB_MAX, 1);
    if (slot < HUB_MAX) hubs[slot] = (int32_t)(e & 0xffffffff);
}

__global__ __launch_bounds__(BLOCK) void k_hub_bounds(GraphArgs gr, const int32_t *hubs, int32_t *bounds,
                                                      int64_t stride)
{
    __shared__ HubBoundsSmem sm;
    hub_bounds_block(sm, gr, hubs, bounds, stride);
}

template <int W, int WC>
__global__ __launch_bounds__(BLOCK) void k_push_hub(SlotArgs s, GraphArgs gr, GroupDesc g, OutArgs o, int32_t round,
                                                    const int32_t *hubs, const int32_t *bounds, int64_t stride)
{
    __shared__ HubSmem<W> sm;
    clear_ahead_part(s, round, (int64_t)blockIdx.x * BLOCK + threadIdx.x, (int64_t)gridDim.x * BLOCK);
    push_hub_block<W, WC>(sm, s, gr, g, o, round, hubs, bounds, stride, blockIdx.x);
}

__global__ __launch_bounds__(BLOCK) void k_bits_to_queue(SlotArgs s, GraphArgs gr, int32_t fround, int32_t what)
{
    __shared__ BitsQueueSmem sm;
    bits_to_queue_block(sm, s, gr, fround, what);
}

template <int W, int WC>
__global__ __launch_bounds__(BLOCK) void k_pull(SlotArgs s, GraphArgs gr, GroupDesc g, OutArgs o, int32_t round,
                                               int32_t form, int32_t queue)
{
    __shared__ PullSmem<W> sm;
    clear_ahead_part(s, round, (int64_t)blockIdx.x * BLOCK + threadIdx.x, (int64_t)gridDim.x * BLOCK);
    pull_tile<W, WC>(sm, s, gr, g, o, round, blockIdx.x, form, queue != 0);
}

template <int W, int WC>
__global__ void k_finalize(SlotArgs s, int64_t n, GroupDesc g, OutArgs o)
{
    finalize_part<W, WC>(s, n, g, o, (int64_t)blockIdx.x * blockDim.x + threadIdx.x,
                         (int64_t)gridDim.x * blockDim.x);
}

// The outputs of a cluster whose status is not CBFS_OK are defined as
// dist = CBFS_UNREACHED and every mask word 0 (its search was cut short or
// its radius did not hold, so no partial result is handed back).  With
// abort_flag set (the persistent kernel stopped early), every cluster of the
// batch gets CBFS_E_HIP first.  Grid (x, C): blocks of cluster blockIdx.y
// stride over its dist row and its 2R+1 contiguous mask planes.
__global__ __launch_bounds__(BLOCK) void k_scrub(OutArgs o, int64_t n, int32_t WC, const int32_t *abort_flag)
{
    const int32_t c = blockIdx.y;
    const bool aborted = abort_flag && *abort_flag != 0;
    if (!aborted && o.status[c] == 0) return;  // block-uniform
    __syncthreads();  // every thread has read the status before it is overwritten
    if (aborted && blockIdx.x == 0 && threadIdx.x == 0) o.status[c] = E_HIP;
    const int64_t tid = (int64_t)blockIdx.x * BLOCK + threadIdx.x, stride = (int64_t)gridDim.x * BLOCK;
    uint32_t *d = o.dist + (size_t)c * (size_t)n;
    for (int64_t v = tid; v < n; v += stride) d[v] = UNREACHED;
    const int64_t words = planes_of(o) * n * WC;
    uint64_t *m = o.masks + (size_t)c * (size_t)words;
    for (int64_t k = tid; k < words; k += stride) m[k] = 0;
}

// ---------------------------------------------------------------------------
// Persistent batch kernel.
// ---------------------------------------------------------------------------

// Barriers of the cooperative launch, where every block is resident.
//
// One flat barrier over all blocks registers each block on its die (XCD, read
// from HW_REG_XCC_ID).  After that the work is partitioned by die, and each
// level of the search ends in a barrier over the blocks of one die only: every
// block waits for its own stores to reach L2 and counts itself in; the last
// arrival releases at agent scope (the die's dirty L2 lines go out) and opens
// the die's next generation; every block then acquires at agent scope before
// reading the level's results.  Arrivals and polls are relaxed atomics,
// performed coherently without touching cached data.  The waits are bounded:
// after BARRIER_TIMEOUT_TICKS of the constant-rate wall clock (or once another
// block has aborted) a block raises the abort flag, and every block leaves its
// loops at the next check, so the grid always drains.
constexpr unsigned long long BARRIER_TIMEOUT_TICKS = 400000000ull;  // 4 s at 100 MHz

__device__ __forceinline__ unsigned int ld_relaxed(const unsigned int *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Bounded wait until *p != old (thread 0 only).  Returns false on timeout/abort.
__device__ __forceinline__ bool wait_change(const unsigned int *p, unsigned int old, int32_t *abort_flag)
{
    const unsigned long long t0 = wall_clock64();
    unsigned int naps = 1;
    while (ld_relaxed(p) == old) {
        for (unsigned int k = 0; k < naps; k++) __builtin_amdgcn_s_sleep(4);
        if (naps < 16) naps <<= 1;
        if (wall_clock64() - t0 > BARRIER_TIMEOUT_TICKS ||
            __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
            __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
    }
    return true;
}

__device__ __forceinline__ unsigned int die_id()
{
    return __builtin_amdgcn_s_getreg(20 | (0 << 6) | (3 << 11)) & (DIES - 1);  // HW_REG_XCC_ID[3:0]
}

// Flat barrier over all blocks, used once to register the blocks of each die.
__device__ bool flat_barrier(unsigned int *ctl, unsigned int nblocks, int32_t *abort_flag, int32_t &s_abort)
{
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned int *gen = ctl + CTL_LINE * CTL_GEN, *count = ctl + CTL_LINE * CTL_COUNT;
        const unsigned int g = ld_relaxed(gen);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (__hip_atomic_fetch_add(count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == nblocks - 1) {
            __hip_atomic_store(count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __hip_atomic_fetch_add(gen, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            wait_change(gen, g, abort_flag);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        s_abort = __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
    }
    __syncthreads();
    return s_abort != 0;
}

// Barrier over the blocks of one die: the last arrival releases (agent scope)
// and opens the die's next generation; every block then acquires (agent
// scope).  Blocks of other dies are not involved.
__device__ __forceinline__ bool die_barrier(unsigned int *ctl, unsigned int die, unsigned int dtotal,
                                            int32_t *abort_flag, int32_t &s_abort)
{
    __builtin_amdgcn_s_waitcnt(0);  // this wave's stores have reached L2
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned int *dcount = ctl + CTL_LINE * (CTL_DIE_COUNT + die);
        unsigned int *dgen = ctl + CTL_LINE * (CTL_DIE_GEN + die);
        const unsigned int dg = ld_relaxed(dgen);
        if (__hip_atomic_fetch_add(dcount, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == dtotal - 1) {
            __hip_atomic_store(dcount, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __hip_atomic_fetch_add(dgen, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            wait_change(dgen, dg, abort_flag);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        // one read of the flag for the whole block, so every wave takes the same exit
        s_abort = __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
    }
    __syncthreads();
    return s_abort != 0;
}

__device__ __forceinline__ unsigned long long ld_ctr(const unsigned long long *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Block-uniform: copy the descriptors of slot `slot` (holding group `group`)
// into LDS, where the global stores of the round cannot alias them, and
// record which local slot they hold.  Every write of these LDS words happens
// here, between two barriers, so every wave reads the same values afterwards.
__device__ __forceinline__ void load_desc(const PersistArgs &a, int32_t slot, int32_t group, int32_t tag,
                                          SlotArgs &s_slot, GroupDesc &s_group, int32_t &s_cached)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        s_slot = a.slots[slot];
        s_group = a.groups[group];
        s_cached = tag;
    }
    __syncthreads();
}

// The batch, partitioned by die: after one device-wide registration, the
// groups are dealt to the dies that have blocks (group g to die rank g mod
// nd) and so are the slots (die rank r owns slots [r*spd, (r+1)*spd)).  Each
// die runs its own level loop over its slots with its own barrier, so no
// data moves between dies during the search, a die's L2 holds only its own
// groups' frontiers, and a die never waits for another.
template <int W, int WC>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(3, 8))) void k_persistent(PersistArgs a)
{
    __shared__ RoundSmem<W> sm;
    __shared__ int32_t s_dense[MAX_SLOTS];
    __shared__ int32_t s_done[MAX_SLOTS];   // frontier emptied: the slot's counters are no longer maintained
    __shared__ int32_t s_sparse[MAX_SLOTS];
    __shared__ int64_t s_work[MAX_SLOTS];   // push chunks or pull tiles
    __shared__ int64_t s_nq[MAX_SLOTS];     // pieces in F_i
    __shared__ int32_t s_epb[MAX_SLOTS];    // queue entries per push chunk
    __shared__ int32_t s_pulls[MAX_SLOTS];  // dense rounds so far
    __shared__ int64_t s_nprev[MAX_SLOTS];  // pieces in F_{i-1}
    __shared__ int64_t s_pref[MAX_SLOTS + 1];
    __shared__ int tmp[WAVES + 1];
    __shared__ int32_t s_stop;
    __shared__ int64_t s_grab;
    __shared__ SlotArgs s_slot;
    __shared__ GroupDesc s_group;
    __shared__ int32_t s_cached;
    __shared__ int32_t s_abort;
    __shared__ uint32_t s_dix, s_ndies, s_drank, s_dtotal;

    const unsigned int die = die_id();
    // register this block on its die (its index there), then learn the dies
    if (threadIdx.x == 0)
        s_dix = __hip_atomic_fetch_add(a.ctl + CTL_LINE * (CTL_DIE_TOTAL + die), 1u, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
    bool aborted = flat_barrier(a.ctl, gridDim.x, a.err, s_abort);
    if (threadIdx.x == 0) {
        uint32_t k = 0, r = 0;
        for (int d = 0; d < DIES; d++)
            if (ld_relaxed(a.ctl + CTL_LINE * (CTL_DIE_TOTAL + d)) > 0) {
                if ((unsigned int)d < die) r++;
                k++;
            }
        s_ndies = k;
        s_drank = r;
        s_dtotal = ld_relaxed(a.ctl + CTL_LINE * (CTL_DIE_TOTAL + die));
    }
    __syncthreads();
    const int32_t S = a.num_slots;
    const int32_t nd = (int32_t)s_ndies < S ? (int32_t)s_ndies : S;  // dies that take groups
    const int32_t drank = (int32_t)s_drank;
    const unsigned int dtotal = s_dtotal, dix = s_dix;
    if (aborted || drank >= nd) return;  // block-uniform; no later barrier counts this die
    const int32_t spd = S / nd;           // slots of this die
    const int32_t slot0 = drank * spd;
    const int32_t Gd = a.num_groups > drank ? (a.num_groups - drank + nd - 1) / nd : 0;
    const int64_t dtid = (int64_t)dix * BLOCK + threadIdx.x;
    const int64_t dstride = (int64_t)dtotal * BLOCK;
    unsigned long long *work = a.work + 3 * die;

    for (int32_t q0 = 0; q0 < Gd && !aborted; q0 += spd) {
        const int32_t active = Gd - q0 < spd ? Gd - q0 : spd;
        auto group_of = [&](int32_t sl) { return drank + nd * (q0 + sl); };
        for (int32_t sl = 0; sl < active; sl++) {
            load_desc(a, slot0 + sl, group_of(sl), sl, s_slot, s_group, s_cached);
            init_part<W>(s_slot, a.gr.n, s_group, a.o, dtid, dstride);
        }
        if (dix == 0 && threadIdx.x < 3) work[threadIdx.x] = 0;
        if ((aborted = die_barrier(a.ctl, die, dtotal, a.err, s_abort))) break;
        for (int32_t sl = (int32_t)dix; sl < active; sl += (int32_t)dtotal) {
            load_desc(a, slot0 + sl, group_of(sl), sl, s_slot, s_group, s_cached);
            seed_block<W, WC>(sm.push.st, s_slot, a.gr, s_group, a.sources, a.cluster_ptr);
        }
        if (threadIdx.x < MAX_SLOTS) {
            s_dense[threadIdx.x] = a.force_pull ? 1 : 0;
            s_pulls[threadIdx.x] = 0;
            s_done[threadIdx.x] = 0;
        }
        if ((aborted = die_barrier(a.ctl, die, dtotal, a.err, s_abort))) break;

        for (int32_t round = 0;; round++) {
            // Decision: thread sl reads slot sl's counters (F_i and F_{i-1});
            // every block of the die takes the same decisions from the same values.
            int64_t items = 0, wk = 0;
            const int32_t sl_me = threadIdx.x;
            if (sl_me < active && !s_done[sl_me]) {
                const SlotArgs &sd = a.slots[slot0 + sl_me];
                const unsigned long long *c = ctr_buf(sd, round);
                const int64_t pieces = (int64_t)ld_ctr(c + 0), verts = (int64_t)ld_ctr(c + 1),
                              degsum = (int64_t)ld_ctr(c + 2);
                const int64_t nprev = round > 0 ? (int64_t)ld_ctr(ctr_buf(sd, round - 1) + 0) : 0;
                if (verts > 0) {
                    // direction choice (Appendix A, Algorithm "EdgeMap")
                    int32_t dense = s_dense[sl_me];
                    if (a.force_pull) dense = 1;
                    else if (a.alpha < 0.f) dense = 0;
                    else if (!dense) dense = (double)(verts + degsum) > (double)a.gr.m / a.alpha;
                    else dense = (double)verts > (double)a.gr.n / a.beta;
                    // 2: the wave form over every neighbour (first dense round with
                    // a frontier carrying most arcs), 1: the walking form
                    if (dense && s_pulls[sl_me] == 0 && a.gamma > 0.f &&
                        (double)degsum > (double)a.gamma * (double)a.gr.m)
                        dense = 2;
                    else if (dense)
                        dense = 1;
                    if (dense) s_pulls[sl_me]++;
                    s_dense[sl_me] = dense;
                    const int32_t epb = push_entries_per_block(pieces, degsum);
                    s_epb[sl_me] = epb;
                    wk = dense ? a.gr.ntiles : (pieces + epb - 1) / epb;
                    // bitmap words of F_{i-1} to clear: sparse through its queue
                    // when that is cheaper than a dense pass
                    const bool sparse = nprev * 4 < sd.nwords;
                    s_sparse[sl_me] = sparse;
                    const int64_t clears = round == 0 ? 0
                                           : (sparse ? (nprev + BLOCK - 1) / BLOCK
                                                     : (sd.nwords + CLEAR_WORDS - 1) / CLEAR_WORDS);
                    items = wk + clears;
                    if (dix == 0) {
                        long long *st = a.stats + STAT_WORDS * (int64_t)group_of(sl_me);
                        st[0] += 1;
                        st[dense ? 2 : 1] += 1;
                        st[3] += verts;
                        st[4] += degsum;
                        if (dense) st[5] += verts;
                    }
                }
                if (verts == 0) s_done[sl_me] = 1;
                s_work[sl_me] = wk;
                s_nq[sl_me] = pieces;
                s_nprev[sl_me] = nprev;
            } else if (sl_me < active) {
                s_work[sl_me] = 0;
            }
            // items of the slots, in slot order (active <= MAX_SLOTS <= BLOCK)
            int total_work;
            block_exclusive_scan(wk > 0 ? 1 : 0, tmp, &total_work);
            {
                // 64-bit prefix of the item counts over the first `active` threads
                const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
                int64_t v = items;
#pragma unroll
                for (int d = 1; d < 64; d <<= 1) {
                    const int64_t y = __shfl_up(v, d, 64);
                    if (lane >= d) v += y;
                }
                // MAX_SLOTS <= 64: the slots all sit in wave 0
                if (wid == 0 && threadIdx.x < active) s_pref[threadIdx.x + 1] = v;
                if (threadIdx.x == 0) {
                    s_pref[0] = 0;
                    s_stop = total_work == 0 ? 1 : (round > a.max_rounds ? 2 : 0);
                    if (s_stop == 2 && dix == 0)
                        __hip_atomic_store(a.err, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
            __syncthreads();
            if (s_stop) break;
            // the work counter of round i+2 last served round i-1
            if (dix == 0 && threadIdx.x == 0) work[(round + 2) % 3] = 0;
            // the die's blocks take items at a fixed stride of one (or GRAB at a
            // time from the round's counter), items being slot-major: push
            // chunks or pull tiles, then bitmap clears
            const int64_t total = s_pref[active];
            unsigned long long *wctr = work + (round % 3);
            const int64_t grab = a.schedule == 1 ? GRAB : 1;
            int32_t sl = 0;
            for (int64_t next = (int64_t)dix * grab;; next += (int64_t)dtotal * grab) {
                if (a.schedule == 1) {
                    if (threadIdx.x == 0) s_grab = (int64_t)atomicAdd(wctr, (unsigned long long)GRAB);
                    __syncthreads();
                    next = s_grab;
                    __syncthreads();
                }
                const int64_t first = next;
                if (first >= total) break;
                const int64_t last = first + grab < total ? first + grab : total;
                for (int64_t item = first; item < last; item++) {
                    if (item < s_pref[sl]) sl = 0;
                    while (item >= s_pref[sl + 1]) sl++;
                    const int64_t local = item - s_pref[sl];
                    if (sl != s_cached) load_desc(a, slot0 + sl, group_of(sl), sl, s_slot, s_group, s_cached);
                    if (local >= s_work[sl]) {
                        __syncthreads();
                        clear_item(s_slot, round, s_sparse[sl] != 0, s_nprev[sl], local - s_work[sl]);
                    } else if (s_dense[sl]) {
                        pull_tile<W, WC>(sm.pull, s_slot, a.gr, s_group, a.o, round, (int32_t)local,
                                         s_dense[sl] == 2 ? PULL_WAVE : PULL_WALK);
                    } else {
                        push_chunk<W, WC>(sm.push, s_slot, a.gr, s_group, a.o, round, s_nq[sl], local, s_epb[sl]);
                    }
                }
            }
            if ((aborted = die_barrier(a.ctl, die, dtotal, a.err, s_abort))) break;
        }
        if (aborted) break;
        for (int32_t sl = 0; sl < active; sl++) {
            load_desc(a, slot0 + sl, group_of(sl), sl, s_slot, s_group, s_cached);
            finalize_part<W, WC>(s_slot, a.gr.n, s_group, a.o, dtid, dstride);
        }
        if ((aborted = die_barrier(a.ctl, die, dtotal, a.err, s_abort))) break;
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
        else if ((W_) == 16 && (WC_) == 1) { constexpr int W = 16, WC = 1; CALL; } \
        else if ((W_) == 16 && (WC_) == 2) { constexpr int W = 16, WC = 2; CALL; } \
        else if ((W_) == 16 && (WC_) == 4) { constexpr int W = 16, WC = 4; CALL; } \
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
                       const int32_t *sources, const int32_t *cluster_ptr, int32_t num_sources, hipStream_t st)
{
    const int blocks = std::max(1, (num_sources + SEED_PER_BLOCK - 1) / SEED_PER_BLOCK);
    CBFS_DISPATCH(W, WC, (k_seed<W, WC><<<blocks, BLOCK, 0, st>>>(s, gr, g, sources, cluster_ptr)));
    return hipGetLastError();
}

hipError_t launch_push(int W, int WC, const SlotArgs &s, const GraphArgs &gr, const GroupDesc &g,
                       const OutArgs &o, int32_t round, int64_t nq, int64_t degsum, hipStream_t st)
{
    const int32_t epb = push_entries_per_block(nq, degsum);
    int64_t work = (nq + epb - 1) / epb;
    int64_t blocks = std::max<int64_t>(work, clear_blocks(s.nwords));
    CBFS_DISPATCH(W, WC, (k_push<W, WC><<<(unsigned)blocks, BLOCK, 0, st>>>(s, gr, g, o, round, nq, epb)));
    return hipGetLastError();
}

hipError_t launch_push_hub(int W, int WC, const SlotArgs &s, const GraphArgs &gr, const GroupDesc &g,
                           const OutArgs &o, int32_t round, int64_t nq, int64_t degsum, int32_t *hubs,
                           int32_t *bounds, hipStream_t st)
{
    // the host guarantees at most HUB_MAX frontier vertices
    hipError_t e = hipMemsetAsync(hubs + HUB_MAX, 0, sizeof(int32_t), st);
    if (e != hipSuccess) return e;
    if (nq > 0) {
        k_hub_list<<<(unsigned)((nq + BLOCK - 1) / BLOCK), BLOCK, 0, st>>>(s, round, nq, hubs);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // the slice starts of every (frontier vertex, owned range); the blocks
    // stride over the arcs, so the degree sum only sizes the grid
    const int64_t stride = hub_bounds_stride(gr.n);
    const int64_t bb = std::min<int64_t>(std::max<int64_t>(1, (degsum + HB_CHUNK - 1) / HB_CHUNK), 4096);
    k_hub_bounds<<<(unsigned)bb, BLOCK, 0, st>>>(gr, hubs, bounds, stride);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int64_t blocks = std::max<int64_t>((gr.n + HUB_RANGE - 1) / HUB_RANGE, clear_blocks(s.nwords));
    CBFS_DISPATCH(W, WC, (k_push_hub<W, WC><<<(unsigned)blocks, BLOCK, 0, st>>>(s, gr, g, o, round, hubs, bounds,
                                                                                 stride)));
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int64_t per_block = (int64_t)BLOCK * BQ_VPT;
    k_bits_to_queue<<<(unsigned)((gr.n + per_block - 1) / per_block), BLOCK, 0, st>>>(s, gr, round + 1, BITS_COUNT);
    return hipGetLastError();
}

hipError_t launch_build_queue(const SlotArgs &s, const GraphArgs &gr, int32_t round, hipStream_t st)
{
    const int64_t per_block = (int64_t)BLOCK * BQ_VPT;
    k_bits_to_queue<<<(unsigned)((gr.n + per_block - 1) / per_block), BLOCK, 0, st>>>(s, gr, round, BITS_QUEUE);
    return hipGetLastError();
}

hipError_t launch_pull(int W, int WC, const SlotArgs &s, const GraphArgs &gr, const GroupDesc &g,
                       const OutArgs &o, int32_t round, int32_t form, bool queue, hipStream_t st)
{
    CBFS_DISPATCH(W, WC, (k_pull<W, WC><<<(unsigned)gr.ntiles, BLOCK, 0, st>>>(s, gr, g, o, round, form,
                                                                                queue ? 1 : 0)));
    return hipGetLastError();
}

hipError_t launch_finalize(int W, int WC, const SlotArgs &s, int64_t n, const GroupDesc &g, const OutArgs &o,
                           hipStream_t st)
{
    int blocks = (int)std::min<int64_t>(8192, (n + BLOCK - 1) / BLOCK);
    CBFS_DISPATCH(W, WC, (k_finalize<W, WC><<<blocks, BLOCK, 0, st>>>(s, n, g, o)));
    return hipGetLastError();
}

hipError_t launch_scrub(const OutArgs &o, int64_t n, int32_t C, int32_t WC, const int32_t *abort_flag,
                        hipStream_t st)
{
    const int64_t per = (n + BLOCK * 64 - 1) / (BLOCK * 64);  // about 64 vertices per thread
    const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(per, 32));
    k_scrub<<<dim3(nb, (unsigned)C), BLOCK, 0, st>>>(o, n, WC, abort_flag);
    return hipGetLastError();
}

hipError_t persistent_grid(int W, int WC, int want_per_cu, int *blocks)
{
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    CBFS_DISPATCH(W, WC, (e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persistent<W, WC>, BLOCK, 0)));
    if (e != hipSuccess) return e;
    if (want_per_cu > 0 && want_per_cu < per_cu) per_cu = want_per_cu;
    *blocks = per_cu * cus;
    return *blocks > 0 ? hipSuccess : hipErrorInvalidValue;
}

hipError_t launch_persistent(int W, int WC, const PersistArgs &a, int blocks, hipStream_t st)
{
    PersistArgs arg = a;
    void *params[] = {&arg};
    hipError_t e = hipErrorInvalidValue;
    CBFS_DISPATCH(W, WC, (e = hipLaunchCooperativeKernel((const void *)k_persistent<W, WC>, dim3(blocks),
                                                         dim3(BLOCK), params, 0, st)));
    return e;
}

}  // namespace cbfs
