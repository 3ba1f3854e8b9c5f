// cbfs_run_batch: argument checks, workspace layout, cluster grouping, and the
// two ways to run the level loop (Algorithm "Cluster-BFS search from S": init,
// then rounds of vertex phase + edge phase until the frontier is empty):
//   - host loop: one launch per round, the frontier counters read back each
//     round to choose the direction and to stop;
//   - persistent: one cooperative launch for the whole batch.
// Also the per-thread diagnostics (run statistics and kernel timing).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "cbfs.h"
#include "cbfs_internal.h"
#include "cbfs_kernels.h"

namespace cbfs {

namespace {
thread_local std::string g_last_error;

constexpr size_t ALIGN = 256;
size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

// ---- diagnostics ----------------------------------------------------------
struct ProfRecord {
    int kind;
    hipEvent_t start, stop;
};
thread_local bool g_prof_on = false;
thread_local std::vector<ProfRecord> g_prof;
thread_local int64_t g_prof_launches[CBFS_KERNEL_KINDS];
thread_local double g_prof_ms[CBFS_KERNEL_KINDS];

struct LastRun {
    bool valid = false;
    bool device_stats = false;
    hipStream_t stream = nullptr;
    const long long *stats = nullptr;  // device [groups][STAT_WORDS] (persistent mode)
    const int32_t *err = nullptr;      // device error flag (persistent mode)
    cbfs_run_stats host{};
};
thread_local LastRun g_last;

// Brackets one launch with events when profiling is on.
struct ProfScope {
    int kind;
    hipStream_t st;
    hipEvent_t a = nullptr, b = nullptr;
    ProfScope(int k, hipStream_t s) : kind(k), st(s)
    {
        if (!g_prof_on) return;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
            a = b = nullptr;
            return;
        }
        hipEventRecord(a, st);
    }
    ~ProfScope()
    {
        if (!a) return;
        hipEventRecord(b, st);
        g_prof.push_back({kind, a, b});
    }
};
}  // namespace

cbfs_status fail(cbfs_status s, const char *msg)
{
    g_last_error = msg ? msg : "";
    return s;
}

cbfs_status hip_fail(const char *what, int err)
{
    g_last_error = std::string(what) + ": " + hipGetErrorString((hipError_t)err);
    return CBFS_E_HIP;
}

void prof_begin(int kind, hipStream_t st, void **token)
{
    *token = nullptr;
    if (!g_prof_on) return;
    *token = new ProfScope(kind, st);
}

void prof_end(void *token) { delete (ProfScope *)token; }

// How a batch is laid out: W words per vertex per group, WC words per cluster,
// clusters packed W/WC per group in batch order; `slots` groups searched side
// by side in the persistent mode.
struct Plan {
    int64_t n = 0, m = 0;
    int32_t C = 0, R = 0;
    int32_t minrel = 0;   // CBFS_ENCODE_MIN: R is the cluster diameter, R + 1 planes
    int32_t WC = 1;       // words per cluster (output W)
    int32_t W = 1;        // words per vertex in a group
    int32_t flog = 6;     // a cluster's field in a search word: 2^flog bits (6 = the whole word)
    int32_t fpw = 1;      // clusters per word (64 >> flog; WC = 1 when above 1)
    int32_t per_group = 1;
    int32_t groups = 0;
    int32_t slots = 1;
    int32_t mode = CBFS_MODE_PERSISTENT;
    float alpha = 5.0f, beta = 20.0f, gamma = 0.5f;
    int32_t force_pull = 0;
    int64_t hub_arcs = 65536;  // range-owned push from this many frontier arcs; <= 0: never
    int32_t blocks_per_cu = 0, schedule = 0;
    int32_t ntiles = 0;
    int64_t nwords = 0;
    int64_t qcap = 0;
    int32_t total_sources = 0;
    // workspace offsets
    size_t off_tiles_row = 0, off_tiles_edge = 0, off_cptr = 0, off_src = 0, off_center = 0;
    size_t off_slotdesc = 0, off_groupdesc = 0, off_ctl = 0, off_stats = 0, off_hub = 0, off_hubbounds = 0;
    size_t off_slots = 0, slot_bytes = 0;
    size_t total = 0;
};

static bool valid_w(int W, int WC)
{
    return (W == 1 && WC == 1) || (W == 3 && WC == 3) || (W == 2 && (WC == 1 || WC == 2)) ||
           ((W == 4 || W == 8 || W == 16) && (WC == 1 || WC == 2 || WC == 4));
}

static cbfs_status make_plan(const cbfs_csr *g, const cbfs_batch *b, const cbfs_tuning *t, Plan &p,
                             bool check_sources)
{
    if (!g || !b) return fail(CBFS_E_ARG, "cbfs_run_batch: null graph or batch");
    if (g->n < 1 || g->n >= INT32_MAX || g->m < 0 || g->m >= INT32_MAX || !g->row_ptr || (g->m > 0 && !g->col))
        return fail(CBFS_E_ARG, "cbfs_run_batch: bad graph sizes or pointers");
    if (b->num_clusters < 1 || !b->cluster_ptr || !b->sources)
        return fail(CBFS_E_ARG, "cbfs_run_batch: empty batch or null cluster arrays");
    if (b->radius < 0 || b->radius > 1024) return fail(CBFS_E_ARG, "cbfs_run_batch: radius outside [0, 1024]");
    if (b->encoding != CBFS_ENCODE_CENTER && b->encoding != CBFS_ENCODE_MIN)
        return fail(CBFS_E_ARG, "cbfs_run_batch: unknown encoding");
    if (b->cluster_ptr[0] != 0) return fail(CBFS_E_ARG, "cbfs_run_batch: cluster_ptr[0] != 0");
    int32_t kmax = 0;
    for (int32_t c = 0; c < b->num_clusters; c++) {
        int32_t k = b->cluster_ptr[c + 1] - b->cluster_ptr[c];
        if (k < 1 || k > CBFS_MAX_SOURCES)
            return fail(CBFS_E_TOO_MANY_SOURCES, "cbfs_run_batch: a cluster has 0 or more than 256 sources");
        kmax = std::max(kmax, k);
    }
    if (check_sources) {
        std::vector<int32_t> tmp;
        for (int32_t c = 0; c < b->num_clusters; c++) {
            const int32_t *S = b->sources + b->cluster_ptr[c];
            int32_t k = b->cluster_ptr[c + 1] - b->cluster_ptr[c];
            for (int32_t i = 0; i < k; i++)
                if (S[i] < 0 || S[i] >= g->n) return fail(CBFS_E_RANGE, "cbfs_run_batch: source outside [0, n)");
            tmp.assign(S, S + k);
            std::sort(tmp.begin(), tmp.end());
            if (std::adjacent_find(tmp.begin(), tmp.end()) != tmp.end())
                return fail(CBFS_E_DUP_SOURCE, "cbfs_run_batch: a vertex appears twice in one cluster");
        }
    }
    p.n = g->n;
    p.m = g->m;
    p.C = b->num_clusters;
    p.R = b->radius;
    p.minrel = b->encoding == CBFS_ENCODE_MIN ? 1 : 0;
    p.total_sources = b->cluster_ptr[p.C];
    p.WC = (kmax + 63) / 64;
    // defaults: wide groups share one CSR pass among many clusters (16 words,
    // which the pull splits over two lanes per vertex); sparse (high-diameter)
    // graphs get narrow groups searched side by side
    const bool sparse = p.m < 8 * p.n;
    p.W = p.WC == 3 ? 3 : (sparse ? p.WC : 16);
    if (p.W < p.WC) p.W = p.WC;
    p.mode = sparse ? CBFS_MODE_PERSISTENT : CBFS_MODE_HOST_LOOP;
    int32_t want_slots = 0;
    if (t) {
        if (t->mode < 0 || t->mode > CBFS_MODE_PERSISTENT) return fail(CBFS_E_ARG, "cbfs_tuning: bad mode");
        if (t->mode != CBFS_MODE_AUTO) p.mode = t->mode;
        if (t->group_words != 0) p.W = t->group_words;
        if (t->block_size != 0 && t->block_size != BLOCK) return fail(CBFS_E_ARG, "cbfs_tuning: block_size must be 256");
        if (t->alpha != 0.0f) p.alpha = t->alpha;
        if (t->beta < 0.0f) return fail(CBFS_E_ARG, "cbfs_tuning: beta < 0");
        if (t->beta != 0.0f) p.beta = t->beta;
        if (t->gamma != 0.0f) p.gamma = t->gamma;
        p.force_pull = t->force_pull;
        if (t->hub_arcs != 0) p.hub_arcs = t->hub_arcs;
        if (t->concurrent_groups < 0 || t->concurrent_groups > MAX_SLOTS)
            return fail(CBFS_E_ARG, "cbfs_tuning: concurrent_groups outside [0, 64]");
        want_slots = t->concurrent_groups;
        if (t->blocks_per_cu < 0 || t->blocks_per_cu > 32) return fail(CBFS_E_ARG, "cbfs_tuning: blocks_per_cu");
        if (t->schedule < 0 || t->schedule > 1) return fail(CBFS_E_ARG, "cbfs_tuning: schedule must be 0 or 1");
        p.blocks_per_cu = t->blocks_per_cu;
        p.schedule = t->schedule;
    }
    if (!valid_w(p.W, p.WC))
        return fail(CBFS_E_ARG, "cbfs_tuning: group_words must be one of 1,2,4,8,16 and a multiple of the cluster words");
    // clusters of at most 32 sources share search words: fields of 8, 16 or
    // 32 bits (the smallest that holds the largest cluster)
    {
        int32_t fb = (t && t->field_bits) ? t->field_bits : (p.WC == 1 && kmax <= 32 ? 8 : 64);
        if (!(t && t->field_bits))
            while (fb < 64 && fb < kmax) fb *= 2;
        if ((fb != 8 && fb != 16 && fb != 32 && fb != 64) || (fb < 64 && fb < kmax))
            return fail(CBFS_E_ARG, "cbfs_tuning: field_bits must be 8, 16, 32 or 64 and hold the largest cluster");
        p.flog = fb == 8 ? 3 : (fb == 16 ? 4 : (fb == 32 ? 5 : 6));
        p.fpw = 64 >> p.flog;
    }
    // never pack more words than clusters need
    p.per_group = p.W / p.WC * p.fpw;
    while (p.per_group > 1 && p.per_group / 2 >= p.C && valid_w(p.W / 2, p.WC)) {
        p.W /= 2;
        p.per_group = p.W / p.WC * p.fpw;
    }
    p.groups = (p.C + p.per_group - 1) / p.per_group;
    if (p.mode == CBFS_MODE_PERSISTENT) {
        // dense graphs: one group per die at least (the persistent kernel
        // deals slots to the dies, and a die without a slot sits idle)
        int32_t sl = want_slots ? want_slots : (sparse ? 32 : DIES);
        p.slots = std::max(1, std::min(sl, p.groups));
    } else {
        p.slots = 1;
    }
    p.nwords = (p.n + 63) / 64;
    p.qcap = p.n + p.m / PIECE + 1;
    p.ntiles = (int32_t)((p.n + p.m + TILE_ITEMS - 1) / TILE_ITEMS);
    if (p.ntiles < 1) p.ntiles = 1;

    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align_up(off + bytes);
        return at;
    };
    p.off_tiles_row = take(sizeof(int32_t) * (size_t)(p.ntiles + 1));
    p.off_tiles_edge = take(sizeof(int32_t) * (size_t)(p.ntiles + 1));
    p.off_cptr = take(sizeof(int32_t) * (size_t)(p.C + 1));
    p.off_src = take(sizeof(int32_t) * (size_t)std::max(1, p.total_sources));
    p.off_center = take(sizeof(int32_t) * (size_t)p.C);
    p.off_slotdesc = take(sizeof(SlotArgs) * MAX_SLOTS);
    p.off_groupdesc = take(sizeof(GroupDesc) * (size_t)p.groups);
    p.off_ctl = take(sizeof(unsigned int) * CTL_WORDS + 512);
    p.off_stats = take(sizeof(long long) * STAT_WORDS * (size_t)p.groups);
    p.off_hub = take(sizeof(int32_t) * (HUB_MAX + 1));
    p.off_hubbounds = take(sizeof(int32_t) * (size_t)HUB_MAX * (size_t)hub_bounds_stride(p.n));
    p.off_slots = off;
    size_t sb = 0;
    sb += 3 * align_up(sizeof(uint64_t) * (size_t)p.n * p.W);
    sb += 3 * align_up(sizeof(int64_t) * (size_t)p.qcap);
    sb += 3 * align_up(sizeof(uint64_t) * (size_t)p.nwords);
    sb += align_up(sizeof(unsigned long long) * 16);
    p.slot_bytes = sb;
    p.total = off + sb * (size_t)p.slots;
    return CBFS_OK;
}

static SlotArgs slot_at(const Plan &p, char *ws, int slot)
{
    SlotArgs s{};
    char *b = ws + p.off_slots + p.slot_bytes * (size_t)slot;
    size_t words = align_up(sizeof(uint64_t) * (size_t)p.n * p.W);
    s.A = (uint64_t *)b;
    b += words;
    s.B = (uint64_t *)b;
    b += words;
    s.seen = (uint64_t *)b;
    b += words;
    size_t qb = align_up(sizeof(int64_t) * (size_t)p.qcap);
    s.q0 = (int64_t *)b;
    b += qb;
    s.q1 = (int64_t *)b;
    b += qb;
    s.q2 = (int64_t *)b;
    b += qb;
    size_t bb = align_up(sizeof(uint64_t) * (size_t)p.nwords);
    s.bits0 = (uint64_t *)b;
    b += bb;
    s.bits1 = (uint64_t *)b;
    b += bb;
    s.bits2 = (uint64_t *)b;
    b += bb;
    s.ctr = (unsigned long long *)b;
    s.nwords = p.nwords;
    return s;
}

static GroupDesc group_desc(const Plan &p, const cbfs_batch *b, int32_t grp)
{
    GroupDesc d{};
    d.c0 = grp * p.per_group;
    d.nc = std::min(p.per_group, p.C - d.c0);
    d.flog = p.flog;
    for (int j = 0; j < d.nc; j++) {
        const int32_t k = b->cluster_ptr[d.c0 + j + 1] - b->cluster_ptr[d.c0 + j];
        if (p.fpw > 1) {  // cluster j in field j % fpw of word j / fpw
            d.full[j / p.fpw] |= ((1ull << k) - 1) << ((j % p.fpw) << p.flog);
            continue;
        }
        for (int x = 0; x < p.WC; x++) {
            const int lo = 64 * x;
            uint64_t w = 0;
            if (k >= lo + 64) w = ~0ull;
            else if (k > lo) w = (1ull << (k - lo)) - 1;
            d.full[j * p.WC + x] = w;
        }
    }
    return d;
}

static GraphArgs graph_args(const Plan &p, const cbfs_csr *g, char *ws)
{
    GraphArgs gr{};
    gr.n = p.n;
    gr.m = p.m;
    gr.row_ptr = g->row_ptr;
    gr.col = g->col;
    gr.tile_row = (const int32_t *)(ws + p.off_tiles_row);
    gr.tile_edge = (const int32_t *)(ws + p.off_tiles_edge);
    gr.ntiles = p.ntiles;
    return gr;
}

// ---------------------------------------------------------------------------
// Host resources the library owns: pinned staging buffers for the batch
// tables (a ring, each buffer reused once the event recorded after its upload
// has completed, so a call never waits for the device unless every buffer is
// still in flight), and pinned words the host loop reads the frontier
// counters into.  All of it is released by cbfs_release().
// ---------------------------------------------------------------------------
namespace {
struct StageBuf {
    void *host = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;  // recorded after the upload that last used the buffer
    bool pending = false;
};
constexpr int STAGE_RING = 8;
std::mutex g_res_mu;
std::vector<StageBuf> g_stage;                 // at most STAGE_RING
int g_stage_next = 0;
std::vector<unsigned long long *> g_counters;  // one pinned block per host thread that ran a host loop
unsigned g_res_gen = 1;                        // bumped by cbfs_release; thread caches compare it
}  // namespace

// Copies `bytes` of host memory into a pinned staging buffer and enqueues its
// upload to `dst` on `st`; the buffer is reused only after the upload has run.
static cbfs_status staged_upload(void *dst, const void *src, size_t bytes, hipStream_t st)
{
    std::lock_guard<std::mutex> lock(g_res_mu);
    hipError_t e;
    StageBuf *b = nullptr;
    for (auto &x : g_stage)  // a free buffer that fits
        if (x.cap >= bytes && (!x.pending || hipEventQuery(x.done) == hipSuccess)) {
            b = &x;
            break;
        }
    if (!b && (int)g_stage.size() < STAGE_RING) {
        g_stage.reserve(STAGE_RING);
        g_stage.push_back(StageBuf{});
        b = &g_stage.back();
        if ((e = hipEventCreateWithFlags(&b->done, hipEventDisableTiming)) != hipSuccess) {
            g_stage.pop_back();
            return hip_fail("staging event", e);
        }
    }
    if (!b) {  // every buffer in flight: take the next one in turn once its upload ran
        b = &g_stage[g_stage_next];
        g_stage_next = (g_stage_next + 1) % STAGE_RING;
        if ((e = hipEventSynchronize(b->done)) != hipSuccess) return hip_fail("staging wait", e);
    }
    if (b->pending && (e = hipEventSynchronize(b->done)) != hipSuccess) return hip_fail("staging wait", e);
    b->pending = false;
    if (b->cap < bytes) {
        if (b->host && (e = hipHostFree(b->host)) != hipSuccess) return hip_fail("staging free", e);
        b->host = nullptr;
        b->cap = 0;
        size_t cap = 4096;
        while (cap < bytes) cap *= 2;
        if ((e = hipHostMalloc(&b->host, cap, hipHostMallocDefault)) != hipSuccess)
            return hip_fail("staging allocation", e);
        b->cap = cap;
    }
    std::memcpy(b->host, src, bytes);
    if ((e = hipMemcpyAsync(dst, b->host, bytes, hipMemcpyHostToDevice, st)) != hipSuccess)
        return hip_fail("batch upload", e);
    if ((e = hipEventRecord(b->done, st)) != hipSuccess) return hip_fail("staging event record", e);
    b->pending = true;
    return CBFS_OK;
}

// Pinned host words the level loop reads the frontier counters into (one
// block per host thread, allocated on its first host-loop call).
static unsigned long long *pinned_counters()
{
    thread_local unsigned long long *buf = nullptr;
    thread_local unsigned gen = 0;
    std::lock_guard<std::mutex> lock(g_res_mu);
    if (!buf || gen != g_res_gen) {
        void *p = nullptr;
        if (hipHostMalloc(&p, 64, hipHostMallocDefault) != hipSuccess) return nullptr;
        buf = (unsigned long long *)p;
        gen = g_res_gen;
        g_counters.push_back(buf);
    }
    return buf;
}

#define PROF(kind, st, call)          \
    [&]() {                           \
        void *tok__;                  \
        prof_begin(kind, st, &tok__); \
        hipError_t e__ = (call);      \
        prof_end(tok__);              \
        return e__;                   \
    }()

// hc: host words the frontier counters are read into each round (pinned
// words of the library, or caller memory in the no-allocation form)
static cbfs_status run_host_loop(const Plan &p, const cbfs_csr *g, const cbfs_batch *b, uint32_t *dist,
                                 uint64_t *masks, int32_t *status, char *ws, hipStream_t st,
                                 unsigned long long *hc)
{
    const GraphArgs gr = graph_args(p, g, ws);
    const int32_t *d_cptr = (const int32_t *)(ws + p.off_cptr);
    const int32_t *d_src = (const int32_t *)(ws + p.off_src);
    OutArgs o{dist, masks, status, p.R, p.minrel, (const int32_t *)(ws + p.off_center)};
    hipError_t e;
    cbfs_run_stats &rs = g_last.host;
    const SlotArgs s = slot_at(p, ws, 0);
    const int64_t max_rounds = p.n + 2 * (int64_t)p.R + 4;
    for (int32_t grp = 0; grp < p.groups; grp++) {
        const GroupDesc gd = group_desc(p, b, grp);
        if ((e = PROF(CBFS_KERNEL_INIT, st, launch_init(p.W, s, p.n, gd, o, st))) != hipSuccess)
            return hip_fail("init", e);
        const int32_t nsrc = b->cluster_ptr[gd.c0 + gd.nc] - b->cluster_ptr[gd.c0];
        if ((e = PROF(CBFS_KERNEL_SEED, st, launch_seed(p.W, p.WC, s, gr, gd, d_src, d_cptr, nsrc, st))) != hipSuccess)
            return hip_fail("seed", e);
        bool dense = false;
        int32_t pulls = 0;
        // whether F_round's queue exists: the seed and the arc-parallel push
        // build it; pull rounds and the range-owned push leave only the bitmap
        // and the counters, and a push round builds the queue first
        bool queued = true;
        for (int32_t round = 0;; round++) {
            if (round > max_rounds) return fail(CBFS_E_HIP, "cbfs_run_batch: level loop did not terminate");
            if ((e = hipMemcpyAsync(hc, s.ctr + 4 * (round & 3), 3 * sizeof(unsigned long long),
                                    hipMemcpyDeviceToHost, st)) != hipSuccess)
                return hip_fail("counter copy", e);
            if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail("level sync", e);
            const int64_t pieces = (int64_t)hc[0], verts = (int64_t)hc[1], degsum = (int64_t)hc[2];
            if (verts == 0) break;
            // direction choice (Appendix A, Algorithm "EdgeMap"): dense when the
            // frontier plus its out-arcs is a large share of the graph; stay dense
            // while the frontier is still large.
            if (p.force_pull) dense = true;
            else if (p.alpha < 0) dense = false;
            else if (!dense) dense = (double)(verts + degsum) > (double)p.m / p.alpha;
            else dense = (double)verts > (double)p.n / p.beta;
            rs.rounds++;
            (dense ? rs.pull_rounds : rs.push_rounds)++;
            rs.frontier_vertices += verts;
            rs.frontier_arcs += degsum;
            if (dense) rs.pull_frontier_vertices += verts;
            // the group's first dense round, with a frontier carrying most of
            // the arcs: few rows can be complete yet, and the wave form gathers
            // every neighbour's set (the sets of non-members add nothing new,
            // Section 3.2, and the membership test would pass for most arcs)
            const int32_t form =
                pulls == 0 && p.gamma > 0.0f && (double)degsum > (double)p.gamma * (double)p.m ? PULL_WAVE
                                                                                               : PULL_WALK;
            if (dense) pulls++;
            // a push from a few vertices with many arcs: targets owned by blocks
            const bool hub = !dense && p.hub_arcs > 0 && verts <= HUB_MAX && degsum >= p.hub_arcs;
            if (!dense && !queued) {
                if ((e = PROF(CBFS_KERNEL_PUSH, st, launch_build_queue(s, gr, round, st))) != hipSuccess)
                    return hip_fail("queue", e);
            }
            queued = !dense && !hub;
            if (dense) e = PROF(CBFS_KERNEL_PULL, st, launch_pull(p.W, p.WC, s, gr, gd, o, round, form, false, st));
            else if (hub)
                e = PROF(CBFS_KERNEL_PUSH, st,
                         launch_push_hub(p.W, p.WC, s, gr, gd, o, round, pieces, degsum, (int32_t *)(ws + p.off_hub),
                                         (int32_t *)(ws + p.off_hubbounds), st));
            else e = PROF(CBFS_KERNEL_PUSH, st, launch_push(p.W, p.WC, s, gr, gd, o, round, pieces, degsum, st));
            if (e != hipSuccess) return hip_fail(dense ? "pull" : "push", e);
        }
        if ((e = PROF(CBFS_KERNEL_FINALIZE, st, launch_finalize(p.W, p.WC, s, p.n, gd, o, st))) != hipSuccess)
            return hip_fail("finalize", e);
    }
    return CBFS_OK;
}

static cbfs_status run_persistent(const Plan &p, const cbfs_csr *g, uint32_t *dist, uint64_t *masks,
                                  int32_t *status, char *ws, hipStream_t st)
{
    int blocks = 0;
    hipError_t e;
    if ((e = persistent_grid(p.W, p.WC, p.blocks_per_cu, &blocks)) != hipSuccess)
        return hip_fail("persistent occupancy", e);
    g_last.host.persistent_blocks = blocks;
    if (p.slots > blocks) return fail(CBFS_E_ARG, "cbfs_run_batch: more group slots than resident blocks");
    PersistArgs a{};
    a.gr = graph_args(p, g, ws);
    a.o = OutArgs{dist, masks, status, p.R, p.minrel, (const int32_t *)(ws + p.off_center)};
    a.slots = (const SlotArgs *)(ws + p.off_slotdesc);
    a.groups = (const GroupDesc *)(ws + p.off_groupdesc);
    a.num_groups = p.groups;
    a.num_slots = p.slots;
    a.sources = (const int32_t *)(ws + p.off_src);
    a.cluster_ptr = (const int32_t *)(ws + p.off_cptr);
    a.ctl = (unsigned int *)(ws + p.off_ctl);
    a.err = (int32_t *)(ws + p.off_ctl + sizeof(unsigned int) * CTL_WORDS);
    a.work = (unsigned long long *)(ws + p.off_ctl + sizeof(unsigned int) * CTL_WORDS + 128);
    a.stats = (long long *)(ws + p.off_stats);
    a.alpha = p.alpha;
    a.beta = p.beta;
    a.gamma = p.gamma;
    a.force_pull = p.force_pull;
    a.schedule = p.schedule;
    a.max_rounds = p.n + 2 * (int64_t)p.R + 4;
    // barrier, error flag and statistics start at zero (plain memsets: this
    // path is never captured into a graph)
    if ((e = hipMemsetAsync(ws + p.off_ctl, 0, sizeof(unsigned int) * CTL_WORDS + 512, st)) != hipSuccess)
        return hip_fail("control reset", e);
    if ((e = hipMemsetAsync(ws + p.off_stats, 0, sizeof(long long) * STAT_WORDS * (size_t)p.groups, st)) !=
        hipSuccess)
        return hip_fail("stats reset", e);
    if ((e = PROF(CBFS_KERNEL_PERSISTENT, st, launch_persistent(p.W, p.WC, a, blocks, st))) != hipSuccess)
        return hip_fail("persistent launch", e);
    g_last.device_stats = true;
    g_last.stats = a.stats;
    g_last.err = a.err;
    return CBFS_OK;
}

}  // namespace cbfs

using namespace cbfs;

extern "C" const char *cbfs_status_string(cbfs_status s)
{
    switch (s) {
    case CBFS_OK: return "CBFS_OK";
    case CBFS_E_ARG: return "CBFS_E_ARG";
    case CBFS_E_RANGE: return "CBFS_E_RANGE";
    case CBFS_E_DUP_SOURCE: return "CBFS_E_DUP_SOURCE";
    case CBFS_E_TOO_MANY_SOURCES: return "CBFS_E_TOO_MANY_SOURCES";
    case CBFS_E_RADIUS: return "CBFS_E_RADIUS";
    case CBFS_E_WORKSPACE: return "CBFS_E_WORKSPACE";
    case CBFS_E_HIP: return "CBFS_E_HIP";
    case CBFS_E_NOMEM: return "CBFS_E_NOMEM";
    default: return "CBFS_E_UNKNOWN";
    }
}

extern "C" const char *cbfs_last_error(void) { return g_last_error.c_str(); }

extern "C" size_t cbfs_run_batch_workspace_size(const cbfs_csr *g, const cbfs_batch *b, const cbfs_tuning *t)
{
    Plan p;
    if (make_plan(g, b, t, p, false) != CBFS_OK) return 0;
    return p.total;
}

// The batch on a planned, checked workspace.  no_alloc: take no pinned host
// memory (the tables go up from pageable memory followed by one stream wait;
// the host loop reads its counters into a local array).
static cbfs_status run_batch_planned(const Plan &p, const cbfs_csr *g, const cbfs_batch *b, uint32_t *dist,
                                     uint64_t *masks, int32_t *cluster_status, char *ws, hipStream_t st,
                                     bool no_alloc)
{
    cbfs_status rc;
    g_last = LastRun{};
    g_last.valid = true;
    g_last.stream = st;
    g_last.host.groups = p.groups;
    g_last.host.group_words = p.W;
    g_last.host.slots = p.slots;
    g_last.host.mode = p.mode;

    // one upload of the batch tables through a pinned staging buffer (no wait
    // for earlier work on the stream); the host arrays are not used afterwards
    // the tables occupy workspace bytes [off_cptr, off_ctl)
    const size_t lo = p.off_cptr, hi = p.off_ctl;
    std::vector<char> stage(hi - lo, 0);
    std::memcpy(stage.data() + (p.off_cptr - lo), b->cluster_ptr, sizeof(int32_t) * (size_t)(p.C + 1));
    std::memcpy(stage.data() + (p.off_src - lo), b->sources, sizeof(int32_t) * (size_t)p.total_sources);
    for (int32_t c = 0; c < p.C; c++)
        reinterpret_cast<int32_t *>(stage.data() + (p.off_center - lo))[c] = b->sources[b->cluster_ptr[c]];
    for (int32_t sl = 0; sl < p.slots; sl++) {
        SlotArgs s = slot_at(p, ws, sl);
        std::memcpy(stage.data() + (p.off_slotdesc - lo) + sizeof(SlotArgs) * sl, &s, sizeof(SlotArgs));
    }
    for (int32_t grp = 0; grp < p.groups; grp++) {
        GroupDesc d = group_desc(p, b, grp);
        std::memcpy(stage.data() + (p.off_groupdesc - lo) + sizeof(GroupDesc) * grp, &d, sizeof(GroupDesc));
    }
    hipError_t e;
    if (!no_alloc) {
        if ((rc = staged_upload(ws + lo, stage.data(), hi - lo, st)) != CBFS_OK) return rc;
    } else {
        // pageable source: wait for the copy before `stage` goes away
        if ((e = hipMemcpyAsync(ws + lo, stage.data(), hi - lo, hipMemcpyHostToDevice, st)) != hipSuccess)
            return hip_fail("batch upload", e);
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail("batch upload wait", e);
    }
    if ((e = PROF(CBFS_KERNEL_TILES, st,
                  launch_tiles(g->row_ptr, p.n, p.m, p.ntiles, (int32_t *)(ws + p.off_tiles_row),
                               (int32_t *)(ws + p.off_tiles_edge), st))) != hipSuccess)
        return hip_fail("tiles", e);
    const int32_t *abort_flag = nullptr;
    if (p.mode == CBFS_MODE_HOST_LOOP) {
        unsigned long long local[4] = {0, 0, 0, 0};
        unsigned long long *hc = no_alloc ? local : pinned_counters();
        if (!hc) return fail(CBFS_E_NOMEM, "cbfs_run_batch: pinned host counters");
        rc = run_host_loop(p, g, b, dist, masks, cluster_status, ws, st, hc);
    } else {
        rc = run_persistent(p, g, dist, masks, cluster_status, ws, st);
        abort_flag = (const int32_t *)(ws + p.off_ctl + sizeof(unsigned int) * CTL_WORDS);
    }
    if (rc != CBFS_OK) return rc;
    // clusters whose status is not CBFS_OK: defined outputs (UNREACHED, zero masks)
    const OutArgs o{dist, masks, cluster_status, p.R, p.minrel};
    if ((e = PROF(CBFS_KERNEL_FINALIZE, st, launch_scrub(o, p.n, p.C, p.WC, abort_flag, st))) != hipSuccess)
        return hip_fail("status scrub", e);
    return CBFS_OK;
}

extern "C" cbfs_status cbfs_run_batch(const cbfs_csr *g, const cbfs_batch *b, const cbfs_tuning *t,
                                      uint32_t *dist, uint64_t *masks, int32_t *cluster_status,
                                      void *workspace, size_t workspace_bytes, void *stream)
{
    g_last_error.clear();
    Plan p;
    cbfs_status rc = make_plan(g, b, t, p, true);
    if (rc != CBFS_OK) return rc;
    if (!dist || !masks || !cluster_status || !workspace)
        return fail(CBFS_E_ARG, "cbfs_run_batch: null output or workspace");
    if (workspace_bytes < p.total) return fail(CBFS_E_WORKSPACE, "cbfs_run_batch: workspace too small");
    return run_batch_planned(p, g, b, dist, masks, cluster_status, (char *)workspace, (hipStream_t)stream, false);
}

// ---------------------------------------------------------------------------
// The batch with the library's own device array as its workspace, for callers
// that cannot allocate.  `scratch` is a host-side name only: host code uses
// the device address looked up once per device (hipGetSymbolAddress with that
// device current), never the array's name.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[CBFS_STATIC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES];  // address of `scratch` on each device, once looked up
}  // namespace

static cbfs_status scratch_of_current_device(void **out)
{
    int dev = -1;
    hipError_t e;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return hip_fail("current device", e);
    if (dev < 0 || dev >= MAX_DEVICES) return fail(CBFS_E_ARG, "cbfs_run_batch_static: device index >= 64");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        if ((e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch))) != hipSuccess)
            return hip_fail("scratch address", e);
        if (!ptr) return fail(CBFS_E_HIP, "cbfs_run_batch_static: scratch address is null");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return CBFS_OK;
}

extern "C" cbfs_status cbfs_run_batch_static(const cbfs_csr *g, const cbfs_batch *b, const cbfs_tuning *t,
                                             uint32_t *dist, uint64_t *masks, int32_t *cluster_status,
                                             void *stream)
{
    g_last_error.clear();
    Plan p;
    cbfs_status rc = make_plan(g, b, t, p, true);
    if (rc != CBFS_OK) return rc;
    if (!dist || !masks || !cluster_status) return fail(CBFS_E_ARG, "cbfs_run_batch_static: null output");
    if (p.total > (size_t)CBFS_STATIC_SCRATCH_BYTES)
        return fail(CBFS_E_WORKSPACE, "cbfs_run_batch_static: the batch needs more than the static scratch");
    void *ws = nullptr;
    if ((rc = scratch_of_current_device(&ws)) != CBFS_OK) return rc;
    return run_batch_planned(p, g, b, dist, masks, cluster_status, (char *)ws, (hipStream_t)stream, true);
}

extern "C" cbfs_status cbfs_release(void)
{
    std::lock_guard<std::mutex> lock(g_res_mu);
    cbfs_status rc = CBFS_OK;
    for (auto &b : g_stage) {
        if (b.pending && hipEventSynchronize(b.done) != hipSuccess) rc = CBFS_E_HIP;
        if (b.done && hipEventDestroy(b.done) != hipSuccess) rc = CBFS_E_HIP;
        if (b.host && hipHostFree(b.host) != hipSuccess) rc = CBFS_E_HIP;
    }
    g_stage.clear();
    g_stage_next = 0;
    for (auto *c : g_counters)
        if (hipHostFree(c) != hipSuccess) rc = CBFS_E_HIP;
    g_counters.clear();
    g_res_gen++;
    for (auto &r : g_prof) {
        hipEventDestroy(r.start);
        hipEventDestroy(r.stop);
    }
    g_prof.clear();
    g_prof_on = false;
    return rc == CBFS_OK ? CBFS_OK : fail(rc, "cbfs_release: a HIP call failed");
}

extern "C" cbfs_status cbfs_last_run_stats(cbfs_run_stats *out)
{
    if (!out) return fail(CBFS_E_ARG, "cbfs_last_run_stats: null output");
    if (!g_last.valid) return fail(CBFS_E_ARG, "cbfs_last_run_stats: no cbfs_run_batch call on this thread");
    cbfs_run_stats r = g_last.host;
    if (g_last.device_stats) {
        std::vector<long long> st(STAT_WORDS * (size_t)r.groups);
        int32_t err = 0;
        hipError_t e;
        if ((e = hipStreamSynchronize(g_last.stream)) != hipSuccess) return hip_fail("stats sync", e);
        if ((e = hipMemcpy(st.data(), g_last.stats, sizeof(long long) * st.size(), hipMemcpyDeviceToHost)) !=
            hipSuccess)
            return hip_fail("stats copy", e);
        if ((e = hipMemcpy(&err, g_last.err, sizeof(int32_t), hipMemcpyDeviceToHost)) != hipSuccess)
            return hip_fail("error flag copy", e);
        for (int64_t grp = 0; grp < r.groups; grp++) {
            const long long *sg = st.data() + STAT_WORDS * grp;
            r.rounds += sg[0];
            r.push_rounds += sg[1];
            r.pull_rounds += sg[2];
            r.frontier_vertices += sg[3];
            r.frontier_arcs += sg[4];
            r.pull_frontier_vertices += sg[5];
        }
        r.device_error = err;
    }
    *out = r;
    if (r.device_error == 1) return fail(CBFS_E_HIP, "persistent kernel: grid barrier timed out");
    if (r.device_error == 2) return fail(CBFS_E_HIP, "persistent kernel: level loop did not terminate");
    return CBFS_OK;
}

extern "C" cbfs_status cbfs_profile_enable(int32_t enable)
{
    for (auto &r : g_prof) {
        hipEventDestroy(r.start);
        hipEventDestroy(r.stop);
    }
    g_prof.clear();
    for (int k = 0; k < CBFS_KERNEL_KINDS; k++) {
        g_prof_launches[k] = 0;
        g_prof_ms[k] = 0.0;
    }
    g_prof_on = enable != 0;
    return CBFS_OK;
}

extern "C" cbfs_status cbfs_profile_read(int64_t *launches, double *total_ms)
{
    if (!launches || !total_ms) return fail(CBFS_E_ARG, "cbfs_profile_read: null output");
    for (auto &r : g_prof) {
        hipError_t e = hipEventSynchronize(r.stop);
        if (e != hipSuccess) return hip_fail("profile event sync", e);
        float ms = 0.f;
        hipEventElapsedTime(&ms, r.start, r.stop);
        g_prof_launches[r.kind]++;
        g_prof_ms[r.kind] += ms;
        hipEventDestroy(r.start);
        hipEventDestroy(r.stop);
    }
    g_prof.clear();
    for (int k = 0; k < CBFS_KERNEL_KINDS; k++) {
        launches[k] = g_prof_launches[k];
        total_ms[k] = g_prof_ms[k];
    }
    return CBFS_OK;
}

// ---------------------------------------------------------------------------
// Autotuner: coordinate descent over the launch knobs on a sample of the
// batch (the first clusters), each candidate timed from host to stream
// completion after one warm-up run.
// ---------------------------------------------------------------------------
namespace {

struct Tuner {
    const cbfs_csr *g;
    cbfs_batch sample;
    uint32_t *dist;
    uint64_t *masks;
    int32_t *status;
    void *ws;
    size_t ws_bytes;
    hipStream_t st;
    cbfs_trial *out;
    int32_t max_out;
    int32_t count = 0;
    std::vector<cbfs_tuning> seen;
    cbfs_tuning best{};
    float best_ms = -1.f;

    static bool same(const cbfs_tuning &a, const cbfs_tuning &b) { return std::memcmp(&a, &b, sizeof a) == 0; }

    // returns CBFS_OK unless a run failed
    cbfs_status eval(const cbfs_tuning &t)
    {
        for (const auto &x : seen)
            if (same(x, t)) return CBFS_OK;
        seen.push_back(t);
        Plan p;
        float ms = -1.f;
        int32_t mode = 0;
        if (make_plan(g, &sample, &t, p, false) == CBFS_OK && p.total <= ws_bytes) {
            mode = p.mode;
            hipError_t e;
            cbfs_status rc = cbfs_run_batch(g, &sample, &t, dist, masks, status, ws, ws_bytes, st);
            if (rc != CBFS_OK) return rc;
            if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail("autotune sync", e);
            const auto t0 = std::chrono::steady_clock::now();
            rc = cbfs_run_batch(g, &sample, &t, dist, masks, status, ws, ws_bytes, st);
            if (rc != CBFS_OK) return rc;
            if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail("autotune sync", e);
            ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
            if (best_ms < 0.f || ms < best_ms) {
                best_ms = ms;
                best = t;
            }
        }
        if (out && count < max_out) out[count] = cbfs_trial{t, ms, mode};
        count++;
        return CBFS_OK;
    }
};

cbfs_batch sample_of(const cbfs_batch *b, int32_t sample_clusters)
{
    cbfs_batch s = *b;
    int32_t S = sample_clusters > 0 ? sample_clusters : 16;
    if (S > b->num_clusters) S = b->num_clusters;
    s.num_clusters = S;
    return s;
}

const int32_t kTuneWords[] = {1, 2, 4, 8, 16};
const int32_t kTuneSlots[] = {4, 8, 16, 32, 64};

}  // namespace

extern "C" size_t cbfs_autotune_workspace_size(const cbfs_csr *g, const cbfs_batch *b, int32_t sample_clusters)
{
    if (!g || !b || b->num_clusters < 1 || !b->cluster_ptr) return 0;
    const cbfs_batch sb = sample_of(b, sample_clusters);
    size_t mx = 0;
    for (int32_t mode : {CBFS_MODE_HOST_LOOP, CBFS_MODE_PERSISTENT})
        for (int32_t w : kTuneWords)
            for (int32_t sl : kTuneSlots) {
                cbfs_tuning t{};
                t.mode = mode;
                t.group_words = w;
                t.concurrent_groups = sl;
                Plan p;
                if (make_plan(g, &sb, &t, p, false) == CBFS_OK) mx = std::max(mx, p.total);
            }
    return mx;
}

extern "C" cbfs_status cbfs_autotune(const cbfs_csr *g, const cbfs_batch *b, const cbfs_tuning *start,
                                     int32_t sample_clusters, uint32_t *dist, uint64_t *masks,
                                     int32_t *cluster_status, void *workspace, size_t workspace_bytes,
                                     void *stream, cbfs_tuning *best, cbfs_trial *trials, int32_t max_trials,
                                     int32_t *num_trials)
{
    g_last_error.clear();
    if (!g || !b || !best || !dist || !masks || !cluster_status || !workspace)
        return fail(CBFS_E_ARG, "cbfs_autotune: null argument");
    if (sample_clusters < 0) return fail(CBFS_E_ARG, "cbfs_autotune: sample_clusters < 0");
    if (trials && max_trials < 0) return fail(CBFS_E_ARG, "cbfs_autotune: max_trials < 0");
    Plan p0;
    cbfs_status rc = make_plan(g, b, start, p0, true);  // validates the whole batch once
    if (rc != CBFS_OK) return rc;
    Tuner tu{g, sample_of(b, sample_clusters), dist, masks, cluster_status, workspace, workspace_bytes,
             (hipStream_t)stream, trials, trials ? max_trials : 0};
    cbfs_tuning cur{};
    if (start) cur = *start;
    const bool sparse = g->m < 8 * g->n;
    auto step = [&](auto &&mutate, const auto &values) -> cbfs_status {
        const cbfs_tuning base = tu.best_ms >= 0.f ? tu.best : cur;
        for (const auto &v : values) {
            cbfs_tuning t = base;
            mutate(t, v);
            if (cbfs_status r = tu.eval(t); r != CBFS_OK) return r;
        }
        return CBFS_OK;
    };
    if ((rc = tu.eval(cur)) != CBFS_OK) return rc;
    // launch mode (the host loop costs a round trip per round: not tried on
    // sparse graphs, which run thousands of rounds)
    if (!sparse) {
        const int32_t modes[] = {CBFS_MODE_HOST_LOOP, CBFS_MODE_PERSISTENT};
        if ((rc = step([](cbfs_tuning &t, int32_t v) { t.mode = v; }, modes)) != CBFS_OK) return rc;
    }
    std::vector<int32_t> words;  // packings valid for the whole batch's clusters
    for (int32_t w : kTuneWords)
        if (valid_w(w, p0.WC)) words.push_back(w);
    if ((rc = step([](cbfs_tuning &t, int32_t v) { t.group_words = v; }, words)) != CBFS_OK) return rc;
    const float alphas[] = {5.f, 15.f, 45.f};
    if ((rc = step([](cbfs_tuning &t, float v) { t.alpha = v; }, alphas)) != CBFS_OK) return rc;
    const float gammas[] = {0.25f, 0.5f, -1.f};
    if ((rc = step([](cbfs_tuning &t, float v) { t.gamma = v; }, gammas)) != CBFS_OK) return rc;
    Plan pb;
    if (make_plan(g, &tu.sample, &tu.best, pb, false) == CBFS_OK && pb.mode == CBFS_MODE_PERSISTENT)
        if ((rc = step([](cbfs_tuning &t, int32_t v) { t.concurrent_groups = v; }, kTuneSlots)) != CBFS_OK)
            return rc;
    if (pb.mode == CBFS_MODE_HOST_LOOP) {
        const int32_t hubs[] = {16384, 65536, -1};
        if ((rc = step([](cbfs_tuning &t, int32_t v) { t.hub_arcs = v; }, hubs)) != CBFS_OK) return rc;
    }
    if (tu.best_ms < 0.f) return fail(CBFS_E_WORKSPACE, "cbfs_autotune: no candidate fits the workspace");
    *best = tu.best;
    if (num_trials) *num_trials = tu.count;
    return CBFS_OK;
}
