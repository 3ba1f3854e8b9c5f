/*
 * cbfs.h -- C ABI of the MI355X (gfx950) Cluster-BFS library, libcbfs.so.
 *
 * Cluster-BFS (C-BFS; paper Section 3, Algorithm "Cluster-BFS search from S"):
 * one breadth-first search from a cluster S = {s_0, ..., s_{k-1}} of nearby
 * sources that yields, for every vertex v, the hop distance from the cluster
 * center s_0 plus, for each offset o in [-R, R], the bit-subset of sources
 * whose distance to v is d(s_0, v) + o.  This is the paper's cluster distance
 * vector (Section 3.1, subset equation) re-based on the center, the storage
 * the paper uses for star clusters (Section 5.3: a distance and d bit-subsets
 * per cluster per vertex).  All arithmetic is exact integer arithmetic.
 *
 * Conventions
 *   - Vertex ids are int32 in [0, n).  Graphs are CSR: row_ptr[n+1] and col[m]
 *     (int32, m < 2^31); row v lists the out-neighbours of v.  The searches
 *     need a symmetric graph (every arc (u,v) has its reverse (v,u)), which
 *     cbfs_build_csr produces; the pull direction reads rows as in-neighbours.
 *   - Source i of a cluster is bit (i % 64) of word (i / 64); source 0 is the
 *     cluster center.  A cluster has 1..256 sources, all distinct.
 *   - "device" pointers are HIP device memory of the current device; "host"
 *     pointers are ordinary process memory.  The library never allocates
 *     device memory: every device buffer, including the workspace, belongs to
 *     the caller (the one exception is the fixed scratch array that
 *     cbfs_run_batch_static uses in place of a workspace, part of the
 *     library's code object).  Host arrays are read (and host outputs
 *     written) before the call returns.
 *   - stream is a hipStream_t passed as void* (NULL = the null stream).
 *   - Every entry point returns a cbfs_status.  Argument errors are detected on
 *     the host before anything is enqueued; such a call writes no output.
 *     CBFS_E_HIP reports a failed HIP call; cbfs_last_error() gives the detail
 *     for the calling thread.
 */
#ifndef CBFS_H
#define CBFS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t cbfs_status;
enum {
    CBFS_OK = 0,
    CBFS_E_ARG = -1,              /* null pointer, bad size or bad tuning value      */
    CBFS_E_RANGE = -2,            /* a vertex id outside [0, n)                      */
    CBFS_E_DUP_SOURCE = -3,       /* a vertex listed twice in one cluster            */
    CBFS_E_TOO_MANY_SOURCES = -4, /* a cluster with 0 or more than 256 sources       */
    CBFS_E_RADIUS = -5,           /* (per cluster) some offset falls outside [-R, R] */
    CBFS_E_WORKSPACE = -6,        /* workspace or output capacity too small          */
    CBFS_E_HIP = -7,              /* a HIP runtime call failed                       */
    CBFS_E_NOMEM = -8             /* host allocation failed                          */
};

#define CBFS_MAX_SOURCES 256
#define CBFS_UNREACHED 0xFFFFFFFFu

/* Human-readable name of a status code (static string). */
const char *cbfs_status_string(cbfs_status s);
/* Detail of the last error raised on the calling thread ("" if none). */
const char *cbfs_last_error(void);

/* ------------------------------------------------------------------------ *
 * Graph ingest (host).  The paper's inputs are undirected graphs (Section 5
 * setup) and its applications assume them (Section 4).
 *
 * Turns an edge list into a cleaned CSR: flags select
 *   CBFS_CSR_SYMMETRIZE       add the reverse of every arc
 *   CBFS_CSR_DEDUP            drop repeated arcs
 *   CBFS_CSR_DROP_SELF_LOOPS  drop arcs (v, v)
 *   CBFS_CSR_KEEP_LCC         keep only the largest connected component (arcs
 *                             taken as undirected; ties go to the component
 *                             holding the smallest input id)
 * Kept vertices are renumbered 0..n_out-1 in ascending input-id order, and each
 * row is sorted ascending.
 *   n_in                   vertex ids in src/dst lie in [0, n_in), n_in < 2^31
 *   src, dst [num_edges]   host, int64 endpoints
 *   row_ptr  [n_in + 1]    host output (first n_out+1 entries written)
 *   col      [col_capacity] host output (first m_out entries written);
 *                          2*num_edges always suffices
 *   n_out, m_out           host outputs: vertex and arc counts
 *   old_to_new [n_in]      host output, nullable: new id or -1 if dropped
 * Errors: CBFS_E_ARG (null/negative), CBFS_E_RANGE (endpoint out of range),
 * CBFS_E_WORKSPACE (col_capacity < m_out or m_out >= 2^31), CBFS_E_NOMEM.
 * ------------------------------------------------------------------------ */
enum {
    CBFS_CSR_SYMMETRIZE = 1,
    CBFS_CSR_DEDUP = 2,
    CBFS_CSR_DROP_SELF_LOOPS = 4,
    CBFS_CSR_KEEP_LCC = 8,
    CBFS_CSR_ALL = 15
};
cbfs_status cbfs_build_csr(int64_t n_in, int64_t num_edges, const int64_t *src, const int64_t *dst,
                           uint32_t flags, int32_t *row_ptr, int32_t *col, int64_t col_capacity,
                           int64_t *n_out, int64_t *m_out, int64_t *old_to_new);

/* ------------------------------------------------------------------------ *
 * Cluster selection (host).  Section 4.2 builds clusters around high-degree
 * centers; the rules here are the ones the seeded workloads use.
 *
 * cbfs_top_degree: the `count` vertices of largest degree (row length), ties
 * by ascending id, written to out[count] in that order.
 *
 * cbfs_select_clusters: for each center c (host centers[num_centers]), the
 * cluster is c followed by the lowest-id vertices at hop distance 1..hops from
 * c, ascending, k_max sources at most.  Outputs cluster_ptr[num_centers+1]
 * (host) and sources[sources_capacity] (host); num_centers*k_max suffices.
 * Errors: CBFS_E_ARG, CBFS_E_RANGE, CBFS_E_TOO_MANY_SOURCES (k_max outside
 * 1..256), CBFS_E_WORKSPACE (capacity), CBFS_E_NOMEM.
 * ------------------------------------------------------------------------ */
cbfs_status cbfs_top_degree(int64_t n, const int32_t *row_ptr, int32_t count, int32_t *out);

/* cbfs_select_landmarks: clusters of landmarks as Section 4.2 ("Selecting
 * Landmarks in Clusters") builds them for a cluster size k and diameter d:
 * the unmarked vertex of highest degree is a center; among its unmarked
 * vertices within floor(d/2) hops the k-1 of highest degree join it; every
 * vertex of the cluster is marked and never selected again; repeated until
 * num_clusters clusters exist or every vertex is marked.  Degree ties go to
 * the lower id.  Each cluster lists its center first, then its members by
 * descending degree.  Outputs cluster_ptr[num_clusters+1] and
 * sources[sources_capacity] (host; num_clusters*k suffices) and
 * *num_selected, the clusters made.  Every cluster has diameter <= d.
 * Errors: CBFS_E_ARG, CBFS_E_TOO_MANY_SOURCES (k outside 1..256),
 * CBFS_E_WORKSPACE (capacity), CBFS_E_NOMEM. */
cbfs_status cbfs_select_landmarks(int64_t n, const int32_t *row_ptr, const int32_t *col, int32_t num_clusters,
                                  int32_t k, int32_t diameter, int32_t *cluster_ptr, int32_t *sources,
                                  int64_t sources_capacity, int32_t *num_selected);
cbfs_status cbfs_select_clusters(int64_t n, const int32_t *row_ptr, const int32_t *col,
                                 int32_t num_centers, const int32_t *centers, int32_t k_max,
                                 int32_t hops, int32_t *cluster_ptr, int32_t *sources,
                                 int64_t sources_capacity);

/* ------------------------------------------------------------------------ *
 * Cluster-BFS over a batch of clusters (device).
 *
 * Input: a graph and clusters with radius R (Algorithm "Cluster-BFS search
 * from S": a graph and a cluster of diameter d).  Output, for every cluster c
 * and vertex v (Section 3.1 subset equation, center-relative):
 *   dist[c][v]            = d(s_0, v), or CBFS_UNREACHED
 *   masks[c][o + R][v][w] = word w of the set {i : d(s_i, v) = d(s_0, v) + o},
 *                           o in [-R, R]; all zero where dist is CBFS_UNREACHED
 * or, with encoding CBFS_ENCODE_MIN and radius = the cluster diameter d, the
 * paper's cluster distance vector <S_v[0..d], Delta_v> (Section 3.1):
 *   dist[c][v]            = Delta_v = min_i d(s_i, v), or CBFS_UNREACHED
 *   masks[c][j][v][w]     = word w of {i : d(s_i, v) = Delta_v + j}, j in [0, d]
 * (a source that reaches v more than d beyond Delta_v, or not at all while
 * another source does, is a violation of the given diameter).
 *   cluster_status[c]     = CBFS_OK, or CBFS_E_RADIUS when some source of c
 *                           lies at an offset outside [-R, R] at some vertex
 *                           (or reaches a vertex the center does not), or
 *                           CBFS_E_HIP when the persistent kernel stopped
 *                           early (see cbfs_last_run_stats).  A cluster whose
 *                           status is not CBFS_OK has dist = CBFS_UNREACHED
 *                           and every mask word 0 at every vertex.
 * W (words per mask) = ceil(max_c k_c / 64) over the batch.  By the Fact and
 * Corollary of Section 3.1 every offset is bounded by the source's distance to
 * the center, so R >= that distance for every source guarantees CBFS_OK on a
 * symmetric graph.
 *
 * The level-synchronous search follows Algorithm "Cluster-BFS search from S":
 * per round a vertex phase (new bits = next minus seen, first round, subset
 * write, seen update) and an edge phase in either direction of Algorithm
 * "EdgeMap" (push with 64-bit atomic OR, or pull with early exit), chosen per
 * round from the frontier size and degree sum (Appendix A).  Clusters are
 * packed several to a vertex word group and share one level loop.
 * ------------------------------------------------------------------------ */
typedef struct {
    int64_t n;              /* vertices                               */
    int64_t m;              /* arcs (= row_ptr[n])                    */
    const int32_t *row_ptr; /* device [n+1]                           */
    const int32_t *col;     /* device [m]                             */
} cbfs_csr;

enum {
    CBFS_ENCODE_CENTER = 0,  /* dist = d(s_0, v), planes for offsets -R..R (2R+1), the
                                star storage of Section 5.3                           */
    CBFS_ENCODE_MIN = 1      /* the paper's own form, Section 3.1: dist = Delta_v =
                                min over the sources of d(s, v), and plane i the subset
                                S_v[i] = {s : d(s, v) = Delta_v + i}, i = 0..d, for a
                                cluster of diameter d given in `radius` (d+1 planes)  */
};

typedef struct {
    int32_t num_clusters;       /* C >= 1                                          */
    const int32_t *cluster_ptr; /* host [C+1], cluster_ptr[0] = 0, non-decreasing  */
    const int32_t *sources;     /* host; cluster c = sources[cluster_ptr[c] ..
                                   cluster_ptr[c+1]), its first entry the center   */
    int32_t radius;             /* CBFS_ENCODE_CENTER: R >= 0, 2R+1 offset planes;
                                   CBFS_ENCODE_MIN: the diameter d >= 0, d+1 planes */
    int32_t encoding;           /* CBFS_ENCODE_* (0: center-relative)              */
} cbfs_batch;

enum {
    CBFS_MODE_AUTO = 0,       /* library's choice: host loop on graphs with average degree
                                 >= 8, persistent below (many rounds, small frontiers)     */
    CBFS_MODE_HOST_LOOP = 1,  /* one launch per round, frontier size read back each round  */
    CBFS_MODE_PERSISTENT = 2  /* one cooperative launch for the whole batch, device-side
                                 level loop with grid barriers, no host round trips         */
};

/* Tuning knobs (nullable: all defaults).  No knob changes any output bit. */
typedef struct {
    int32_t mode;              /* CBFS_MODE_*                                          */
    int32_t group_words;       /* words per vertex of a cluster group: 0 = auto (16,
                                  fewer when the batch has fewer clusters; the
                                  cluster's words on sparse graphs), else a multiple
                                  of W in {1,2,4,8,16}                                 */
    int32_t concurrent_groups; /* group slots searched side by side: 0 = auto          */
    int32_t block_size;        /* 0 = auto, else 256                                    */
    float alpha;               /* pull when |F| + sum deg(F) > m / alpha; 0 = auto (5);
                                  < 0 forces push every round                           */
    float beta;                /* stay pull while |F| > n / beta; 0 = auto              */
    int32_t force_pull;        /* 1: pull every round (testing)                         */
    int32_t blocks_per_cu;     /* persistent mode: resident blocks per compute unit;
                                  0 = as many as fit                                    */
    int32_t schedule;          /* persistent mode: 0 = fixed stride over the items
                                  (default), 1 = blocks take work items from a shared
                                  counter                                               */
    float gamma;               /* a group's first pull round runs in the wave form (every
                                  neighbour's set OR-ed, no frontier-bitmap test) when
                                  sum deg(F) > gamma * m; 0 = auto (0.5), < 0 = never   */
    int32_t hub_arcs;          /* host-loop mode: a push round whose frontier has at most
                                  256 vertices and at least hub_arcs arcs runs with
                                  blocks that own target ranges (sets merged in LDS, one
                                  store per target); 0 = auto (65536), < 0 = never      */
    int32_t field_bits;        /* bits a cluster of at most 32 sources takes in a search
                                  word: 8, 16 or 32 (several clusters share each word),
                                  or 64 (one cluster per word); 0 = auto (the smallest of
                                  8, 16, 32 that holds the largest cluster, 64 for
                                  clusters of more than 32 sources).  Outputs do not
                                  depend on it.                                          */
} cbfs_tuning;

/* Bytes of device workspace cbfs_run_batch needs for these arguments. */
size_t cbfs_run_batch_workspace_size(const cbfs_csr *g, const cbfs_batch *b, const cbfs_tuning *t);

/*
 *   dist           device [C][n]          uint32 output
 *   masks          device [C][P][n][WC]   uint64 output, WC = ceil(k_max / 64)
 *                                         words per cluster (k_max: the largest
 *                                         cluster), P = 2R+1 (center) or d+1
 *                                         (min, d = radius)
 *   cluster_status device [C]             int32 output
 *   workspace      device, workspace_bytes >= cbfs_run_batch_workspace_size(...)
 * Ordering: everything is enqueued on `stream`.  In CBFS_MODE_PERSISTENT the
 * call returns without waiting for the device: the batch tables go up from a
 * pinned staging buffer the library owns (a ring of buffers, each reused
 * once its upload has run; only when all of them are still in flight does a
 * call wait for the oldest upload).  CBFS_MODE_HOST_LOOP waits on the stream
 * once per round to read the frontier counters.  The outputs are complete
 * when the stream reaches the end of the call's work.
 * Errors: CBFS_E_ARG, CBFS_E_RANGE, CBFS_E_DUP_SOURCE, CBFS_E_TOO_MANY_SOURCES,
 * CBFS_E_WORKSPACE (before any launch); CBFS_E_HIP, CBFS_E_NOMEM.
 */
cbfs_status cbfs_run_batch(const cbfs_csr *g, const cbfs_batch *b, const cbfs_tuning *t,
                           uint32_t *dist, uint64_t *masks, int32_t *cluster_status,
                           void *workspace, size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------------------ *
 * cbfs_run_batch without any allocation, for callers that cannot allocate
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, outputs, statuses and kernels as
 * cbfs_run_batch, except that the workspace is the library's own device array
 * of CBFS_STATIC_SCRATCH_BYTES bytes (one per device, created when the library's
 * code is loaded on that device and held until the process ends).  The call
 * makes no device or pinned host allocation of any kind.
 *   - The current device must be the one that owns the stream and the
 *     buffers; the array's device address is looked up on the first call on
 *     each device.
 *   - The batch tables go up from pageable host memory, so the call waits
 *     for the stream once (after that upload).  CBFS_MODE_HOST_LOOP also
 *     waits once per round, as in cbfs_run_batch.
 *   - Every call on one device shares that device's array, which keeps the
 *     last call's contents (the search clears what it needs): calls that
 *     overlap on one device (other threads, other streams) race and give
 *     undefined outputs.  Serialise them.
 * Errors: those of cbfs_run_batch; CBFS_E_WORKSPACE (before any launch) when
 * cbfs_run_batch_workspace_size for these arguments exceeds
 * CBFS_STATIC_SCRATCH_BYTES.
 * ------------------------------------------------------------------------ */
#define CBFS_STATIC_SCRATCH_BYTES (64u << 20)
cbfs_status cbfs_run_batch_static(const cbfs_csr *g, const cbfs_batch *b, const cbfs_tuning *t,
                                  uint32_t *dist, uint64_t *masks, int32_t *cluster_status, void *stream);

/* Releases the host resources the library holds (the pinned staging buffers
 * and their events, the pinned counter words of the host loop, the calling
 * thread's profiling events), after waiting for the uploads still in flight.
 * Later calls allocate them again as needed.  Meant for process exit, while
 * the HIP runtime is still up (the Python binding registers it with atexit):
 * the library then holds no HIP object when the runtime is torn down.
 * Errors: CBFS_E_HIP (a release call failed; the rest are still released). */
cbfs_status cbfs_release(void);

/* ------------------------------------------------------------------------ *
 * Diagnostics (host).
 *
 * cbfs_last_run_stats: counts of the calling thread's last cbfs_run_batch,
 * waiting for it to finish.  frontier_vertices is the sum over groups and
 * rounds of |F_i|, frontier_arcs the sum of the out-degrees of those
 * frontiers (how many arcs a frontier-only traversal touches).  device_error:
 * 0, or 1 (persistent grid barrier timed out) / 2 (round limit hit), in which
 * case the call returns CBFS_E_HIP and the outputs are unspecified.
 *
 * cbfs_profile_enable(1) starts timing every kernel launch the calling thread
 * makes through this library (HIP events recorded on the call's stream around
 * each launch; previous records are dropped); cbfs_profile_enable(0) stops.
 * cbfs_profile_read waits for the recorded launches and returns, per kernel
 * kind, the launch count and the summed milliseconds (arrays of
 * CBFS_KERNEL_KINDS entries, host).
 * ------------------------------------------------------------------------ */
typedef struct {
    int64_t groups;            /* cluster groups searched                     */
    int64_t group_words;       /* words per vertex of each group              */
    int64_t slots;             /* groups searched side by side                */
    int64_t mode;              /* CBFS_MODE_HOST_LOOP or CBFS_MODE_PERSISTENT */
    int64_t rounds;            /* level-loop rounds, summed over groups       */
    int64_t push_rounds;
    int64_t pull_rounds;
    int64_t frontier_vertices; /* sum of |F_i|                                */
    int64_t frontier_arcs;     /* sum of deg over F_i                         */
    int64_t device_error;
    int64_t persistent_blocks; /* grid of the persistent launch (0 in host-loop mode) */
    int64_t pull_frontier_vertices; /* sum of |F_i| over the pull rounds           */
} cbfs_run_stats;

cbfs_status cbfs_last_run_stats(cbfs_run_stats *out);

enum {
    CBFS_KERNEL_TILES = 0,
    CBFS_KERNEL_INIT = 1,
    CBFS_KERNEL_SEED = 2,
    CBFS_KERNEL_PUSH = 3,
    CBFS_KERNEL_PULL = 4,
    CBFS_KERNEL_FINALIZE = 5,
    CBFS_KERNEL_PERSISTENT = 6,
    CBFS_KERNEL_LABELS = 7,
    CBFS_KERNEL_QUERY = 8,
    CBFS_KERNEL_LOCAL = 9,
    CBFS_KERNEL_PLL = 10,
    CBFS_KERNEL_KINDS = 11
};
cbfs_status cbfs_profile_enable(int32_t enable);
cbfs_status cbfs_profile_read(int64_t *launches, double *total_ms);

/* ------------------------------------------------------------------------ *
 * Autotuner for batched launches (Lemma "word_cost" and Theorem
 * "batchBFScost", Section 3.2: the cost of a search is set by the arcs it
 * touches times the words per vertex; which packing, direction thresholds
 * and launch form are fastest depends on the graph).  Coordinate descent
 * over launch mode, group width (words per vertex), the push/pull
 * thresholds alpha and gamma, and in persistent mode the number of groups
 * searched side by side: each candidate runs cbfs_run_batch twice (one
 * warm-up) on the first sample_clusters clusters of the batch, timed from
 * host to stream completion, and the fastest is kept.  No knob changes an
 * output bit, so the choice only affects speed.
 *
 * start:      knobs to start from (nullable: library defaults); fields the
 *             search does not touch are kept.
 * sample_clusters: 0 = min(C, 16).
 * dist/masks/cluster_status: device outputs for at least sample_clusters
 *             clusters (the batch's own output buffers may be passed; the
 *             first clusters' outputs are overwritten by the trials).
 * workspace:  device memory; a candidate whose workspace does not fit is
 *             skipped (reported with ms < 0).  cbfs_autotune_workspace_size
 *             gives the size that fits every candidate.
 * best:       receives the fastest knobs.
 * trials:     nullable host array of max_trials entries receiving every
 *             candidate tried, in order; *num_trials receives the count.
 * The call synchronises the stream.  Errors: those of cbfs_run_batch,
 * returned from the first candidate that fails.
 * ------------------------------------------------------------------------ */
typedef struct {
    cbfs_tuning tuning;
    float ms;               /* wall time of the timed run; < 0 if skipped */
    int32_t mode;           /* the mode the run used (CBFS_MODE_HOST_LOOP or _PERSISTENT) */
} cbfs_trial;

size_t cbfs_autotune_workspace_size(const cbfs_csr *g, const cbfs_batch *b, int32_t sample_clusters);
cbfs_status cbfs_autotune(const cbfs_csr *g, const cbfs_batch *b, const cbfs_tuning *start,
                          int32_t sample_clusters, uint32_t *dist, uint64_t *masks, int32_t *cluster_status,
                          void *workspace, size_t workspace_bytes, void *stream, cbfs_tuning *best,
                          cbfs_trial *trials, int32_t max_trials, int32_t *num_trials);

/* ------------------------------------------------------------------------ *
 * Landmark-labeling queries over cluster labels (Section 4.2; Algorithm
 * "Framework of Landmark Labeling", Query).  query(s, t) = min over clusters c
 * and sources x of c of d(x, s) + d(x, t); per cluster this is
 * d(c,s) + d(c,t) plus the lowest offset sum a + b < 0 whose subsets
 * intersect (M_a(s) & M_b(t) non-empty), else plus 0: the center alone gives
 * offset sum 0.  A pair with a + b < 0 has both offsets <= R - 1, so the
 * labels keep offsets -R .. R-1 (2R planes; none for R = 0).  Requires one
 * mask word per cluster (k <= 64).
 *
 * cbfs_labels_pack: cluster-major C-BFS outputs (dist [C][n], masks
 * [C][2R+1][n][1], device) -> vertex-major labels dist_vm [n][C] and
 * mask_vm [n][C][2R] (planes o = -R .. R-1, device; may be NULL for R = 0),
 * so one query reads two contiguous rows.
 *
 * cbfs_query_batch: ans[j] = query(s[j], t[j]) (device arrays of length q),
 * CBFS_UNREACHED when no cluster reaches both endpoints.  Vertex ids are not
 * range-checked on the device: out-of-range ids are the caller's error.
 * Errors: CBFS_E_ARG (null pointers, sizes, R outside [0, 1024]); CBFS_E_HIP.
 * ------------------------------------------------------------------------ */
typedef struct {
    int64_t n;               /* vertices                        */
    int32_t num_clusters;    /* C                               */
    int32_t radius;          /* R                               */
    const uint32_t *dist_vm; /* device [n][C]                   */
    const uint64_t *mask_vm; /* device [n][C][2R]               */
} cbfs_labels;

cbfs_status cbfs_labels_pack(const uint32_t *dist, const uint64_t *masks, int32_t num_clusters,
                             int64_t n, int32_t radius, uint32_t *dist_vm, uint64_t *mask_vm,
                             void *stream);
cbfs_status cbfs_query_batch(const cbfs_labels *L, int64_t q, const int32_t *s, const int32_t *t,
                             uint32_t *ans, void *stream);

/* ------------------------------------------------------------------------ *
 * Compact labels under a memory budget (Section 5.3, landmark-labeling
 * experiments): a cluster of at most w sources stores, per vertex, a one-byte
 * distance and its 2R subsets as w-bit words, 1 + 2R w / 8 bytes (R = 1:
 * 3 bytes at w = 8, 17 at w = 64); with a budget of t bytes per vertex, t /
 * (1 + 2R w / 8) clusters fit.
 *
 * cbfs_labels_pack_compact: cluster-major C-BFS outputs (dist [C][n], masks
 * [C][2R+1][n][1], device) -> dist8 [n][C] (uint8, 255 = unreached) and
 * masks_out [n][C][2R] w-bit words (offsets -R .. R-1; uint8/16/32/64 for
 * w = 8/16/32/64; may be NULL for R = 0), device, caller-owned.  Waits for the
 * stream at its end.  Errors: CBFS_E_ARG; CBFS_E_RANGE (a distance >= 255, or
 * a source bit at or above w: the outputs are then not usable); CBFS_E_HIP.
 *
 * cbfs_query_batch_compact: cbfs_query_batch over compact labels (the same
 * answers while every distance is below 255).
 * ------------------------------------------------------------------------ */
typedef struct {
    int64_t n;              /* vertices                                  */
    int32_t num_clusters;   /* C                                         */
    int32_t radius;         /* R                                         */
    int32_t w;              /* mask width in bits: 8, 16, 32 or 64       */
    const uint8_t *dist8;   /* device [n][C], 255 = unreached            */
    const void *masks;      /* device [n][C][2R] w-bit words             */
} cbfs_compact_labels;

cbfs_status cbfs_labels_pack_compact(const uint32_t *dist, const uint64_t *masks, int32_t num_clusters, int64_t n,
                                     int32_t radius, int32_t w, uint8_t *dist8, void *masks_out, void *stream);
cbfs_status cbfs_query_batch_compact(const cbfs_compact_labels *L, int64_t q, const int32_t *s, const int32_t *t,
                                     uint32_t *ans, void *stream);

/* ------------------------------------------------------------------------ *
 * Bidirectional local search of the query path (Appendix B, "Applying
 * Bi-Directional Search in the Queries").  From each endpoint a BFS in FIFO
 * order (root first, then each dequeued vertex's neighbours in the order of
 * its CSR row, a vertex counted when first seen) discovers its first tau
 * vertices, each with its exact distance; the local answer is the lowest
 * d(s, x) + d(t, x) over the vertices both searches discovered, none if they
 * share none.  The common vertices act as landmarks found at query time, so
 * the final answer is the minimum of the local and the landmark answers.
 *
 * cbfs_query_local: ans[j] = min(ans[j], local(s[j], t[j])) for j < q (device
 * arrays; ans unsigned, CBFS_UNREACHED as "none"): run it after
 * cbfs_query_batch on the same stream for the combined answer, or on ans
 * filled with CBFS_UNREACHED for the local answer alone.  g is the graph the
 * labels were built on (device CSR).  1 <= tau <= CBFS_LOCAL_TAU_MAX; the
 * search state lives in on-chip memory (8 bytes per set slot, the set holding
 * at least 1.5 (tau + 64) slots, plus 12 bytes per list entry: about 50 KiB
 * per query at tau = 2048).  Vertex ids are not range-checked on the device.
 * Errors: CBFS_E_ARG (null pointers, sizes, tau out of range); CBFS_E_HIP.
 * ------------------------------------------------------------------------ */
#define CBFS_LOCAL_TAU_MAX 2048
cbfs_status cbfs_query_local(const cbfs_csr *g, int64_t q, const int32_t *s, const int32_t *t, int32_t tau,
                             uint32_t *ans, void *stream);

/* ------------------------------------------------------------------------ *
 * Exact 2-hop distance oracle (the paper's appendix on the exact distance
 * oracle: pruned landmark labeling, whose phase 1 is a C-BFS batch and whose
 * phase 2 runs a pruned BFS from every remaining vertex, in batches of growing
 * size searched side by side).
 *
 * Phase 1: the center-relative labels of a C-BFS batch (cbfs_run_batch, then
 * cbfs_labels_pack), passed as bp; they answer the shortest path through any
 * of the batch's sources.  bp may be NULL (no phase 1).
 *
 * cbfs_pll_build: phase 2.  order (device [count]) lists the roots by rank
 * (rank k = order[k]); the phase-1 sources need not be listed (the index
 * already covers every pair through them, so they would add nothing).  Batch i
 * holds the next b_i roots: b_0 = first, b_{i+1} = min(max_batch,
 * floor(b_i * growth)).  Root h of a batch runs a BFS; at vertex u, reached at
 * distance d, the index as it stood when the batch began answers (h, u) (the
 * phase-1 labels, and the ranks r with (r, d_hr) in the label of h and
 * (r, d_ur) in the label of u: d_hr + d_ur); an answer at most d prunes u (no
 * label, not expanded), else (rank(h), d) joins u's label and u's neighbours
 * are visited.  Labels added in a batch are seen from the next batch on, so
 * the result does not depend on how the device runs a batch.
 * Outputs (device, caller-owned): lab_cnt [n] and labels [n][label_cap], the
 * entries of vertex v being labels[v][0 .. lab_cnt[v]) = (rank << 32) |
 * distance, sorted by rank.  1 <= label_cap <= CBFS_PLL_LABEL_CAP_MAX.
 * Workspace: cbfs_pll_workspace_size(n, params) bytes (per search slot a
 * visited bitmap and two frontier queues of n entries).  The call waits for
 * the stream at its end, to read the overflow flag.
 * Errors: CBFS_E_ARG; CBFS_E_WORKSPACE (workspace too small, or a vertex's
 * label would exceed label_cap: the outputs are then incomplete); CBFS_E_HIP.
 *
 * cbfs_pll_query: ans[j] = the lower of the phase-1 answer (bp, may be NULL)
 * and min over ranks in both labels of the two distances' sum, for device
 * arrays s, t of length q; exact when the labels come from cbfs_pll_build over
 * all non-source vertices.  CBFS_UNREACHED when nothing covers the pair.
 * ------------------------------------------------------------------------ */
#define CBFS_PLL_LABEL_CAP_MAX 4096
#define CBFS_PLL_PHASE1_WORDS_MAX 2048 /* phase-1 mask words per vertex (clusters x 2R) */
typedef struct {
    int32_t first;     /* roots in the first batch: 0 = 200                          */
    float growth;      /* batch growth factor (>= 1): 0 = 1.5                          */
    int32_t max_batch; /* largest batch: 0 = 1000                                      */
    int32_t slots;     /* roots searched at once (a batch runs in chunks of this many):
                          0 = min(max_batch, 1024)                                     */
} cbfs_pll_params;

size_t cbfs_pll_workspace_size(int64_t n, const cbfs_pll_params *params);
cbfs_status cbfs_pll_build(const cbfs_csr *g, const cbfs_labels *bp, const int32_t *order, int64_t count,
                           const cbfs_pll_params *params, int32_t label_cap, int32_t *lab_cnt, uint64_t *labels,
                           void *workspace, size_t workspace_bytes, void *stream);
cbfs_status cbfs_pll_query(const cbfs_labels *bp, int64_t n, int32_t label_cap, const int32_t *lab_cnt,
                           const uint64_t *labels, int64_t q, const int32_t *s, const int32_t *t, uint32_t *ans,
                           void *stream);

#ifdef __cplusplus
}
#endif
#endif /* CBFS_H */
