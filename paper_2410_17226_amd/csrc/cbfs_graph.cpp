// Host-side graph ingest and cluster selection of libcbfs (cbfs.h).
//
// Graph ingest: the paper runs on undirected graphs (Section 5 setup) and its
// applications assume them (Section 4); cbfs_build_csr turns a raw edge list
// into the symmetric, duplicate-free, loop-free CSR of the largest connected
// component that the kernels traverse.
//
// Cluster selection: clusters are built around centers (Section 4.2 picks
// high-degree centers and their nearby vertices); here a cluster is its center
// followed by the lowest-id vertices within `hops`.
#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

#include "cbfs.h"
#include "cbfs_internal.h"

namespace {

template <class F>
void parallel_for(int64_t n, F f)
{
    unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if (n < 65536 || nt == 1) {
        f(0, n);
        return;
    }
    std::vector<std::thread> th;
    int64_t chunk = (n + nt - 1) / nt;
    for (unsigned t = 0; t < nt; t++) {
        int64_t lo = t * chunk, hi = std::min<int64_t>(n, lo + chunk);
        if (lo >= hi) break;
        th.emplace_back([=] { f(lo, hi); });
    }
    for (auto &x : th) x.join();
}

}  // namespace

extern "C" cbfs_status cbfs_build_csr(int64_t n_in, int64_t num_edges, const int64_t *src,
                                      const int64_t *dst, uint32_t flags, int32_t *row_ptr,
                                      int32_t *col, int64_t col_capacity, int64_t *n_out,
                                      int64_t *m_out, int64_t *old_to_new)
{
    if (n_in <= 0 || n_in >= INT32_MAX || num_edges < 0 || !row_ptr || !n_out || !m_out ||
        (num_edges > 0 && (!src || !dst)) || (flags & ~uint32_t(CBFS_CSR_ALL)))
        return cbfs::fail(CBFS_E_ARG, "cbfs_build_csr: bad argument");
    try {
        std::atomic<int> bad{0};
        parallel_for(num_edges, [&](int64_t lo, int64_t hi) {
            for (int64_t e = lo; e < hi; e++)
                if (src[e] < 0 || src[e] >= n_in || dst[e] < 0 || dst[e] >= n_in) bad = 1;
        });
        if (bad) return cbfs::fail(CBFS_E_RANGE, "cbfs_build_csr: endpoint outside [0, n_in)");
        const bool sym = flags & CBFS_CSR_SYMMETRIZE, dedup = flags & CBFS_CSR_DEDUP,
                   noloop = flags & CBFS_CSR_DROP_SELF_LOOPS, lcc = flags & CBFS_CSR_KEEP_LCC;

        // 1. bucket arcs by tail (counting sort)
        std::vector<int64_t> start(n_in + 1, 0);
        for (int64_t e = 0; e < num_edges; e++) {
            if (noloop && src[e] == dst[e]) continue;
            start[src[e] + 1]++;
            if (sym) start[dst[e] + 1]++;
        }
        for (int64_t v = 0; v < n_in; v++) start[v + 1] += start[v];
        std::vector<int32_t> arcs(std::max<int64_t>(1, start[n_in]));
        {
            std::vector<int64_t> pos(start.begin(), start.end() - 1);
            for (int64_t e = 0; e < num_edges; e++) {
                if (noloop && src[e] == dst[e]) continue;
                arcs[pos[src[e]]++] = int32_t(dst[e]);
                if (sym) arcs[pos[dst[e]]++] = int32_t(src[e]);
            }
        }
        // 2. sort and dedup each row in place; len[v] = kept row length
        std::vector<int64_t> len(n_in);
        parallel_for(n_in, [&](int64_t lo, int64_t hi) {
            for (int64_t v = lo; v < hi; v++) {
                int32_t *b = arcs.data() + start[v], *e = arcs.data() + start[v + 1];
                std::sort(b, e);
                if (dedup) e = std::unique(b, e);
                len[v] = e - b;
            }
        });
        // 3. components by BFS in ascending id order: the first component found
        //    of each size holds the smallest id among components of that size
        std::vector<uint8_t> keep(n_in, 1);
        if (lcc) {
            std::vector<int32_t> comp(n_in, -1), queue(n_in);
            // arcs are followed in both directions: add in-arcs if not symmetrized
            std::vector<int64_t> rstart;
            std::vector<int32_t> rarcs;
            if (!sym) {
                rstart.assign(n_in + 1, 0);
                for (int64_t v = 0; v < n_in; v++)
                    for (int64_t j = 0; j < len[v]; j++) rstart[arcs[start[v] + j] + 1]++;
                for (int64_t v = 0; v < n_in; v++) rstart[v + 1] += rstart[v];
                rarcs.resize(std::max<int64_t>(1, rstart[n_in]));
                std::vector<int64_t> p(rstart.begin(), rstart.end() - 1);
                for (int64_t v = 0; v < n_in; v++)
                    for (int64_t j = 0; j < len[v]; j++) rarcs[p[arcs[start[v] + j]]++] = int32_t(v);
            }
            int32_t ncomp = 0, best = -1;
            int64_t best_size = 0;
            for (int64_t r = 0; r < n_in; r++) {
                if (comp[r] >= 0) continue;
                int64_t head = 0, tail = 0;
                comp[r] = ncomp;
                queue[tail++] = int32_t(r);
                while (head < tail) {
                    int32_t u = queue[head++];
                    for (int64_t j = 0; j < len[u]; j++) {
                        int32_t w = arcs[start[u] + j];
                        if (comp[w] < 0) { comp[w] = ncomp; queue[tail++] = w; }
                    }
                    if (!sym)
                        for (int64_t j = rstart[u]; j < rstart[u + 1]; j++) {
                            int32_t w = rarcs[j];
                            if (comp[w] < 0) { comp[w] = ncomp; queue[tail++] = w; }
                        }
                }
                if (tail > best_size) { best_size = tail; best = ncomp; }
                ncomp++;
            }
            for (int64_t v = 0; v < n_in; v++) keep[v] = comp[v] == best;
        }
        // 4. renumber kept vertices in ascending id order and compact
        std::vector<int64_t> newid(n_in);
        int64_t n = 0;
        for (int64_t v = 0; v < n_in; v++) newid[v] = keep[v] ? n++ : -1;
        std::vector<int64_t> kept_len(n_in, 0);
        parallel_for(n_in, [&](int64_t lo, int64_t hi) {
            for (int64_t v = lo; v < hi; v++) {
                if (!keep[v]) continue;
                int64_t c = 0;
                for (int64_t j = 0; j < len[v]; j++) c += keep[arcs[start[v] + j]];
                kept_len[v] = c;
            }
        });
        int64_t m = 0;
        std::vector<int64_t> out_start(n_in);
        for (int64_t v = 0; v < n_in; v++) {
            out_start[v] = m;
            m += kept_len[v];
        }
        if (m >= INT32_MAX || m > col_capacity || (m > 0 && !col))
            return cbfs::fail(CBFS_E_WORKSPACE, "cbfs_build_csr: col capacity too small or m >= 2^31");
        parallel_for(n_in, [&](int64_t lo, int64_t hi) {
            for (int64_t v = lo; v < hi; v++) {
                if (!keep[v]) continue;
                int64_t p = out_start[v];
                for (int64_t j = 0; j < len[v]; j++) {
                    int32_t w = arcs[start[v] + j];
                    if (keep[w]) col[p++] = int32_t(newid[w]);
                }
                row_ptr[newid[v]] = int32_t(out_start[v]);
            }
        });
        row_ptr[n] = int32_t(m);
        if (old_to_new) std::memcpy(old_to_new, newid.data(), sizeof(int64_t) * n_in);
        *n_out = n;
        *m_out = m;
        return CBFS_OK;
    } catch (const std::bad_alloc &) {
        return cbfs::fail(CBFS_E_NOMEM, "cbfs_build_csr: out of host memory");
    }
}

extern "C" cbfs_status cbfs_top_degree(int64_t n, const int32_t *row_ptr, int32_t count, int32_t *out)
{
    if (n <= 0 || !row_ptr || !out || count < 0 || count > n)
        return cbfs::fail(CBFS_E_ARG, "cbfs_top_degree: bad argument");
    try {
        std::vector<int32_t> ids(n);
        for (int64_t v = 0; v < n; v++) ids[v] = int32_t(v);
        auto deg = [&](int32_t v) { return row_ptr[v + 1] - row_ptr[v]; };
        std::partial_sort(ids.begin(), ids.begin() + count, ids.end(), [&](int32_t a, int32_t b) {
            return deg(a) != deg(b) ? deg(a) > deg(b) : a < b;
        });
        std::copy(ids.begin(), ids.begin() + count, out);
        return CBFS_OK;
    } catch (const std::bad_alloc &) {
        return cbfs::fail(CBFS_E_NOMEM, "cbfs_top_degree: out of host memory");
    }
}

extern "C" cbfs_status cbfs_select_clusters(int64_t n, const int32_t *row_ptr, const int32_t *col,
                                            int32_t num_centers, const int32_t *centers,
                                            int32_t k_max, int32_t hops, int32_t *cluster_ptr,
                                            int32_t *sources, int64_t sources_capacity)
{
    if (n <= 0 || !row_ptr || !col || num_centers < 0 || (num_centers > 0 && !centers) ||
        hops < 0 || !cluster_ptr || !sources)
        return cbfs::fail(CBFS_E_ARG, "cbfs_select_clusters: bad argument");
    if (k_max < 1 || k_max > CBFS_MAX_SOURCES)
        return cbfs::fail(CBFS_E_TOO_MANY_SOURCES, "cbfs_select_clusters: k_max outside 1..256");
    for (int32_t j = 0; j < num_centers; j++)
        if (centers[j] < 0 || centers[j] >= n)
            return cbfs::fail(CBFS_E_RANGE, "cbfs_select_clusters: center outside [0, n)");
    try {
        // hop-limited BFS with a stamp array; the ball is collected, sorted and cut
        std::vector<int32_t> stamp(n, -1), frontier, next, ball;
        int64_t pos = 0;
        cluster_ptr[0] = 0;
        for (int32_t j = 0; j < num_centers; j++) {
            const int32_t c = centers[j];
            ball.clear();
            frontier.assign(1, c);
            stamp[c] = j;
            for (int32_t h = 0; h < hops && !frontier.empty(); h++) {
                next.clear();
                for (int32_t u : frontier)
                    for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; e++) {
                        int32_t w = col[e];
                        if (stamp[w] != j) {
                            stamp[w] = j;
                            next.push_back(w);
                        }
                    }
                ball.insert(ball.end(), next.begin(), next.end());
                frontier.swap(next);
            }
            size_t take = std::min<size_t>(ball.size(), size_t(k_max - 1));
            std::partial_sort(ball.begin(), ball.begin() + take, ball.end());
            if (pos + 1 + int64_t(take) > sources_capacity)
                return cbfs::fail(CBFS_E_WORKSPACE, "cbfs_select_clusters: sources capacity too small");
            sources[pos++] = c;
            for (size_t i = 0; i < take; i++) sources[pos++] = ball[i];
            cluster_ptr[j + 1] = int32_t(pos);
        }
        return CBFS_OK;
    } catch (const std::bad_alloc &) {
        return cbfs::fail(CBFS_E_NOMEM, "cbfs_select_clusters: out of host memory");
    }
}

// Landmark clusters as the paper builds them (Section 4.2, "Selecting
// Landmarks in Clusters"): repeatedly take the unmarked vertex of highest
// degree as a center; among its unmarked vertices within floor(d/2) hops take
// the k-1 of highest degree; mark the whole cluster so that no later cluster
// reuses a vertex.  Degree ties go to the lower id.  Sources are listed center
// first, then in selection order (degree descending).  Stops early when every
// vertex is marked.
extern "C" cbfs_status cbfs_select_landmarks(int64_t n, const int32_t *row_ptr, const int32_t *col,
                                             int32_t num_clusters, int32_t k, int32_t diameter,
                                             int32_t *cluster_ptr, int32_t *sources, int64_t sources_capacity,
                                             int32_t *num_selected)
{
    if (n <= 0 || !row_ptr || !col || num_clusters < 0 || diameter < 0 || !cluster_ptr || !sources ||
        !num_selected)
        return cbfs::fail(CBFS_E_ARG, "cbfs_select_landmarks: bad argument");
    if (k < 1 || k > CBFS_MAX_SOURCES)
        return cbfs::fail(CBFS_E_TOO_MANY_SOURCES, "cbfs_select_landmarks: k outside 1..256");
    try {
        // vertices by degree descending, ties by ascending id
        std::vector<int32_t> order(n);
        for (int64_t v = 0; v < n; v++) order[v] = (int32_t)v;
        auto deg = [&](int32_t v) { return row_ptr[v + 1] - row_ptr[v]; };
        auto before = [&](int32_t a, int32_t b) { return deg(a) != deg(b) ? deg(a) > deg(b) : a < b; };
        std::stable_sort(order.begin(), order.end(), before);
        std::vector<char> marked(n, 0);
        std::vector<int32_t> stamp(n, -1), frontier, next, ball;
        const int32_t hops = diameter / 2;
        int64_t pos = 0, scan = 0;
        int32_t made = 0;
        cluster_ptr[0] = 0;
        while (made < num_clusters) {
            while (scan < n && marked[order[scan]]) scan++;
            if (scan == n) break;
            const int32_t c = order[scan];
            ball.clear();
            frontier.assign(1, c);
            stamp[c] = made;
            for (int32_t h = 0; h < hops && !frontier.empty(); h++) {
                next.clear();
                for (int32_t u : frontier)
                    for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; e++) {
                        const int32_t w = col[e];
                        if (stamp[w] != made) {
                            stamp[w] = made;
                            next.push_back(w);
                            if (!marked[w]) ball.push_back(w);
                        }
                    }
                frontier.swap(next);
            }
            const size_t take = std::min<size_t>(ball.size(), size_t(k - 1));
            std::partial_sort(ball.begin(), ball.begin() + take, ball.end(), before);
            if (pos + 1 + int64_t(take) > sources_capacity)
                return cbfs::fail(CBFS_E_WORKSPACE, "cbfs_select_landmarks: sources capacity too small");
            sources[pos++] = c;
            marked[c] = 1;
            for (size_t i = 0; i < take; i++) {
                sources[pos++] = ball[i];
                marked[ball[i]] = 1;
            }
            cluster_ptr[++made] = int32_t(pos);
        }
        *num_selected = made;
        return CBFS_OK;
    } catch (const std::bad_alloc &) {
        return cbfs::fail(CBFS_E_NOMEM, "cbfs_select_landmarks: out of host memory");
    }
}
