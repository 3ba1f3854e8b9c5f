"""Pins of the CPU oracle against things other than itself (no GPU needed).

* single-source distances against scipy's shortest paths (a library routine);
* the encoded cluster distance vectors against the definition evaluated on an
  independent all-pairs distance matrix, against closed forms (path, cycle,
  complete graph, star, undamaged grid with Manhattan distances) and a
  hand-worked fixture;
* invariants from the Fact / Corollary of Section 3.1;
* the two query oracles against each other, against true distances (one-sided
  error, Section 4.2) and against the fixture;
* the bidirectional local search (Appendix B) against scipy's BFS order and
  all-pairs distances, the path closed form, full coverage and tau = 1;
* the BFS certificate against planted mistakes;
* the oracle's C cleanup against its numpy/scipy form.
"""
import os

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import breadth_first_order, shortest_path

import oracle
import synth

U32MAX = np.uint32(0xFFFFFFFF)


def csr_of(n, edges):
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    return oracle.clean_csr(n, e[:, 0], e[:, 1], flags=7)[:2]


def apsp(row_ptr, col):
    n = row_ptr.size - 1
    A = sp.csr_matrix((np.ones(col.size), col, row_ptr), shape=(n, n))
    D = shortest_path(A, method="D", unweighted=True, directed=True)
    D[np.isinf(D)] = -1
    return D.astype(np.int64)


def encode_from_apsp(D, cluster, R, W=None):
    """The subset equation re-based on the center, evaluated on a distance matrix."""
    n = D.shape[0]
    k = len(cluster)
    W = W or (k + 63) // 64
    dist = np.full(n, U32MAX, dtype=np.uint32)
    masks = np.zeros((2 * R + 1, n, W), dtype=np.uint64)
    ok = True
    c = cluster[0]
    for v in range(n):
        if D[c, v] < 0:
            ok &= all(D[s, v] < 0 for s in cluster)
            continue
        dist[v] = D[c, v]
        for i, s in enumerate(cluster):
            if D[s, v] < 0:
                ok = False
                continue
            o = D[s, v] - D[c, v]
            if abs(o) > R:
                ok = False
                continue
            masks[o + R, v, i // 64] |= np.uint64(1) << np.uint64(i % 64)
    return dist, masks, ok


def small_graphs():
    out = []
    for seed in range(6):
        out.append(("gnp", synth.random_graph(60, 0.06, seed)))
        out.append(("tree", synth.random_tree(50, seed)))
    out.append(("grid", synth.grid_edges(9, 0.2, seed=3)))
    out.append(("gnp_sparse_disconnected", synth.random_graph(80, 0.015, 7)))
    return out


@pytest.mark.parametrize("name,g", small_graphs())
def test_bfs_matches_library_shortest_paths(name, g):
    n, s, d = g
    rp, col, _ = oracle.clean_csr(n, s, d, flags=7)
    D = apsp(rp, col)
    for src in range(0, rp.size - 1, 7):
        assert np.array_equal(oracle.bfs(rp, col, src), D[src])


@pytest.mark.parametrize("name,g", small_graphs())
def test_cbfs_equals_definition_on_apsp(name, g):
    n, s, d = g
    rp, col, _ = oracle.clean_csr(n, s, d, flags=7)
    D = apsp(rp, col)
    nv = rp.size - 1
    rng = np.random.default_rng(11)
    clusters = []
    for c in range(nv):  # every vertex as a star center
        clusters.append(oracle.cluster_around(rp, col, c, 64, 1))
    for c in rng.choice(nv, size=min(10, nv), replace=False):
        clusters.append(oracle.cluster_around(rp, col, int(c), 64, 2))
    for R in (1, 2):
        cp = np.zeros(len(clusters) + 1, np.int32)
        cp[1:] = np.cumsum([x.size for x in clusters])
        dist, masks, status = oracle.cbfs(rp, col, cp, np.concatenate(clusters), R)
        for ci, cl in enumerate(clusters):
            ed, em, ok = encode_from_apsp(D, list(cl), R)
            assert (status[ci] == 0) == ok, (ci, R)
            if ok:
                assert np.array_equal(dist[ci], ed)
                assert np.array_equal(masks[ci], em)


def encode_min_from_apsp(D, cluster, d, W=None):
    """Section 3.1's subset equation evaluated on a distance matrix:
    Delta_v = min_s delta(s,v), S_v[i] = {s : delta(s,v) = Delta_v + i}, i <= d."""
    n = D.shape[0]
    k = len(cluster)
    W = W or (k + 63) // 64
    delta = np.full(n, U32MAX, dtype=np.uint32)
    subs = np.zeros((d + 1, n, W), dtype=np.uint64)
    ok = True
    for v in range(n):
        ds = [D[s, v] for s in cluster]
        if all(x < 0 for x in ds):
            continue
        if any(x < 0 for x in ds):
            ok = False
            continue
        m = min(ds)
        delta[v] = m
        for i, x in enumerate(ds):
            if x - m > d:
                ok = False
                continue
            subs[x - m, v, i // 64] |= np.uint64(1) << np.uint64(i % 64)
    return delta, subs, ok


@pytest.mark.parametrize("name,g", small_graphs())
def test_cbfs_min_equals_definition_on_apsp(name, g):
    """The paper's own encoding <S_v[0..d], Delta_v> against the subset
    equation evaluated on scipy's all-pairs distances, for balls of radius h
    (diameter at most 2h) declared with diameters 2h-1 (violations possible),
    2h and 2h+1, and for random scattered clusters."""
    n, s, d = g
    rp, col, _ = oracle.clean_csr(n, s, d, flags=7)
    D = apsp(rp, col)
    nv = rp.size - 1
    rng = np.random.default_rng(5)
    for h in (1, 2, 3):
        clusters = [oracle.cluster_around(rp, col, int(c), 64, h) for c in rng.choice(nv, size=min(8, nv), replace=False)]
        clusters.append(rng.choice(nv, size=min(10, nv), replace=False).astype(np.int32))
        cp = np.zeros(len(clusters) + 1, np.int32)
        cp[1:] = np.cumsum([x.size for x in clusters])
        for dd in (2 * h - 1, 2 * h, 2 * h + 1):
            delta, subs, status = oracle.cbfs_min(rp, col, cp, np.concatenate(clusters), dd)
            for ci, cl in enumerate(clusters):
                ed, es, ok = encode_min_from_apsp(D, list(cl), dd)
                assert (status[ci] == 0) == ok, (name, h, dd, ci)
                if ok:
                    assert np.array_equal(delta[ci], ed)
                    assert np.array_equal(subs[ci], es)
                else:
                    assert (delta[ci] == U32MAX).all() and not subs[ci].any()


def test_cbfs_min_path_closed_form():
    """Path 0-1-...-39, cluster = the consecutive vertices a..b: Delta_v is the
    distance to the nearer end of [a, b] (0 inside), and source s_j sits in
    subset |s_j - v| - Delta_v."""
    n, a, b = 40, 12, 17
    rp, col = csr_of(n, [(i, i + 1) for i in range(n - 1)])
    S = list(range(a, b + 1))
    dd = b - a
    delta, subs, st = oracle.cbfs_min(rp, col, [0, len(S)], S, dd)
    assert st[0] == 0
    for v in range(n):
        m = a - v if v < a else (v - b if v > b else 0)
        assert delta[0, v] == m
        for j, sj in enumerate(S):
            i = abs(sj - v) - m
            assert (int(subs[0, i, v, 0]) >> j) & 1, (v, j)
    # each source exactly once per vertex
    total = np.zeros(n, np.int64)
    for i in range(dd + 1):
        total += np.array([bin(int(x)).count("1") for x in subs[0, i, :, 0]])
    assert (total == len(S)).all()


def test_cbfs_min_complete_graph_and_invariants():
    """K_n with a cluster of k vertices: a member sees itself at subset 0 and
    the others at 1; a non-member sees all k at subset 0 (Delta = 1)."""
    n, k = 12, 5
    rp, col = csr_of(n, [(i, j) for i in range(n) for j in range(i + 1, n)])
    S = [3, 0, 7, 9, 11]
    delta, subs, st = oracle.cbfs_min(rp, col, [0, k], S, 1)
    assert st[0] == 0
    full = (1 << k) - 1
    for v in range(n):
        if v in S:
            j = S.index(v)
            assert delta[0, v] == 0 and subs[0, 0, v, 0] == 1 << j and subs[0, 1, v, 0] == full ^ (1 << j)
        else:
            assert delta[0, v] == 1 and subs[0, 0, v, 0] == full and subs[0, 1, v, 0] == 0
    # diameter 0 for a cluster of two distinct vertices is broken
    _, _, st0 = oracle.cbfs_min(rp, col, [0, 2], S[:2], 0)
    assert st0[0] == -5


def test_cbfs_min_agrees_with_center_relative_on_stars():
    """Both encodings of one search: the center's bit sits in subset j_c, and
    then d(c,v) = Delta_v + j_c and M[o] = S_v[j_c + o] (the re-basing of the
    star storage of Section 5.3)."""
    n, s, d = synth.rmat_edges(9, 8, seed=3)
    rp, col, _ = oracle.clean_csr(n, s, d)
    cp, src = oracle.build_clusters(rp, col, oracle.top_degree(rp, 6), 64, 1)
    delta, subs, st = oracle.cbfs_min(rp, col, cp, src, 2)
    dist, masks, st2 = oracle.cbfs(rp, col, cp, src, R=2)
    assert (st == 0).all() and (st2 == 0).all()
    for c in range(cp.size - 1):
        reach = delta[c] != U32MAX
        jc = np.argmax((subs[c, :, :, 0] & np.uint64(1)) != 0, axis=0)
        assert np.array_equal(dist[c][reach], delta[c][reach] + jc[reach])
        for v in np.nonzero(reach)[0][:400]:
            for o in range(-2, 3):
                i = jc[v] + o
                want = subs[c, i, v, 0] if 0 <= i <= 2 else 0
                assert masks[c, o + 2, v, 0] == want


def test_path_graph_closed_form():
    n = 40
    rp, col = csr_of(n, [(i, i + 1) for i in range(n - 1)])
    c = 17
    dist, masks, st = oracle.cbfs(rp, col, [0, 3], [c, c - 1, c + 1], R=1)
    assert st[0] == 0
    for v in range(n):
        assert dist[0, v] == abs(v - c)
        m = masks[0, :, v, 0]
        if v > c:      # c+1 (bit 2) is one nearer, c-1 (bit 1) one farther
            assert list(m) == [0b100, 0b001, 0b010]
        elif v < c:
            assert list(m) == [0b010, 0b001, 0b100]
        else:          # at the center both neighbours are one farther
            assert list(m) == [0, 0b001, 0b110]


def test_cycle_closed_form():
    n = 31
    rp, col = csr_of(n, [(i, (i + 1) % n) for i in range(n)])
    c = 5
    cl = [c, c - 1, c + 1]
    dist, masks, st = oracle.cbfs(rp, col, [0, 3], cl, R=1)
    cyc = lambda a, b: min(abs(a - b), n - abs(a - b))  # noqa: E731
    for v in range(n):
        assert dist[0, v] == cyc(c, v)
        for i, s in enumerate(cl):
            o = cyc(s, v) - cyc(c, v)
            assert (masks[0, o + 1, v, 0] >> np.uint64(i)) & np.uint64(1) == 1


def test_complete_graph_closed_form():
    n = 12
    rp, col = csr_of(n, [(i, j) for i in range(n) for j in range(i + 1, n)])
    cl = list(range(n))  # center 0 and every other vertex
    dist, masks, st = oracle.cbfs(rp, col, [0, n], cl, R=1)
    full = (1 << n) - 1
    for v in range(n):
        m = [int(x) for x in masks[0, :, v, 0]]
        if v == 0:
            assert dist[0, v] == 0 and m == [0, 1, full ^ 1]
        else:  # its own bit is one nearer, every other source at the center's distance
            assert dist[0, v] == 1 and m == [1 << v, full ^ (1 << v), 0]


def test_star_closed_form():
    L = 20
    rp, col = csr_of(L + 1, [(0, i) for i in range(1, L + 1)])
    cl = list(range(L + 1))
    dist, masks, st = oracle.cbfs(rp, col, [0, L + 1], cl, R=1)
    full = (1 << (L + 1)) - 1
    for v in range(1, L + 1):
        m = [int(x) for x in masks[0, :, v, 0]]
        assert dist[0, v] == 1
        assert m == [1 << v, 1, full ^ 1 ^ (1 << v)]


def test_undamaged_grid_manhattan_radius2():
    side = 24
    n, s, d = synth.grid_edges(side, 0.0, seed=0)
    rp, col, _ = oracle.clean_csr(n, s, d)
    center = 10 * side + 7
    cl = oracle.cluster_around(rp, col, center, 64, 2)
    assert cl.size == 13  # the radius-2 ball of a 4-neighbour grid interior
    dist, masks, st = oracle.cbfs(rp, col, [0, cl.size], cl, R=2)
    assert st[0] == 0
    rr, cc = np.divmod(np.arange(n), side)
    man = lambda a: np.abs(rr - a // side) + np.abs(cc - a % side)  # noqa: E731
    assert np.array_equal(dist[0], man(center).astype(np.uint32))
    for i, src in enumerate(cl):
        o = man(int(src)) - man(center)
        bit = (masks[0, o + 2, np.arange(n), 0] >> np.uint64(i)) & np.uint64(1)
        assert np.all(bit == 1)


def test_single_source_reduces_to_bfs():
    n, s, d = synth.random_graph(70, 0.05, 4)
    rp, col, _ = oracle.clean_csr(n, s, d, flags=7)
    for src in (0, 13, 40):
        dist, masks, st = oracle.cbfs(rp, col, [0, 1], [src], R=1)
        b = oracle.bfs(rp, col, src)
        assert np.array_equal(dist[0].astype(np.int64), np.where(b < 0, 0xFFFFFFFF, b.astype(np.int64)))
        assert np.array_equal(masks[0, 1, :, 0], (b >= 0).astype(np.uint64))
        assert not masks[0, 0].any() and not masks[0, 2].any()


def test_invariants_random():
    """Fact/Corollary of Section 3.1: offsets bounded by the source's distance to the center;
    one plane per source per reached vertex; the center is always at offset 0."""
    n, s, d = synth.rmat_edges(10, 8, seed=3)
    rp, col, _ = oracle.clean_csr(n, s, d)
    centers = oracle.top_degree(rp, 6)
    cp, src = oracle.build_clusters(rp, col, centers, 64, 1)
    dist, masks, st = oracle.cbfs(rp, col, cp, src, R=1)
    assert np.all(st == 0)
    for c in range(cp.size - 1):
        cl = src[cp[c]:cp[c + 1]]
        m = masks[c, :, :, 0]
        assert not np.any(m[0] & m[1]) and not np.any(m[1] & m[2]) and not np.any(m[0] & m[2])
        full = np.uint64((1 << cl.size) - 1) if cl.size < 64 else np.uint64(2**64 - 1)
        reach = dist[c] != U32MAX
        assert np.all((m[0] | m[1] | m[2])[reach] == full)
        assert np.all((m[1][reach] & np.uint64(1)) == 1)
        dc = oracle.bfs(rp, col, int(cl[0]))
        for j, v in enumerate(cl):  # at v = s_j, bit j is at offset -delta(c, s_j)
            o = -int(dc[v])
            assert (m[o + 1, v] >> np.uint64(j)) & np.uint64(1) == 1


def test_multiword_cluster():
    n, s, d = synth.rmat_edges(11, 16, seed=5)
    rp, col, _ = oracle.clean_csr(n, s, d)
    c = int(oracle.top_degree(rp, 1)[0])
    cl = oracle.cluster_around(rp, col, c, 150, 1)
    assert cl.size == 150
    D = apsp(rp, col)
    dist, masks, st = oracle.cbfs(rp, col, [0, 150], cl, R=1)
    assert masks.shape[-1] == 3
    ed, em, ok = encode_from_apsp(D, list(cl), 1)
    assert ok and st[0] == 0
    assert np.array_equal(dist[0], ed) and np.array_equal(masks[0], em)


def test_radius_violation_and_unreachable():
    # path 0-1-2-3 plus a separate edge 4-5
    rp, col = csr_of(6, [(0, 1), (1, 2), (2, 3), (4, 5)])
    dist, masks, st = oracle.cbfs(rp, col, [0, 2, 4], [1, 3, 1, 0], R=1)
    assert st[0] == oracle.E_RADIUS       # source 3 is two hops from center 1
    assert st[1] == 0
    assert dist[1, 4] == U32MAX and dist[1, 5] == U32MAX
    assert not masks[1, :, 4:].any()
    dist, masks, st = oracle.cbfs(rp, col, [0, 2], [1, 3], R=2)
    assert st[0] == 0
    dist, masks, st = oracle.cbfs(rp, col, [0, 2], [1, 4], R=5)  # source unreachable from center
    assert st[0] == oracle.E_RADIUS


def test_violating_cluster_outputs_are_cleared():
    """A cluster whose radius does not hold returns dist = UINT32_MAX and zero
    masks at every vertex; clusters beside it in the same call are unaffected
    (each equals its own single-cluster call)."""
    rp, col = csr_of(6, [(0, 1), (1, 2), (2, 3), (4, 5)])
    cp, src = [0, 2, 4, 6], [1, 3, 1, 0, 2, 1]
    dist, masks, st = oracle.cbfs(rp, col, cp, src, R=1)
    assert list(st) == [oracle.E_RADIUS, 0, 0]
    assert (dist[0] == U32MAX).all() and not masks[0].any()
    for c in (1, 2):
        d1, m1, s1 = oracle.cbfs(rp, col, [0, 2], src[cp[c]:cp[c + 1]], R=1)
        assert s1[0] == 0 and np.array_equal(dist[c], d1[0]) and np.array_equal(masks[c], m1[0])
    assert dist[1, 1] == 0 and dist[1, 3] == 2   # the valid cluster keeps its distances


def read_fixture(golden_dir):
    fx = {"vertex": [], "query": []}
    with open(os.path.join(golden_dir, "hand_example.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            key, *rest = line.split()
            if key == "n":
                fx["n"] = int(rest[0])
            elif key == "edges":
                fx["edges"] = [tuple(int(x) for x in e.split("-")) for e in rest]
            elif key == "sources":
                fx["sources"] = [int(x) for x in rest]
            elif key == "R":
                fx["R"] = int(rest[0])
            else:
                fx[key].append([int(x) for x in rest])
    return fx


def test_radius_zero():
    """R = 0: a single-source cluster is plain BFS (scipy); a second source
    always sits at a non-zero offset somewhere (at itself), a violation."""
    n, s, d = synth.random_graph(80, 0.06, 4)
    rp, col, _ = oracle.clean_csr(n, s, d)
    nv = rp.size - 1
    A = sp.csr_matrix((np.ones(col.size), col, rp), shape=(nv, nv))
    D = shortest_path(A, unweighted=True)
    src = np.array([0, 7, nv - 1], np.int32)
    dist, masks, st = oracle.cbfs(rp, col, np.arange(4, dtype=np.int32), src, R=0)
    assert masks.shape == (3, 1, nv, 1) and (st == 0).all()
    for i, x in enumerate(src):
        assert np.array_equal(dist[i].astype(np.int64), D[x].astype(np.int64))
        assert np.all(masks[i, 0, :, 0] == 1)
    nb = int(col[rp[0]])
    _, _, st2 = oracle.cbfs(rp, col, [0, 2], [0, nb], R=0)
    assert st2[0] == oracle.E_RADIUS


def test_hand_worked_fixture(golden_dir):
    fx = read_fixture(golden_dir)
    rp, col = csr_of(fx["n"], fx["edges"])
    S = fx["sources"]
    dist, masks, st = oracle.cbfs(rp, col, [0, len(S)], S, R=fx["R"])
    assert st[0] == 0
    for v, dv, m1, m0, p1 in fx["vertex"]:
        assert dist[0, v] == dv
        assert [int(x) for x in masks[0, :, v, 0]] == [m1, m0, p1]
    qs = np.array([q[0] for q in fx["query"]], np.int32)
    qt = np.array([q[1] for q in fx["query"]], np.int32)
    want = np.array([q[2] for q in fx["query"]], np.uint32)
    truth = np.array([q[3] for q in fx["query"]])
    assert np.array_equal(oracle.query_landmarks(rp, col, [0, len(S)], S, qs, qt), want)
    assert np.array_equal(oracle.query_labels(dist, masks, qs, qt), want)
    D = apsp(rp, col)
    assert np.array_equal(D[qs, qt], truth)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_query_oracles_agree_and_bound(seed):
    n, s, d = synth.rmat_edges(10, 8, seed=seed + 20)
    rp, col, _ = oracle.clean_csr(n, s, d)
    centers = oracle.top_degree(rp, 5)
    cp, src = oracle.build_clusters(rp, col, centers, 64, 1)
    dist, masks, st = oracle.cbfs(rp, col, cp, src, R=1)
    nv = rp.size - 1
    qs, qt = synth.query_pairs(nv, 3000, seed)
    qs[:50] = src[:50]             # some endpoints are landmarks
    qt[50:60] = qs[50:60]          # s == t
    a = oracle.query_landmarks(rp, col, cp, src, qs, qt)
    b = oracle.query_labels(dist, masks, qs, qt)
    assert np.array_equal(a, b)
    D = apsp(rp, col)
    true = D[qs, qt]
    assert np.all(a.astype(np.int64) >= true)               # one-sided error
    assert np.array_equal(a[:50].astype(np.int64), true[:50])  # landmark endpoint: exact
    for j in range(50, 60):                                 # s == t: twice the nearest landmark
        assert a[j] == 2 * min(D[x, qs[j]] for x in src)


@pytest.mark.parametrize("name,g", small_graphs())
def test_pair_distances_match_library_shortest_paths(name, g):
    """Exact pair distances (the ground truth of the landmark bound) against
    scipy's all-pairs shortest paths, unreachable pairs included."""
    n, s, d = g
    rp, col, _ = oracle.clean_csr(n, s, d, flags=7)
    D = apsp(rp, col)
    nv = rp.size - 1
    qs, qt = synth.query_pairs(nv, 500, 3)
    qs[:5] = qt[:5]  # s == t
    got = oracle.pair_distances(rp, col, qs, qt, nthreads=3)
    want = D[qs, qt]
    assert np.array_equal(got[want >= 0].astype(np.int64), want[want >= 0])
    assert (got[want < 0] == U32MAX).all()
    assert (got[:5] == 0).all()


def test_pair_distances_path_closed_form():
    n = 30
    rp, col = csr_of(n, [(i, i + 1) for i in range(n - 1)])
    qs, qt = np.meshgrid(np.arange(n, dtype=np.int32), np.arange(n, dtype=np.int32))
    got = oracle.pair_distances(rp, col, qs.ravel(), qt.ravel())
    assert np.array_equal(got.astype(np.int64), np.abs(qs.ravel() - qt.ravel()).astype(np.int64))


def local_from_library(rp, col, D, s, t, tau):
    """The local search answer from scipy's BFS discovery order (FIFO, row
    order) and an all-pairs distance matrix."""
    n = rp.size - 1
    A = sp.csr_matrix((np.ones(col.size), col, rp), shape=(n, n))
    a = breadth_first_order(A, int(s), directed=True, return_predecessors=False)[:tau]
    b = set(breadth_first_order(A, int(t), directed=True, return_predecessors=False)[:tau].tolist())
    c = [int(D[s, x] + D[t, x]) for x in a if int(x) in b]
    return min(c) if c else int(U32MAX)


@pytest.mark.parametrize("name,g", small_graphs()[::3] + [small_graphs()[-1]])
def test_local_search_matches_library_bfs_order(name, g):
    n, s, d = g
    rp, col, _ = oracle.clean_csr(n, s, d, flags=7)
    D = apsp(rp, col)
    nv = rp.size - 1
    qs, qt = synth.query_pairs(nv, 60, 11)
    qs[:3] = qt[:3]
    for tau in (1, 2, 3, 7, 20, nv):
        got = oracle.local_search(rp, col, qs, qt, tau, nthreads=2)
        want = [local_from_library(rp, col, D, a, b, tau) for a, b in zip(qs, qt)]
        assert got.tolist() == want, tau
        ok = D[qs, qt] >= 0
        assert np.all(got[ok].astype(np.int64) >= D[qs, qt][ok])  # never below the true distance
        assert np.all(got[~ok] == U32MAX)


def test_local_search_row_order_matters():
    """The discovery order follows each row's stored order (not sorted ids)."""
    rp = np.array([0, 3, 4, 5, 6, 7], np.int32)   # row 0 stored as 3, 1, 2; 1, 2, 3 and 4 point to 0
    col = np.array([3, 1, 2, 0, 0, 0, 0], np.int32)
    D = apsp(rp, col)
    for t in range(5):
        for tau in (1, 2, 3, 4):
            assert oracle.local_search(rp, col, [0], [t], tau)[0] == local_from_library(rp, col, D, 0, t, tau)
    # tau = 2 from 0 finds {0, 3} (first stored neighbour), not {0, 1}
    assert oracle.local_search(rp, col, [0], [3], 2)[0] == 1
    assert oracle.local_search(rp, col, [0], [1], 2)[0] == 1  # 1 finds 0 itself


def test_local_search_path_closed_form():
    """On a path with sorted rows, a search of tau vertices from an interior
    s covers s - ceil((tau-1)/2) .. s + floor((tau-1)/2); two searches meet iff
    the intervals overlap, and then the answer is exact."""
    n = 200
    rp, col = csr_of(n, [(i, i + 1) for i in range(n - 1)])
    for tau in (1, 2, 3, 4, 9, 16):
        lo_r, hi_r = (tau - 1 + 1) // 2, (tau - 1) // 2
        for s in range(60, 80):
            for t in range(s, s + 40):
                want = t - s if s + hi_r >= t - lo_r else int(U32MAX)
                assert oracle.local_search(rp, col, [s], [t], tau)[0] == want, (tau, s, t)


def test_local_search_full_coverage_is_exact():
    """tau >= n: both searches cover their components, so the answer is the
    exact distance (none across components)."""
    n, s, d = synth.random_graph(90, 0.02, 5)
    rp, col, _ = oracle.clean_csr(n, s, d, flags=7)
    D = apsp(rp, col)
    nv = rp.size - 1
    qs, qt = synth.query_pairs(nv, 400, 2)
    got = oracle.local_search(rp, col, qs, qt, nv)
    want = D[qs, qt]
    assert np.array_equal(got[want >= 0].astype(np.int64), want[want >= 0])
    assert (got[want < 0] == U32MAX).all()
    # tau = 1: only s == t meets
    one = oracle.local_search(rp, col, qs, qt, 1)
    assert np.array_equal(one == 0, qs == qt) and np.all(one[qs != qt] == U32MAX)


def test_query_labels_radius2_matches_bruteforce():
    n, s, d = synth.grid_edges(20, 0.1, seed=9)
    rp, col, _ = oracle.clean_csr(n, s, d)
    nv = rp.size - 1
    centers = synth.random_centers(nv, 4, 9)
    cp, src = oracle.build_clusters(rp, col, centers, 64, 2)
    dist, masks, st = oracle.cbfs(rp, col, cp, src, R=2)
    assert np.all(st == 0)
    qs, qt = synth.query_pairs(nv, 2000, 9)
    assert np.array_equal(oracle.query_landmarks(rp, col, cp, src, qs, qt),
                          oracle.query_labels(dist, masks, qs, qt))


def test_certificate_accepts_oracle_and_rejects_planted_mistakes():
    n, s, d = synth.rmat_edges(10, 8, seed=8)
    rp, col, _ = oracle.clean_csr(n, s, d)
    c = int(oracle.top_degree(rp, 1)[0])
    cl = oracle.cluster_around(rp, col, c, 64, 1)
    dist, masks, st = oracle.cbfs(rp, col, [0, cl.size], cl, R=1)
    for cert in (oracle.certificate, oracle.certificate_words):
        assert cert(rp, col, cl, 1, dist[0], masks[0]) == 0
        bad = masks[0].copy()
        v = 100
        w = bad[:, v, 0].copy()            # move source 5's bit to a neighbouring plane
        p = [i for i in range(3) if (w[i] >> np.uint64(5)) & np.uint64(1)][0]
        bad[p, v, 0] ^= np.uint64(1 << 5)
        bad[(p + 1) % 3, v, 0] ^= np.uint64(1 << 5)
        assert cert(rp, col, cl, 1, dist[0], bad) > 0
        bd = dist[0].copy()
        bd[200] += 1
        assert cert(rp, col, cl, 1, bd, masks[0]) > 0
        dropped = masks[0].copy()              # a source missing at one vertex
        dropped[:, 300, 0] &= ~np.uint64(1 << 7)
        assert cert(rp, col, cl, 1, dist[0], dropped) > 0


def test_certificate_words_agrees_on_wide_disconnected_and_radius2():
    """Multi-word clusters, unreachable vertices and radius 2: the word form
    accepts the oracle's exact outputs and rejects a shifted center."""
    n, s, d = synth.random_graph(300, 0.01, 21)
    rp, col, _ = oracle.clean_csr(n, s, d, flags=7)   # no LCC: unreachable vertices
    deg = np.diff(rp)
    c = int(np.argmax(deg))
    for R, k in ((1, 150), (2, 64)):
        cl = oracle.cluster_around(rp, col, c, k, R)
        dist, masks, st = oracle.cbfs(rp, col, [0, cl.size], cl, R=R)
        assert st[0] == 0 and (dist[0] == U32MAX).any()
        assert oracle.certificate(rp, col, cl, R, dist[0], masks[0]) == 0
        assert oracle.certificate_words(rp, col, cl, R, dist[0], masks[0]) == 0
    # the center's bit moved off offset 0, with dist moved to keep delta_0(v):
    # the word form also checks that the center sits at offset 0
    cl = oracle.cluster_around(rp, col, c, 64, 1)
    dist, masks, st = oracle.cbfs(rp, col, [0, cl.size], cl, R=1)
    v = int(np.nonzero((dist[0] != U32MAX) & (dist[0] > 0))[0][0])
    bd, bm = dist[0].copy(), masks[0].copy()
    bm[1, v, 0] &= ~np.uint64(1)
    bm[0, v, 0] |= np.uint64(1)
    bd[v] += 1
    assert oracle.certificate_words(rp, col, cl, 1, bd, bm) > 0


def _plant_cases(cl, dist, masks, R):
    """Planted mistakes in words >= 1 of a multi-word cluster output, each one a
    copy of (dist, masks) with exactly one defect:
      - a bit of source 70 (word 1) moved to the neighbouring plane at a vertex;
      - the same for source 200 (word 3), when the cluster has that many sources;
      - source 130 (word 2) dropped at one vertex, and at every vertex;
      - a source >= 64 moved from its own offset to offset 0 at its own vertex
        (its distance to itself would read d(c, s) instead of 0)."""
    k = cl.size
    P = 2 * R + 1
    reach = np.nonzero((dist != U32MAX) & (dist >= 2))[0]
    v = int(reach[len(reach) // 2])
    out = []

    def moved(i, vv):
        bad = masks.copy()
        w, b = i // 64, np.uint64(1 << (i % 64))
        p = [pl for pl in range(P) if bad[pl, vv, w] & b][0]
        q = p + 1 if p + 1 < P else p - 1
        bad[p, vv, w] ^= b
        bad[q, vv, w] ^= b
        return bad

    out.append(("move70", dist, moved(70, v)))
    if k > 200:
        out.append(("move200", dist, moved(200, v)))
    drop = masks.copy()
    drop[:, v + 1 if dist[v + 1] != U32MAX else v, 130 // 64] &= ~np.uint64(1 << (130 % 64))
    out.append(("drop130", dist, drop))
    gone = masks.copy()                         # source 130 missing at every vertex
    gone[:, :, 130 // 64] &= ~np.uint64(1 << (130 % 64))
    out.append(("gone130", dist, gone))
    i = k - 1                                   # a source in the last word
    sv = int(cl[i])
    own = masks.copy()
    w, b = i // 64, np.uint64(1 << (i % 64))
    p = [pl for pl in range(P) if own[pl, sv, w] & b][0]
    assert p != R                               # d(c, s_i) >= 1
    own[p, sv, w] ^= b
    own[R, sv, w] |= b
    out.append(("own_offset0", dist, own))
    return out


@pytest.mark.parametrize("k", [150, 256])
def test_certificates_reject_mistakes_in_upper_words(k):
    """Both certificate forms accept exact multi-word outputs (W = 3 and 4) and
    reject a single planted mistake in a word >= 1 (a moved bit, a dropped
    source, a source shifted off its own vertex's level 0)."""
    n, s, d = synth.rmat_edges(11, 16, seed=7)
    rp, col, _ = oracle.clean_csr(n, s, d)
    c = int(oracle.top_degree(rp, 1)[0])
    cl = oracle.cluster_around(rp, col, c, k, 1)
    assert cl.size == k
    dist, masks, st = oracle.cbfs(rp, col, [0, k], cl, R=1)
    assert st[0] == 0 and masks.shape[-1] == (k + 63) // 64
    for cert in (oracle.certificate, oracle.certificate_words):
        assert cert(rp, col, cl, 1, dist[0], masks[0]) == 0
    for name, bd, bm in _plant_cases(cl, dist[0], masks[0], 1):
        for cert in (oracle.certificate, oracle.certificate_words):
            assert cert(rp, col, cl, 1, bd, bm) > 0, f"{cert.__name__} accepted {name} (k={k})"


def test_cleanup_c_matches_numpy_and_scipy():
    for (n, s, d) in [synth.rmat_edges(12, 8, seed=1), synth.grid_edges(40, 0.4, seed=2),
                      synth.random_graph(200, 0.01, 5)]:
        for flags in (15, 7, 11, 13, 14, 0):
            a = oracle.clean_csr(n, s, d, flags)
            b = oracle.clean_csr_numpy(n, s, d, flags)
            for x, y in zip(a, b):
                assert np.array_equal(x, y), flags
        rp, col, o2n = oracle.clean_csr(n, s, d)
        nv = rp.size - 1
        # symmetric, no self-loops, no duplicates, rows ascending
        A = sp.csr_matrix((np.ones(col.size), col, rp), shape=(nv, nv))
        assert (A != A.T).nnz == 0 and A.diagonal().sum() == 0 and A.max() == 1
        assert np.all(np.diff(col)[np.diff(np.repeat(np.arange(nv), np.diff(rp))) == 0] > 0)
        # relabel preserves order; kept ids form one component
        kept = np.nonzero(o2n >= 0)[0]
        assert np.array_equal(o2n[kept], np.arange(kept.size))
        assert sp.csgraph.connected_components(A)[0] == 1


def test_lcc_tie_takes_smallest_id():
    # two triangles of equal size: {5,6,7} and {1,2,3}; the one holding id 1 wins
    e = np.array([(5, 6), (6, 7), (7, 5), (1, 2), (2, 3), (3, 1)], np.int64)
    rp, col, o2n = oracle.clean_csr(9, e[:, 0], e[:, 1])
    assert list(np.nonzero(o2n >= 0)[0]) == [1, 2, 3]


def test_selection_rules():
    deg_rp = np.array([0, 2, 5, 7, 10, 10], np.int32)  # degrees 2,3,2,3,0
    assert list(oracle.top_degree(deg_rp, 3)) == [1, 3, 0]
    n, s, d = synth.grid_edges(10, 0.0, seed=0)
    rp, col, _ = oracle.clean_csr(n, s, d)
    cl = oracle.cluster_around(rp, col, 55, 64, 2)
    assert list(cl) == [55, 35, 44, 45, 46, 53, 54, 56, 57, 64, 65, 66, 75]
    cl = oracle.cluster_around(rp, col, 55, 5, 2)
    assert list(cl) == [55, 35, 44, 45, 46]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_landmark_selection_rule(seed):
    """Section 4.2's selection, checked from its statement on all-pairs
    distances: no vertex in two clusters; each center is the unmarked vertex
    of highest degree (lower id on ties) when it is chosen; every member lies
    within floor(d/2) hops of its center (so the cluster's diameter is at most
    d); the members are the highest-degree unmarked vertices of that ball."""
    n, s, d = synth.rmat_edges(8, 8, seed=seed + 60)
    rp, col, _ = oracle.clean_csr(n, s, d)
    D = apsp(rp, col)
    deg = np.diff(rp)
    nv = rp.size - 1
    for k, dd in ((8, 2), (5, 4), (12, 3)):
        cp, src = oracle.select_landmarks(rp, col, 1000, k, dd)
        assert np.unique(src).size == src.size
        marked = np.zeros(nv, bool)
        for c in range(cp.size - 1):
            cl = src[cp[c]:cp[c + 1]]
            center = cl[0]
            free = np.nonzero(~marked)[0]
            best = free[np.lexsort((free, -deg[free]))[0]]
            assert center == best
            ball = [v for v in free if v != center and 0 <= D[center, v] <= dd // 2]
            ball.sort(key=lambda v: (-deg[v], v))
            assert list(cl[1:]) == ball[: k - 1]
            sub = D[np.ix_(cl, cl)]
            assert sub.max() <= dd
            marked[cl] = True
        assert marked.all()  # 1000 clusters exhaust the graph


# ---------------------------------------------------------------------------
# Exact distance oracle: pruned landmark labeling in batches (phase 2)
# ---------------------------------------------------------------------------
def pll_case(name, g, with_bp):
    n, s, d = g
    rp, col, _ = oracle.clean_csr(n, s, d, flags=7)
    nv = rp.size - 1
    bp, sources = None, np.zeros(0, np.int32)
    if with_bp:
        cp, sources = oracle.select_landmarks(rp, col, 2, 8, 2)
        dist, masks, st = oracle.cbfs(rp, col, cp, sources, R=1)
        assert (st == 0).all()
        bp = (dist, masks)
    deg = np.diff(rp)
    order = np.lexsort((np.arange(nv), -deg)).astype(np.int32)
    order = order[~np.isin(order, sources)]
    return rp, col, nv, bp, sources, order


def pll_expected(D, order, sources, batches):
    """Labels from the characterisation of batched pruned BFS: root h of batch
    b labels v with d(h, v) iff no vertex of an earlier batch (phase-1 sources
    count as earliest) lies on a shortest h-v path."""
    n = D.shape[0]
    batch_of = np.full(n, np.iinfo(np.int64).max)
    batch_of[sources] = -1
    lo = 0
    for i, size in enumerate(batches):
        batch_of[order[lo:lo + size]] = i
        lo += size
    rank_of = np.full(n, -1)
    rank_of[order] = np.arange(order.size)
    labels = [set() for _ in range(n)]
    for h in order:
        b = batch_of[h]
        E = np.nonzero(batch_of < b)[0]
        dh = D[h]
        reach = dh >= 0
        pruned = np.zeros(n, bool)
        if E.size:
            dhE = D[h, E][:, None]
            dEv = D[E, :]
            ok = (dhE >= 0) & (dEv >= 0)
            pruned = ((dhE + dEv == dh[None, :]) & ok).any(axis=0)
        for v in np.nonzero(reach & ~pruned)[0]:
            labels[v].add((int(rank_of[h]), int(dh[v])))
    return labels


def pll_as_sets(cnt, lab):
    return [set((int(e) >> 32, int(e) & 0xFFFFFFFF) for e in lab[v, :cnt[v]]) for v in range(cnt.size)]


PLL_GRAPHS = [("gnp", synth.random_graph(70, 0.06, 3)), ("tree", synth.random_tree(60, 4)),
              ("grid", synth.grid_edges(8, 0.2, seed=2)), ("gnp_disconnected", synth.random_graph(80, 0.02, 9))]
PLL_SCHEDULES = [(1, 1.0, 1), (3, 1.5, 7), (200, 1.5, 1000)]


@pytest.mark.parametrize("name,g", PLL_GRAPHS)
@pytest.mark.parametrize("with_bp", [False, True])
@pytest.mark.parametrize("sched", PLL_SCHEDULES)
def test_pll_labels_match_characterisation_and_cover(name, g, with_bp, sched):
    """Pruned landmark labeling in batches against (a) the set of labels its
    pruning rule implies, evaluated by brute force on all-pairs distances (batch
    size 1 is the canonical labeling of the sequential method), and (b) the
    2-hop cover property: every query answer is the exact distance."""
    rp, col, nv, bp, sources, order = pll_case(name, g, with_bp)
    first, growth, mx = sched
    cnt, lab = oracle.pll(rp, col, order, bp=bp, first=first, growth=growth, max_batch=mx, label_cap=nv, nthreads=3)
    D = apsp(rp, col)
    want = pll_expected(D, order, sources, oracle.pll_batches(order.size, first, growth, mx))
    got = pll_as_sets(cnt, lab)
    for v in range(nv):
        assert got[v] == want[v], (v, sorted(got[v] ^ want[v])[:5])
        assert np.all(np.diff(lab[v, :cnt[v]].astype(np.uint64) >> np.uint64(32)) > 0)  # sorted by rank
    qs, qt = np.meshgrid(np.arange(nv, dtype=np.int32), np.arange(nv, dtype=np.int32))
    ans = oracle.pll_query(cnt, lab, qs.ravel(), qt.ravel(), bp=bp).astype(np.int64)
    ref = D[qs.ravel(), qt.ravel()]
    assert np.array_equal(ans[ref >= 0], ref[ref >= 0])
    assert (ans[ref < 0] == 0xFFFFFFFF).all()


def test_pll_batches_and_capacity():
    assert oracle.pll_batches(5000) == [200, 300, 450, 675, 1000, 1000, 1000, 375]
    assert oracle.pll_batches(3, 1, 1.0, 1) == [1, 1, 1]
    n, s, d = synth.random_graph(60, 0.1, 1)
    rp, col, _ = oracle.clean_csr(n, s, d, flags=7)
    order = np.arange(rp.size - 1, dtype=np.int32)
    with pytest.raises(OverflowError):
        oracle.pll(rp, col, order, label_cap=2)
    # batches change which labels exist, never the answers
    a = oracle.pll(rp, col, order, first=1, growth=1.0, max_batch=1, label_cap=64)
    b = oracle.pll(rp, col, order, label_cap=64)
    assert (a[0] <= b[0]).all() and a[0].sum() < b[0].sum()
