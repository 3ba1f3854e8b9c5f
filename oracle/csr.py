"""Oracle-side graph cleanup and cluster selection (test infrastructure only).

Graph cleanup (the paper tests undirected graphs, Section 5 setup; its
applications assume them, Section 4): drop self-loops, add the reverse of every
arc, drop duplicate arcs, keep the largest connected component (ties: the
component holding the smallest original id) and relabel its vertices 0..n-1 in
ascending original-id order.  Rows of the resulting CSR are sorted ascending.

Cluster selection used by the seeded workloads: centers are either the top
vertices by degree (ties by ascending id) or given ids; a cluster is its center
followed by the lowest-id vertices at hop distance 1..h from it, in ascending
id order, up to k sources in total.  (The paper's own rule, Section 4.2,
prefers high-degree neighbours and marks chosen vertices; the seeded workloads
use this simpler rule.)
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

FLAG_SYMMETRIZE = 1
FLAG_DEDUP = 2
FLAG_DROP_SELF_LOOPS = 4
FLAG_KEEP_LCC = 8
FLAGS_ALL = 15


def clean_csr_numpy(n_in: int, src, dst, flags: int = FLAGS_ALL):
    """numpy/scipy form of the cleanup (pins the C form).  Return ``(row_ptr int32[n+1], col int32[m], old_to_new int64[n_in])``."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    n_in = int(n_in)
    if flags & FLAG_DROP_SELF_LOOPS:
        keep = src != dst
        src, dst = src[keep], dst[keep]
    if flags & FLAG_SYMMETRIZE:
        src, dst = np.concatenate([src, dst]), np.concatenate([dst, src])
    key = np.sort(src * n_in + dst)
    del src, dst
    if flags & FLAG_DEDUP and key.size:
        first_of_run = np.empty(key.size, dtype=bool)
        first_of_run[0] = True
        np.not_equal(key[1:], key[:-1], out=first_of_run[1:])
        key = key[first_of_run]
        del first_of_run
    src, dst = key // n_in, key % n_in
    del key
    if flags & FLAG_KEEP_LCC:
        indptr = np.zeros(n_in + 1, dtype=np.int64)
        np.cumsum(np.bincount(src, minlength=n_in), out=indptr[1:])
        adj = sp.csr_matrix((np.ones(src.size, dtype=np.int8), dst.astype(np.int32), indptr),
                            shape=(n_in, n_in))
        if flags & FLAG_SYMMETRIZE:
            ncomp, label = connected_components(adj, directed=False)
        else:
            ncomp, label = connected_components(adj, directed=True, connection="weak")
        del adj
        sizes = np.bincount(label, minlength=ncomp)
        # smallest original id of each component: ids ascend, so the first hit wins
        first = np.full(ncomp, n_in, dtype=np.int64)
        ids = np.arange(n_in, dtype=np.int64)
        first[label[::-1]] = ids[::-1]
        cand = np.nonzero(sizes == sizes.max())[0]
        best = cand[np.argmin(first[cand])]
        keepv = label == best
    else:
        keepv = np.ones(n_in, dtype=bool)
    old_to_new = np.full(n_in, -1, dtype=np.int64)
    old_to_new[keepv] = np.arange(int(keepv.sum()), dtype=np.int64)
    ek = keepv[src] & keepv[dst]
    s2 = old_to_new[src[ek]]
    d2 = old_to_new[dst[ek]]
    n = int(keepv.sum())
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(s2, minlength=n), out=row_ptr[1:])
    if row_ptr[-1] >= 2 ** 31:
        raise ValueError("more than 2^31-1 arcs")
    return row_ptr.astype(np.int32), d2.astype(np.int32), old_to_new


def top_degree(row_ptr, count: int) -> np.ndarray:
    """The ``count`` vertices of largest degree, ties broken by ascending id."""
    deg = np.diff(np.asarray(row_ptr, dtype=np.int64))
    order = np.lexsort((np.arange(deg.size), -deg))
    return order[:count].astype(np.int32)


def cluster_around(row_ptr, col, center: int, k: int, hops: int = 1) -> np.ndarray:
    """``center`` followed by its lowest-id vertices at distance 1..hops (<= k total)."""
    row_ptr = np.asarray(row_ptr)
    col = np.asarray(col)
    seen = {int(center)}
    layer = [int(center)]
    ball = []
    for _ in range(hops):
        nxt = []
        for u in layer:
            for v in col[row_ptr[u]:row_ptr[u + 1]]:
                v = int(v)
                if v not in seen:
                    seen.add(v)
                    nxt.append(v)
        ball.extend(nxt)
        layer = nxt
    ball.sort()
    return np.array([int(center)] + ball[: k - 1], dtype=np.int32)


def build_clusters(row_ptr, col, centers, k: int, hops: int):
    """``(cluster_ptr int32[C+1], sources int32[...])`` for the given centers."""
    parts = [cluster_around(row_ptr, col, int(c), k, hops) for c in centers]
    cluster_ptr = np.zeros(len(parts) + 1, dtype=np.int32)
    cluster_ptr[1:] = np.cumsum([p.size for p in parts])
    sources = np.concatenate(parts) if parts else np.zeros(0, np.int32)
    return cluster_ptr, sources.astype(np.int32)


def select_landmarks(row_ptr, col, num_clusters: int, k: int, diameter: int):
    """Section 4.2, "Selecting Landmarks in Clusters", written out: the unmarked
    vertex of highest degree (ties: lower id) is a center; among its unmarked
    vertices within floor(d/2) hops, the k-1 of highest degree (same ties) join
    it; every chosen vertex is marked.  Repeated num_clusters times or until
    every vertex is marked.  Each cluster: center, then members by descending
    degree.  Returns (cluster_ptr, sources)."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col)
    n = row_ptr.size - 1
    deg = np.diff(row_ptr)
    order = np.lexsort((np.arange(n), -deg))
    marked = np.zeros(n, dtype=bool)
    hops = diameter // 2
    parts = []
    for c in order:
        if len(parts) == num_clusters:
            break
        if marked[c]:
            continue
        # BFS ball of radius hops around c (through marked vertices too)
        seen = {int(c)}
        layer = [int(c)]
        ball = []
        for _ in range(hops):
            nxt = []
            for u in layer:
                for v in col[row_ptr[u]:row_ptr[u + 1]]:
                    v = int(v)
                    if v not in seen:
                        seen.add(v)
                        nxt.append(v)
            ball.extend(v for v in nxt if not marked[v])
            layer = nxt
        ball.sort(key=lambda v: (-int(deg[v]), v))
        cl = [int(c)] + ball[: k - 1]
        marked[cl] = True
        parts.append(np.array(cl, dtype=np.int32))
    cluster_ptr = np.zeros(len(parts) + 1, dtype=np.int32)
    cluster_ptr[1:] = np.cumsum([p.size for p in parts])
    sources = np.concatenate(parts) if parts else np.zeros(0, np.int32)
    return cluster_ptr, sources.astype(np.int32)
