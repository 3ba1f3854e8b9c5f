"""Cluster-BFS oracle (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It never imports the HIP library or the
product package, and the product package never imports it.

* ``cbfs``            -- one plain FIFO BFS per source, then the encode of the
                         subset equation (Section 3.1) re-based on the cluster
                         center (star-center storage, Section 5.3).  Plain C.
* ``cbfs_min``        -- the same searches encoded in the paper's own form
                         <S_v[0..d], Delta_v> (Section 3.1), for clusters of
                         diameter d.
* ``bfs``             -- single-source BFS (Appendix A, sequential form).
* ``query_landmarks`` -- brute-force landmark-labeling query (Section 4.2,
                         Algorithm "Framework of Landmark Labeling", Query).
* ``pair_distances``  -- exact delta(s, t) per pair (one BFS from s), the
                         ground truth landmark answers bound from above.
* ``local_search``    -- the query path's bidirectional local search
                         (Appendix B), tau vertices from each endpoint.
* ``pll``, ``pll_query`` -- exact 2-hop labels by pruned BFS in batches of
                         growing size (the exact distance oracle), and
                         their query.
* ``query_labels``    -- the same query from encoded labels by the lowest
                         non-empty intersection (Section 4.2).
* ``certificate``     -- BFS-distance certificate of any encoded output.
* ``clean_csr`` / ``top_degree`` / ``cluster_around`` -- the oracle side's own
  graph cleanup and cluster selection (see ``oracle/csr.py``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .csr import clean_csr_numpy, top_degree, cluster_around, build_clusters, select_landmarks  # noqa: F401
from .csr import FLAGS_ALL

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cbfs_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK = 0
E_RADIUS = -5
UNREACHABLE = np.uint32(0xFFFFFFFF)

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C + pthreads)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-pthread", "-fPIC", "-shared",
                               "-Wall", "-Wextra", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64 = ctypes.c_int32, ctypes.c_int64
        lib.oracle_bfs.argtypes = [i64, P, P, i32, P]
        lib.oracle_bfs.restype = ctypes.c_int
        lib.oracle_cbfs.argtypes = [i64, P, P, i32, P, P, i32, i32, P, P, P, i32]
        lib.oracle_cbfs.restype = ctypes.c_int
        lib.oracle_cbfs_min.argtypes = [i64, P, P, i32, P, P, i32, i32, P, P, P, i32]
        lib.oracle_cbfs_min.restype = ctypes.c_int
        lib.oracle_query_landmarks.argtypes = [i64, P, P, i32, P, P, i64, P, P, P, i32]
        lib.oracle_query_landmarks.restype = ctypes.c_int
        lib.oracle_pair_distances.argtypes = [i64, P, P, i64, P, P, P, i32]
        lib.oracle_pair_distances.restype = ctypes.c_int
        lib.oracle_local_search.argtypes = [i64, P, P, i64, P, P, i32, P, i32]
        lib.oracle_local_search.restype = ctypes.c_int
        lib.oracle_pll.argtypes = [i64, P, P, i32, i32, P, P, i64, P, i32, ctypes.c_double, i32, i32, P, P, i32]
        lib.oracle_pll.restype = ctypes.c_int
        lib.oracle_pll_query.argtypes = [i64, i32, i32, P, P, i32, P, P, i64, P, P, P]
        lib.oracle_pll_query.restype = ctypes.c_int
        lib.oracle_query_labels.argtypes = [i64, i32, i32, P, P, i64, P, P, P]
        lib.oracle_query_labels.restype = ctypes.c_int
        lib.oracle_certificate.argtypes = [i64, P, P, i32, P, i32, i32, P, P, i32]
        lib.oracle_certificate.restype = ctypes.c_int64
        lib.oracle_certificate_words.argtypes = [i64, P, P, i32, P, i32, i32, P, P, i32]
        lib.oracle_certificate_words.restype = ctypes.c_int64
        lib.oracle_clean_csr.argtypes = [i64, i64, P, P, ctypes.c_uint32, P, P, P, P, P]
        lib.oracle_clean_csr.restype = ctypes.c_int
        lib.oracle_free.argtypes = [P]
        lib.oracle_free.restype = None
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _csr(row_ptr, col):
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    return row_ptr, col, row_ptr.size - 1


def bfs(row_ptr, col, src: int) -> np.ndarray:
    """Hop distances from ``src`` (int32, -1 = unreachable)."""
    row_ptr, col, n = _csr(row_ptr, col)
    out = np.empty(n, dtype=np.int32)
    rc = _load().oracle_bfs(n, _p(row_ptr), _p(col), int(src), _p(out))
    if rc != 0:
        raise ValueError(f"oracle_bfs failed: {rc}")
    return out


def _clusters(cluster_ptr, sources):
    cluster_ptr = np.ascontiguousarray(cluster_ptr, dtype=np.int32)
    sources = np.ascontiguousarray(sources, dtype=np.int32)
    if cluster_ptr.size < 1 or cluster_ptr[0] != 0 or np.any(np.diff(cluster_ptr) < 0) \
            or cluster_ptr[-1] != sources.size:
        raise ValueError("cluster_ptr must start at 0, not decrease, and end at len(sources)")
    return cluster_ptr, sources, cluster_ptr.size - 1


def words_for(cluster_ptr) -> int:
    k = np.diff(np.asarray(cluster_ptr))
    return max(1, int((int(k.max()) + 63) // 64)) if k.size else 1


def cbfs(row_ptr, col, cluster_ptr, sources, R: int, W: int | None = None, nthreads: int = 0):
    """Center-relative cluster distance vectors for every cluster.

    Returns ``(dist[C][n] uint32, masks[C][2R+1][n][W] uint64, status[C] int32)``.
    """
    row_ptr, col, n = _csr(row_ptr, col)
    cluster_ptr, sources, C = _clusters(cluster_ptr, sources)
    if W is None:
        W = words_for(cluster_ptr)
    P = 2 * R + 1
    dist = np.empty((C, n), dtype=np.uint32)
    masks = np.empty((C, P, n, W), dtype=np.uint64)
    status = np.zeros(C, dtype=np.int32)
    rc = _load().oracle_cbfs(n, _p(row_ptr), _p(col), C, _p(cluster_ptr), _p(sources), int(R),
                             int(W), _p(dist), _p(masks), _p(status), int(nthreads))
    if rc != 0:
        raise ValueError(f"oracle_cbfs failed: {rc}")
    return dist, masks, status


def cbfs_min(row_ptr, col, cluster_ptr, sources, D: int, W: int | None = None, nthreads: int = 0):
    """The paper's cluster distance vectors <S_v[0..d], Delta_v> (Section 3.1,
    subset equation) for clusters of diameter D.

    Returns ``(delta[C][n] uint32, subsets[C][D+1][n][W] uint64, status[C] int32)``.
    """
    row_ptr, col, n = _csr(row_ptr, col)
    cluster_ptr, sources, C = _clusters(cluster_ptr, sources)
    if W is None:
        W = words_for(cluster_ptr)
    delta = np.empty((C, n), dtype=np.uint32)
    subsets = np.empty((C, D + 1, n, W), dtype=np.uint64)
    status = np.zeros(C, dtype=np.int32)
    rc = _load().oracle_cbfs_min(n, _p(row_ptr), _p(col), C, _p(cluster_ptr), _p(sources), int(D), int(W),
                                 _p(delta), _p(subsets), _p(status), int(nthreads))
    if rc != 0:
        raise ValueError(f"oracle_cbfs_min failed: {rc}")
    return delta, subsets, status


def query_landmarks(row_ptr, col, cluster_ptr, sources, qs, qt, nthreads: int = 0) -> np.ndarray:
    """Brute force: min over all landmarks x of delta(x,s) + delta(x,t)."""
    row_ptr, col, n = _csr(row_ptr, col)
    cluster_ptr, sources, C = _clusters(cluster_ptr, sources)
    qs = np.ascontiguousarray(qs, dtype=np.int32)
    qt = np.ascontiguousarray(qt, dtype=np.int32)
    ans = np.empty(qs.size, dtype=np.uint32)
    rc = _load().oracle_query_landmarks(n, _p(row_ptr), _p(col), C, _p(cluster_ptr), _p(sources),
                                        qs.size, _p(qs), _p(qt), _p(ans), int(nthreads))
    if rc != 0:
        raise ValueError(f"oracle_query_landmarks failed: {rc}")
    return ans


def pair_distances(row_ptr, col, qs, qt, nthreads: int = 0) -> np.ndarray:
    """Exact delta(s, t) per pair, one plain BFS from each s (uint32, UINT32_MAX = unreachable)."""
    row_ptr, col, n = _csr(row_ptr, col)
    qs = np.ascontiguousarray(qs, dtype=np.int32)
    qt = np.ascontiguousarray(qt, dtype=np.int32)
    out = np.empty(qs.size, dtype=np.uint32)
    rc = _load().oracle_pair_distances(n, _p(row_ptr), _p(col), qs.size, _p(qs), _p(qt), _p(out),
                                       int(nthreads))
    if rc != 0:
        raise ValueError(f"oracle_pair_distances failed: {rc}")
    return out


def local_search(row_ptr, col, qs, qt, tau: int, nthreads: int = 0) -> np.ndarray:
    """Bidirectional local search (Appendix B): min over the vertices found by
    both tau-bounded BFSs of d(s,x) + d(t,x) (uint32, UINT32_MAX if none)."""
    row_ptr, col, n = _csr(row_ptr, col)
    qs = np.ascontiguousarray(qs, dtype=np.int32)
    qt = np.ascontiguousarray(qt, dtype=np.int32)
    out = np.empty(qs.size, dtype=np.uint32)
    rc = _load().oracle_local_search(n, _p(row_ptr), _p(col), qs.size, _p(qs), _p(qt), int(tau), _p(out),
                                     int(nthreads))
    if rc != 0:
        raise ValueError(f"oracle_local_search failed: {rc}")
    return out


def _bp(bp):
    """Phase-1 labels (dist [C][n], masks [C][2R+1][n][1]) as C arrays, or none."""
    if bp is None:
        return 0, 0, np.zeros(1, np.uint32), np.zeros(1, np.uint64)
    dist, masks = bp
    dist = np.ascontiguousarray(dist, dtype=np.uint32)
    masks = np.ascontiguousarray(masks, dtype=np.uint64)
    C, Pl, n, W = masks.shape
    if W != 1:
        raise ValueError("phase-1 labels need one mask word per vertex")
    return C, (Pl - 1) // 2, dist, masks


def pll(row_ptr, col, order, bp=None, first: int = 200, growth: float = 1.5, max_batch: int = 1000,
        label_cap: int = 256, nthreads: int = 0):
    """Exact 2-hop labels by pruned BFS in batches (the exact distance oracle's
    phase 2): returns (counts int32[n], labels uint64[n][label_cap]), each
    entry (rank << 32) | distance, sorted by rank.  ``bp`` = phase-1 cluster
    labels (dist, masks) or None."""
    row_ptr, col, n = _csr(row_ptr, col)
    order = np.ascontiguousarray(order, dtype=np.int32)
    C, R, bd, bm = _bp(bp)
    cnt = np.zeros(n, dtype=np.int32)
    labels = np.zeros((n, label_cap), dtype=np.uint64)
    rc = _load().oracle_pll(n, _p(row_ptr), _p(col), C, R, _p(bd), _p(bm), order.size, _p(order), int(first),
                            float(growth), int(max_batch), int(label_cap), _p(cnt), _p(labels), int(nthreads))
    if rc == -9:
        raise OverflowError("oracle_pll: a label exceeded label_cap")
    if rc != 0:
        raise ValueError(f"oracle_pll failed: {rc}")
    return cnt, labels


def pll_query(cnt, labels, qs, qt, bp=None) -> np.ndarray:
    """Exact-oracle query: min of the phase-1 answer and the 2-hop label answer."""
    cnt = np.ascontiguousarray(cnt, dtype=np.int32)
    labels = np.ascontiguousarray(labels, dtype=np.uint64)
    n, cap = labels.shape
    C, R, bd, bm = _bp(bp)
    qs = np.ascontiguousarray(qs, dtype=np.int32)
    qt = np.ascontiguousarray(qt, dtype=np.int32)
    ans = np.empty(qs.size, dtype=np.uint32)
    rc = _load().oracle_pll_query(n, C, R, _p(bd), _p(bm), cap, _p(cnt), _p(labels), qs.size, _p(qs), _p(qt),
                                  _p(ans))
    if rc != 0:
        raise ValueError(f"oracle_pll_query failed: {rc}")
    return ans


def pll_batches(count: int, first: int = 200, growth: float = 1.5, max_batch: int = 1000):
    """The batch sizes the exact oracle's phase 2 uses for ``count`` roots."""
    out, b, lo = [], int(first), 0
    while lo < count:
        size = min(b, count - lo)
        out.append(size)
        lo += size
        b = max(1, min(int(max_batch), int(b * growth)))
    return out


def query_labels(dist, masks, qs, qt) -> np.ndarray:
    """Query from encoded labels (W = 1) by the lowest non-empty intersection."""
    dist = np.ascontiguousarray(dist, dtype=np.uint32)
    masks = np.ascontiguousarray(masks, dtype=np.uint64)
    C, P, n, W = masks.shape
    if W != 1:
        raise ValueError("query labels need one mask word per vertex")
    R = (P - 1) // 2
    qs = np.ascontiguousarray(qs, dtype=np.int32)
    qt = np.ascontiguousarray(qt, dtype=np.int32)
    ans = np.empty(qs.size, dtype=np.uint32)
    rc = _load().oracle_query_labels(n, C, R, _p(dist), _p(masks), qs.size, _p(qs), _p(qt), _p(ans))
    if rc != 0:
        raise ValueError(f"oracle_query_labels failed: {rc}")
    return ans


def certificate(row_ptr, col, sources_of_cluster, R: int, dist_c, masks_c, nthreads: int = 0) -> int:
    """Number of BFS-certificate violations of one cluster's encoded output (0 = exact)."""
    row_ptr, col, n = _csr(row_ptr, col)
    S = np.ascontiguousarray(sources_of_cluster, dtype=np.int32)
    dist_c = np.ascontiguousarray(dist_c, dtype=np.uint32)
    masks_c = np.ascontiguousarray(masks_c, dtype=np.uint64)
    P, n2, W = masks_c.shape
    assert n2 == n and P == 2 * R + 1
    r = _load().oracle_certificate(n, _p(row_ptr), _p(col), S.size, _p(S), int(R), int(W),
                                   _p(dist_c), _p(masks_c), int(nthreads))
    if r < 0:
        raise ValueError(f"oracle_certificate failed: {r}")
    return int(r)


def certificate_words(row_ptr, col, sources_of_cluster, R: int, dist_c, masks_c, nthreads: int = 0) -> int:
    """The BFS certificate evaluated a 64-bit word of sources at a time
    (``oracle_certificate_words``): same verdict, O(m * (2R+1) * W) word
    operations, no per-source decode; also checks the center's bit at offset 0."""
    row_ptr, col, n = _csr(row_ptr, col)
    S = np.ascontiguousarray(sources_of_cluster, dtype=np.int32)
    dist_c = np.ascontiguousarray(dist_c, dtype=np.uint32)
    masks_c = np.ascontiguousarray(masks_c, dtype=np.uint64)
    P, n2, W = masks_c.shape
    assert n2 == n and P == 2 * R + 1
    r = _load().oracle_certificate_words(n, _p(row_ptr), _p(col), S.size, _p(S), int(R), int(W),
                                         _p(dist_c), _p(masks_c), int(nthreads))
    if r < 0:
        raise ValueError(f"oracle_certificate_words failed: {r}")
    return int(r)


def clean_csr(n_in: int, src, dst, flags: int = FLAGS_ALL):
    """Oracle graph cleanup in plain C (see ``oracle_clean_csr``).

    Returns ``(row_ptr int32[n+1], col int32[m], old_to_new int64[n_in])``.
    """
    src = np.ascontiguousarray(src, dtype=np.int64)
    dst = np.ascontiguousarray(dst, dtype=np.int64)
    old_to_new = np.empty(int(n_in), dtype=np.int64)
    n_out, m_out = ctypes.c_int64(), ctypes.c_int64()
    rp_p, col_p = ctypes.c_void_p(), ctypes.c_void_p()
    lib = _load()
    rc = lib.oracle_clean_csr(int(n_in), src.size, _p(src), _p(dst), int(flags), _p(old_to_new),
                              ctypes.byref(n_out), ctypes.byref(m_out), ctypes.byref(rp_p),
                              ctypes.byref(col_p))
    if rc != 0:
        raise ValueError(f"oracle_clean_csr failed: {rc}")
    n, m = n_out.value, m_out.value
    row_ptr = np.ctypeslib.as_array((ctypes.c_int32 * (n + 1)).from_address(rp_p.value)).copy()
    col = (np.ctypeslib.as_array((ctypes.c_int32 * m).from_address(col_p.value)).copy()
           if m > 0 else np.zeros(0, np.int32))
    lib.oracle_free(rp_p)
    lib.oracle_free(col_p)
    return row_ptr, col, old_to_new
