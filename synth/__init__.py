"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This module only draws random numbers and lays them out as raw inputs: edge
lists (before any cleanup), random cluster centers and query streams.  It holds
none of the Cluster-BFS arithmetic and none of the graph cleanup; each side
cleans the raw edge lists with its own code.

Every generator takes a master seed and derives an independent substream from
it, keyed by a fixed substream number, so that graph, cluster and query draws
never share random numbers.  The large raw graphs (R-MAT, Chung-Lu) come from
``synth/synth.c``: SplitMix64 used as a counter-based generator, so draw i of
a stream is a pure function of (seed, key, i).  The small draws use numpy's
PCG64 seeded with ``SeedSequence(entropy=seed, spawn_key=(key,))``.

Workloads (the paper measures on real social/web graphs, Section 5 setup; these
seeded graphs stand in for them):

* R-MAT (Chakrabarti et al.) with quadrant probabilities (a, b, c, d): each of
  ``edge_factor * 2**scale`` edges picks, at each of ``scale`` levels, one
  quadrant independently; quadrant c or d sets the row bit, b or d the column
  bit.  No permutation and no noise are applied.
* a 4-neighbour L x L grid with a fixed count of edges deleted uniformly
  without replacement (high-diameter stand-in).
* a Chung-Lu graph with expected degrees following a power law.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBC = None

# substream keys (named, fixed)
KEY_GRAPH = 1
KEY_CLUSTERS = 2
KEY_QUERIES = 3
KEY_SHUFFLE = 4


def rng_for(seed: int, key: int) -> np.random.Generator:
    """Independent PCG64 stream ``key`` of master seed ``seed``."""
    ss = np.random.SeedSequence(entropy=int(seed), spawn_key=(int(key),))
    return np.random.Generator(np.random.PCG64(ss))


def _clib():
    """The compiled raw-edge generators (``synth/synth.c``), built on first use."""
    global _LIBC
    if _LIBC is None:
        src = os.path.join(_HERE, "synth.c")
        so = os.path.join(_HERE, "libsynth.so")
        if not os.path.exists(so) or os.path.getmtime(so) < os.path.getmtime(src):
            build()
        lib = ctypes.CDLL(so)
        P, i32, i64, u64, f64 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                 ctypes.c_uint64, ctypes.c_double)
        lib.synth_stream_base.argtypes = [u64, u64]
        lib.synth_stream_base.restype = u64
        lib.synth_draw.argtypes = [u64, u64]
        lib.synth_draw.restype = u64
        lib.synth_rmat.argtypes = [i32, i64, f64, f64, f64, u64, P, P]
        lib.synth_rmat.restype = None
        lib.synth_alias_build.argtypes = [i64, P, P, P]
        lib.synth_alias_build.restype = ctypes.c_int
        lib.synth_alias_pairs.argtypes = [i64, P, P, i64, u64, P, P]
        lib.synth_alias_pairs.restype = None
        _LIBC = lib
    return _LIBC


def build(force: bool = True) -> str:
    """Compile ``synth/synth.c`` with gcc (C + pthreads)."""
    src = os.path.join(_HERE, "synth.c")
    so = os.path.join(_HERE, "libsynth.so")
    if force or not os.path.exists(so):
        tmp = so + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-pthread", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, src])
        os.replace(tmp, so)
    return so


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def stream_base(seed: int, key: int) -> int:
    """Start of SplitMix64 counter stream ``key`` of master seed ``seed``."""
    return int(_clib().synth_stream_base(int(seed) & (2**64 - 1), int(key)))


def rmat_edges(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19,
               c: float = 0.19, seed: int = 1):
    """Raw R-MAT edge list (int64 src, dst) over vertex ids [0, 2**scale).

    Edge e draws uniforms number e*scale + l (l = 0..scale-1, most significant
    bit first) from the counter-based stream (seed, KEY_GRAPH).  Self-loops and
    duplicates are kept; cleanup belongs to the consumer.
    """
    n_edges = int(edge_factor) << int(scale)
    src = np.empty(n_edges, dtype=np.int64)
    dst = np.empty(n_edges, dtype=np.int64)
    _clib().synth_rmat(int(scale), n_edges, float(a), float(b), float(c),
                       stream_base(seed, KEY_GRAPH), _ptr(src), _ptr(dst))
    return (1 << scale), src, dst


def grid_edges(side: int = 4096, delete_frac: float = 0.05, seed: int = 1):
    """4-neighbour ``side x side`` grid with ``floor(delete_frac * E)`` of its E
    undirected edges removed, chosen uniformly without replacement.

    Vertex id = row * side + col.  Edge ids: horizontal (r, c)-(r, c+1) is
    ``r*(side-1) + c``; vertical (r, c)-(r+1, c) is ``side*(side-1) + r*side + c``.
    The deleted ids are the first ``floor(delete_frac*E)`` entries of a seeded
    uniform permutation of all edge ids.
    """
    L = int(side)
    n_h = L * (L - 1)
    E = 2 * n_h
    n_del = int(np.floor(delete_frac * E))
    rng = rng_for(seed, KEY_GRAPH)
    keep = np.ones(E, dtype=bool)
    if n_del > 0:
        keep[rng.permutation(E)[:n_del]] = False
    ids = np.nonzero(keep)[0].astype(np.int64)
    horiz = ids < n_h
    hid = ids[horiz]
    r, c = hid // (L - 1), hid % (L - 1)
    hs = r * L + c
    ht = hs + 1
    vid = ids[~horiz] - n_h
    r, c = vid // L, vid % L
    vs = r * L + c
    vt = vs + L
    return L * L, np.concatenate([hs, vs]), np.concatenate([ht, vt])


def chung_lu_weights(n: int, beta: float = 2.1, avg_deg: float = 30.0) -> np.ndarray:
    """Expected degrees w_i proportional to (i+1)^(-1/(beta-1)), summing to avg_deg*n."""
    w = np.arange(1, n + 1, dtype=np.float64) ** (-1.0 / (beta - 1.0))
    w *= (avg_deg * n) / w.sum()
    return w


def chung_lu_edges(n: int, beta: float = 2.1, avg_deg: float = 30.0, seed: int = 1):
    """Raw Chung-Lu edge list: ``avg_deg*n/2`` edges whose two endpoints are drawn
    i.i.d. with probability proportional to the Chung-Lu weights (alias method,
    Walker/Vose), from the counter-based stream (seed, KEY_GRAPH)."""
    n = int(n)
    n_edges = int(round(avg_deg * n / 2.0))
    w = chung_lu_weights(n, beta, avg_deg)
    prob = np.empty(n, dtype=np.float64)
    alias = np.empty(n, dtype=np.int64)
    lib = _clib()
    if lib.synth_alias_build(n, _ptr(w), _ptr(prob), _ptr(alias)) != 0:
        raise MemoryError("alias table")
    del w
    src = np.empty(n_edges, dtype=np.int64)
    dst = np.empty(n_edges, dtype=np.int64)
    lib.synth_alias_pairs(n, _ptr(prob), _ptr(alias), n_edges, stream_base(seed, KEY_GRAPH),
                          _ptr(src), _ptr(dst))
    return n, src, dst


def random_centers(n: int, count: int, seed: int) -> np.ndarray:
    """``count`` distinct vertex ids drawn uniformly from [0, n), in draw order."""
    rng = rng_for(seed, KEY_CLUSTERS)
    return rng.choice(n, size=int(count), replace=False).astype(np.int64)


def random_graph(n: int, p: float, seed: int):
    """Erdos-Renyi G(n, p) raw edge list (each unordered pair once), for tiny tests."""
    rng = rng_for(seed, KEY_GRAPH)
    iu, ju = np.triu_indices(n, k=1)
    take = rng.random(iu.size) < p
    return n, iu[take].astype(np.int64), ju[take].astype(np.int64)


def random_tree(n: int, seed: int):
    """Uniform random recursive tree: vertex i>0 attaches to a uniform earlier vertex."""
    rng = rng_for(seed, KEY_GRAPH)
    if n <= 1:
        return n, np.zeros(0, np.int64), np.zeros(0, np.int64)
    parent = (rng.random(n - 1) * np.arange(1, n)).astype(np.int64)
    return n, np.arange(1, n, dtype=np.int64), parent


def query_pairs(n: int, count: int, seed: int):
    """``count`` (s, t) pairs, each endpoint uniform over [0, n)."""
    rng = rng_for(seed, KEY_QUERIES)
    s = rng.integers(0, n, size=int(count), dtype=np.int64)
    t = rng.integers(0, n, size=int(count), dtype=np.int64)
    return s.astype(np.int32), t.astype(np.int32)


def poisson_arrivals(rate_qps: float, count: int, seed: int) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process of rate ``rate_qps``."""
    rng = rng_for(seed, KEY_QUERIES + 100)
    gaps = rng.exponential(1.0 / float(rate_qps), size=int(count))
    return np.cumsum(gaps)
