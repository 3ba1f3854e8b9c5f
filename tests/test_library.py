"""The C-ABI library on the CPU: it loads, exports every entry point its header
declares, and its host-side entry points (graph ingest, cluster selection,
argument checks) agree with the oracle side.  No kernel is launched here."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_2410_17226_amd as P
from paper_2410_17226_amd import _binding as B
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "cbfs.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cbfs_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = P.load()
    declared = header_functions()
    assert len(declared) >= 9
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(P.exported_symbols()) == sorted(B.SYMBOLS)
    assert sorted(B.SYMBOLS) == declared


def test_gather_probe_is_a_separate_library():
    # the measurement probe of bench.py is built beside libcbfs, not into it
    probe = ctypes.CDLL(os.path.join(ROOT, "paper_2410_17226_amd", "libcbfs_probe.so"))
    assert hasattr(probe, "cbfs_probe_gather")
    assert "cbfs_probe_gather" not in P.exported_symbols()


def test_status_strings():
    assert P.status_string(0) == "CBFS_OK"
    assert P.status_string(-5) == "CBFS_E_RADIUS"


@pytest.mark.parametrize("gen", [lambda: synth.rmat_edges(13, 16, seed=3),
                                 lambda: synth.grid_edges(60, 0.3, seed=4),
                                 lambda: synth.chung_lu_edges(1 << 12, 2.1, 30.0, seed=5),
                                 lambda: synth.random_graph(300, 0.004, 6)])
@pytest.mark.parametrize("flags", [15, 7, 11, 13, 14, 3, 0])
def test_build_csr_matches_oracle_cleanup(gen, flags):
    n, s, d = gen()
    a = P.build_csr(n, s, d, flags)
    b = oracle.clean_csr(n, s, d, flags)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_build_csr_errors():
    with pytest.raises(P.CbfsError) as e:
        P.build_csr(10, [0, 11], [1, 2])
    assert e.value.status == -2
    with pytest.raises(P.CbfsError) as e:
        P.build_csr(0, [], [])
    assert e.value.status == -1


def test_selection_matches_oracle():
    n, s, d = synth.rmat_edges(12, 16, seed=9)
    rp, col, _ = P.build_csr(n, s, d)
    for count in (1, 7, 50):
        assert np.array_equal(P.top_degree(rp, count), oracle.top_degree(rp, count))
    centers = P.top_degree(rp, 20)
    for k, hops in ((64, 1), (256, 1), (10, 2), (64, 2)):
        a = P.select_clusters(rp, col, centers, k, hops)
        b = oracle.build_clusters(rp, col, centers, k, hops)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    n, s, d = synth.grid_edges(50, 0.05, seed=2)
    rp, col, _ = P.build_csr(n, s, d)
    centers = synth.random_centers(rp.size - 1, 10, 2)
    a = P.select_clusters(rp, col, centers, 64, 2)
    b = oracle.build_clusters(rp, col, centers, 64, 2)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_landmark_selection_matches_oracle():
    """The library's Section 4.2 selection (degree priority, floor(d/2) hops,
    marking) equals the oracle side's own implementation."""
    for seed in range(3):
        n, s, d = synth.rmat_edges(11, 16, seed=seed)
        rp, col, _ = P.build_csr(n, s, d)
        for C, k, dd in ((20, 64, 2), (50, 16, 4), (3000, 8, 3), (30, 256, 2), (10, 1, 6)):
            a = P.select_landmarks(rp, col, C, k, dd)
            b = oracle.select_landmarks(rp, col, C, k, dd)
            assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), (seed, C, k, dd)


def test_select_clusters_errors():
    rp = np.array([0, 1, 2], np.int32)
    col = np.array([1, 0], np.int32)
    with pytest.raises(P.CbfsError) as e:
        P.select_clusters(rp, col, [5], 4, 1)
    assert e.value.status == -2
    with pytest.raises(P.CbfsError) as e:
        P.select_clusters(rp, col, [0], 300, 1)
    assert e.value.status == -4


class _FakeDev:
    """Stands in for a device tensor in argument-error calls that never launch."""

    def __init__(self, numel):
        self._n = numel

    def numel(self):
        return self._n

    def data_ptr(self):
        return 0x1000


def _call_run_batch(n, m, cluster_ptr, sources, R, ws_bytes=1 << 40, tuning=None):
    g, b, t, cp, src = B._batch_structs(_FakeDev(n + 1), _FakeDev(m), cluster_ptr, sources, R, tuning)
    lib = P.load()
    return lib.cbfs_run_batch(ctypes.byref(g), ctypes.byref(b), ctypes.byref(t) if t is not None else None,
                              ctypes.c_void_p(0x2000), ctypes.c_void_p(0x3000), ctypes.c_void_p(0x4000),
                              ctypes.c_void_p(0x5000), ws_bytes, None)


def test_run_batch_argument_errors_before_launch():
    # duplicate source in one cluster
    assert _call_run_batch(100, 400, [0, 3], [5, 6, 5], 1) == -3
    # source out of range
    assert _call_run_batch(100, 400, [0, 2], [5, 100], 1) == -2
    # too many / zero sources
    assert _call_run_batch(1000, 4000, [0, 257], list(range(257)), 1) == -4
    assert _call_run_batch(100, 400, [0, 0], [], 1) == -4
    # negative radius, bad cluster_ptr
    assert _call_run_batch(100, 400, [0, 2], [1, 2], -1) == -1
    assert _call_run_batch(100, 400, [1, 2], [1, 2], 1) == -1
    # workspace too small
    assert _call_run_batch(100, 400, [0, 2], [1, 2], 1, ws_bytes=16) == -6
    # bad tuning
    assert _call_run_batch(100, 400, [0, 2], [1, 2], 1, tuning=P.Tuning(group_words=3)) == -1
    assert _call_run_batch(100, 400, [0, 2], [1, 2], 1, tuning=P.Tuning(block_size=128)) == -1
    assert _call_run_batch(100, 400, [0, 2], [1, 2], 1, tuning=P.Tuning(concurrent_groups=65)) == -1
    assert _call_run_batch(100, 400, [0, 2], [1, 2], 1, tuning=P.Tuning(mode=3)) == -1


def test_workspace_size_monotone():
    def size(n, m, k, C, tuning=None):
        cp = np.arange(C + 1, dtype=np.int32) * k
        src = np.tile(np.arange(k, dtype=np.int32), C)
        g, b, t, _a, _b = B._batch_structs(_FakeDev(n + 1), _FakeDev(m), cp, src, 1, tuning)
        return P.load().cbfs_run_batch_workspace_size(ctypes.byref(g), ctypes.byref(b),
                                                      ctypes.byref(t) if t is not None else None)
    s1 = size(1000, 5000, 64, 4)
    assert s1 > 3 * 1000 * 8
    assert size(2000, 5000, 64, 4) > s1
    one = dict(concurrent_groups=1)
    assert size(1000, 5000, 64, 4, P.Tuning(group_words=8, **one)) >= size(1000, 5000, 64, 4,
                                                                           P.Tuning(group_words=1, **one))
    # side-by-side group slots each carry their own search state
    assert size(1000, 5000, 64, 4, P.Tuning(group_words=1, concurrent_groups=4)) > \
        size(1000, 5000, 64, 4, P.Tuning(group_words=1, **one))
    assert size(1000, 5000, 300, 1) == 0  # invalid: more than 256 sources


def test_autotune_argument_errors_before_launch():
    """Null outputs or a bad sample size are rejected on the host (no kernel runs)."""
    lib = P.load()
    rp = np.array([0, 1, 2], np.int32)
    col = np.array([1, 0], np.int32)
    g = B._Csr(2, 2, rp.ctypes.data, col.ctypes.data)   # host pointers: never dereferenced here
    cp = np.array([0, 1], np.int32)
    src = np.array([0], np.int32)
    b = B._Batch(1, cp.ctypes.data, src.ctypes.data, 1)
    best = B._Tuning()
    rc = lib.cbfs_autotune(ctypes.byref(g), ctypes.byref(b), None, 0, None, None, None, None, 0, None,
                           ctypes.byref(best), None, 0, None)
    assert rc == -1
    buf = ctypes.c_void_p(1)
    rc = lib.cbfs_autotune(ctypes.byref(g), ctypes.byref(b), None, -1, buf, buf, buf, buf, 0, None,
                           ctypes.byref(best), None, 0, None)
    assert rc == -1
    bad = np.array([0, 0], np.int32)     # empty cluster
    b2 = B._Batch(1, bad.ctypes.data, src.ctypes.data, 1)
    rc = lib.cbfs_autotune(ctypes.byref(g), ctypes.byref(b2), None, 0, buf, buf, buf, buf, 0, None,
                           ctypes.byref(best), None, 0, None)
    assert rc == -4  # CBFS_E_TOO_MANY_SOURCES
    assert lib.cbfs_autotune_workspace_size(ctypes.byref(g), ctypes.byref(b), 0) > 0



_C_TYPES = {"int32_t": ctypes.c_int32, "int64_t": ctypes.c_int64, "float": ctypes.c_float,
            "size_t": ctypes.c_size_t}


def header_structs():
    """Field names and C types of every typedef'd struct in the header."""
    text = open(os.path.join(ROOT, "include", "cbfs.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    out = {}
    for body, name in re.findall(r"typedef struct\s*\{(.*?)\}\s*(cbfs_[a-z_]+)\s*;", text, flags=re.S):
        fields = []
        for decl in body.split(";"):
            decl = " ".join(decl.split())
            if not decl:
                continue
            m = re.match(r"(?:const )?([a-z_0-9]+)\s*(\*?)\s*(.*)", decl)
            ctype, ptr, names = m.groups()
            for fname in names.split(","):
                fname = fname.strip()
                star = ptr or fname.startswith("*")
                fields.append((fname.lstrip("*").strip(), "ptr" if star else ctype))
        out[name] = fields
    return out


@pytest.mark.parametrize("cname,pyname", [("cbfs_csr", "_Csr"), ("cbfs_batch", "_Batch"),
                                          ("cbfs_tuning", "_Tuning"), ("cbfs_trial", "_Trial"),
                                          ("cbfs_run_stats", "_RunStats"), ("cbfs_labels", "_Labels")])
def test_binding_structs_mirror_the_header(cname, pyname):
    """Every ctypes mirror has the header's fields, in order, with the same C types."""
    want = header_structs()[cname]
    got = getattr(B, pyname)._fields_
    assert [n for n, _ in got] == [n for n, _ in want], cname
    for (n, t), (_, c) in zip(got, want):
        if c == "ptr":
            assert t is ctypes.c_void_p, (cname, n)
        elif c in _C_TYPES:
            assert t is _C_TYPES[c], (cname, n, c)
        else:  # a nested struct of the header
            assert t.__name__ == {"cbfs_tuning": "_Tuning"}.get(c, c), (cname, n, c)
