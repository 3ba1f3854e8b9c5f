"""Seeded input generators: determinism and the distributions they promise."""
import numpy as np

import synth
from synth import configs


def test_rmat_deterministic_and_seeded():
    a = synth.rmat_edges(10, 4, seed=3)
    b = synth.rmat_edges(10, 4, seed=3)
    c = synth.rmat_edges(10, 4, seed=4)
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
    assert not np.array_equal(a[1], c[1])


def test_rmat_quadrant_frequencies():
    a, b, c = 0.57, 0.19, 0.19
    n, s, t = synth.rmat_edges(12, 32, a, b, c, seed=1)
    assert n == 4096 and s.size == 32 * 4096
    assert s.min() >= 0 and s.max() < n and t.max() < n
    for lvl in range(12):
        rb = (s >> (11 - lvl)) & 1
        cb = (t >> (11 - lvl)) & 1
        q = np.bincount(rb * 2 + cb, minlength=4) / s.size  # (0,0)=a (0,1)=b (1,0)=c (1,1)=d
        assert np.allclose(q, [a, b, c, 1 - a - b - c], atol=0.006)


def test_counter_stream_is_pure_function_of_index():
    base = synth.stream_base(99, synth.KEY_GRAPH)
    lib = synth._clib()
    assert lib.synth_draw(base, 7) == lib.synth_draw(base, 7)
    assert synth.stream_base(99, 1) != synth.stream_base(99, 2)


def test_grid_deletes_exact_count():
    side, frac = 64, 0.05
    n, s, t = synth.grid_edges(side, frac, seed=5)
    E = 2 * side * (side - 1)
    assert n == side * side
    assert s.size == E - int(np.floor(frac * E))
    d = np.abs(t - s)
    assert np.all((d == 1) | (d == side))
    assert np.all((s % side != side - 1) | (d == side))
    n2, s2, t2 = synth.grid_edges(side, frac, seed=5)
    assert np.array_equal(s, s2) and np.array_equal(t, t2)


def test_chung_lu_expected_degrees():
    n, beta, avg = 1 << 14, 2.1, 30.0
    n_, s, t = synth.chung_lu_edges(n, beta, avg, seed=2)
    w = synth.chung_lu_weights(n, beta, avg)
    assert abs(w.sum() - avg * n) < 1e-6 * avg * n
    deg = np.bincount(np.concatenate([s, t]), minlength=n)
    assert deg.sum() == 2 * s.size == round(avg * n)
    # top vertices: realised degree within 5 sigma of the weight
    top = np.arange(20)
    assert np.all(np.abs(deg[top] - w[top]) < 5 * np.sqrt(w[top]) + 1)
    # aggregate over deciles
    for lo in range(0, n, n // 8):
        hi = lo + n // 8
        assert abs(deg[lo:hi].sum() - w[lo:hi].sum()) < 5 * np.sqrt(w[lo:hi].sum()) + 5


def test_random_centers_and_queries():
    c = synth.random_centers(1000, 50, 3)
    assert np.unique(c).size == 50 and c.max() < 1000
    assert np.array_equal(c, synth.random_centers(1000, 50, 3))
    s, t = synth.query_pairs(500, 10000, 1)
    assert s.min() >= 0 and s.max() < 500 and abs(s.mean() - 249.5) < 10
    arr = synth.poisson_arrivals(1e6, 100000, 1)
    assert np.all(np.diff(arr) > 0)
    assert abs(arr[-1] / arr.size - 1e-6) < 2e-8


def test_workload_table_well_formed():
    for name, cfg in configs.WORKLOADS.items():
        assert cfg["graph"] in ("rmat", "grid", "chung_lu")
        assert cfg["centers"] in ("top_degree", "random")
        assert 1 <= cfg["k"] <= 256 and cfg["R"] >= 1 and cfg["hops"] >= 1
