"""GPU parity: the HIP Cluster-BFS against the CPU oracle, bit for bit.

Each case generates a raw graph with the seeded generators, cleans it and
selects clusters on both sides independently (library entry points vs oracle
code), checks that the inputs agree, then compares every output word: dist,
all offset planes and the per-cluster status (integer work: exact equality).
Tuning knobs (direction, group width) must never change a bit.
"""
import numpy as np
import pytest

import oracle
import synth
from synth import configs

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def prepare(n, s, d, centers_fn, k, hops):
    """Both sides clean and select on their own; they must agree."""
    import paper_2410_17226_amd as P
    rp, col, o2n = P.build_csr(n, s, d)
    orp, ocol, oo2n = oracle.clean_csr(n, s, d)
    assert np.array_equal(rp, orp) and np.array_equal(col, ocol)
    centers = centers_fn(rp)
    cp, src = P.select_clusters(rp, col, centers, k, hops)
    ocp, osrc = oracle.build_clusters(orp, ocol, centers, k, hops)
    assert np.array_equal(cp, ocp) and np.array_equal(src, osrc)
    return (rp, col, cp, src), (orp, ocol, ocp, osrc)


def gpu_cbfs(rp, col, cp, src, R, tuning=None, encoding=0):
    torch = _torch()
    import paper_2410_17226_amd as P
    print(f"[gpu_cbfs] n={rp.size - 1} m={col.size} C={cp.size - 1} R={R} enc={encoding} tuning={tuning}",
          flush=True)
    rp_d = torch.from_numpy(rp).cuda()
    col_d = torch.from_numpy(col if col.size else np.zeros(1, np.int32)).cuda()
    if col.size == 0:
        col_d = col_d[:0]
    dist, masks, st = P.run_batch(rp_d, col_d, cp, src, R, tuning, encoding=encoding)
    torch.cuda.synchronize()
    return (dist.cpu().numpy().view(np.uint32), masks.cpu().numpy().view(np.uint64), st.cpu().numpy())


def assert_same(gpu, ref, where=""):
    """Every output word equal, violating clusters included (their outputs are
    defined: dist UNREACHED and zero masks at every vertex)."""
    gd, gm, gs = gpu
    od, om, os_ = ref
    assert np.array_equal(gs, os_), f"{where} status {gs} vs {os_}"
    for c in range(os_.size):
        if not np.array_equal(gd[c], od[c]):
            bad = np.nonzero(gd[c] != od[c])[0]
            raise AssertionError(f"{where} dist of cluster {c} (status {os_[c]}) differs at {bad[:5].tolist()}")
        if not np.array_equal(gm[c], om[c]):
            bad = np.argwhere(gm[c] != om[c])
            raise AssertionError(f"{where} masks of cluster {c} (status {os_[c]}) differ at {bad[:5].tolist()}")
    bad_c = np.nonzero(os_ != 0)[0]
    assert (gd[bad_c] == 0xFFFFFFFF).all() and not gm[bad_c].any(), f"{where} violating outputs not cleared"


TUNINGS = [None, dict(alpha=-1.0), dict(force_pull=1), dict(group_words=1), dict(group_words=8, alpha=5.0),
           dict(mode=1), dict(mode=1, force_pull=1, group_words=2), dict(mode=1, alpha=-1.0),
           dict(mode=2, concurrent_groups=3, group_words=1), dict(mode=2, concurrent_groups=64, group_words=1,
                                                                   alpha=-1.0),
           dict(mode=1, force_pull=1, gamma=1e-9), dict(mode=2, force_pull=1, gamma=1e-9, concurrent_groups=4),
           dict(gamma=-1.0), dict(mode=1, group_words=16), dict(mode=1, group_words=16, force_pull=1, gamma=1e-9),
           dict(mode=1, hub_arcs=1), dict(mode=1, alpha=-1.0, hub_arcs=1),
           dict(mode=1, alpha=-1.0, hub_arcs=1, group_words=16), dict(mode=1, alpha=-1.0, hub_arcs=1, group_words=1),
           dict(mode=1, hub_arcs=-1), dict(mode=2, group_words=16, concurrent_groups=4),
           dict(mode=2, group_words=16, force_pull=1, gamma=1e-9, concurrent_groups=3),
           dict(field_bits=64), dict(mode=2, field_bits=64, group_words=1, concurrent_groups=5),
           dict(field_bits=32, force_pull=1, gamma=1e-9), dict(mode=2, field_bits=8, concurrent_groups=3)]
TUNING_IDS = ["default", "push", "pull", "w1", "w8", "host", "host_pull_w2", "host_push", "slots3", "slots64",
              "host_pull_all", "pers_pull_all", "always_test", "w16", "w16_pull_all",
              "hub", "hub_push_all", "hub_push_all_w16", "hub_push_all_w1", "no_hub", "pers_w16",
              "pers_w16_pull_all", "unpacked", "pers_unpacked", "fields32_pull_all", "pers_fields8"]


def tuning_of(t, WC=1, kmax=64):
    import paper_2410_17226_amd as P
    if t is None:
        return None
    t = dict(t)
    if "group_words" in t and (t["group_words"] % WC or (WC == 3 and t["group_words"] != 3)):
        t["group_words"] = WC
    if "field_bits" in t:  # the narrowest allowed field that holds the largest cluster
        fb = t["field_bits"]
        while fb < 64 and fb < kmax:
            fb *= 2
        t["field_bits"] = fb
    return P.Tuning(**t)


def small_cases():
    cases = []
    for seed in range(3):
        cases.append(("gnp", lambda seed=seed: synth.random_graph(120, 0.05, seed), 1, 64))
        cases.append(("tree", lambda seed=seed: synth.random_tree(150, seed), 1, 64))
    cases.append(("grid_r2", lambda: synth.grid_edges(30, 0.1, seed=1), 2, 64))
    cases.append(("rmat10", lambda: synth.rmat_edges(10, 16, seed=5), 1, 64))
    cases.append(("rmat10_k150", lambda: synth.rmat_edges(10, 16, seed=6), 1, 150))
    cases.append(("rmat11_k256", lambda: synth.rmat_edges(11, 16, seed=7), 1, 256))
    cases.append(("rmat10_r3", lambda: synth.rmat_edges(10, 4, seed=8), 3, 64))
    return cases


@pytest.mark.parametrize("name,gen,R,k", small_cases(), ids=[c[0] for c in small_cases()])
@pytest.mark.parametrize("tun", TUNINGS, ids=TUNING_IDS)
def test_parity_small(name, gen, R, k, tun):
    n, s, d = gen()
    hops = R
    ncent = 9
    ours, ref_in = prepare(n, s, d, lambda rp: np.concatenate(
        [oracle.top_degree(rp, 5), synth.random_centers(rp.size - 1, 4, 3)]).astype(np.int32)
        if rp.size - 1 >= ncent else np.arange(rp.size - 1, dtype=np.int32), k, hops)
    rp, col, cp, src = ours
    WC = (int(np.diff(cp).max()) + 63) // 64
    gpu = gpu_cbfs(rp, col, cp, src, R, tuning_of(tun, WC, int(np.diff(cp).max())))
    ref = oracle.cbfs(*ref_in, R=R)
    assert_same(gpu, ref, name)


def test_parity_hand_fixture(golden_dir):
    from test_oracle import read_fixture
    fx = read_fixture(golden_dir)
    e = np.array(fx["edges"], np.int64)
    import paper_2410_17226_amd as P
    rp, col, _ = P.build_csr(fx["n"], e[:, 0], e[:, 1])
    S = np.array(fx["sources"], np.int32)
    gd, gm, gs = gpu_cbfs(rp, col, np.array([0, S.size], np.int32), S, fx["R"])
    assert gs[0] == 0
    for v, dv, m1, m0, p1 in fx["vertex"]:
        assert gd[0, v] == dv
        assert [int(x) for x in gm[0, :, v, 0]] == [m1, m0, p1]


def test_parity_disconnected_and_violations():
    # a graph kept whole (no LCC): two components plus isolated vertices
    n, s, d = synth.random_graph(200, 0.012, 11)
    import paper_2410_17226_amd as P
    rp, col, _ = P.build_csr(n, s, d, flags=7)
    orp, ocol, _ = oracle.clean_csr(n, s, d, flags=7)
    assert np.array_equal(rp, orp) and np.array_equal(col, ocol)
    deg = np.diff(rp)
    centers = np.nonzero(deg > 0)[0][:12].astype(np.int32)
    cp, src = P.select_clusters(rp, col, centers, 64, 2)   # radius-2 clusters ...
    for R in (1, 2):                                        # ... violate R = 1
        for tun in (None, dict(force_pull=1), dict(alpha=-1.0), dict(mode=1, alpha=-1.0, hub_arcs=1)):
            gpu = gpu_cbfs(rp, col, cp, src, R, tuning_of(tun))
            ref = oracle.cbfs(orp, ocol, cp, src, R=R)
            assert_same(gpu, ref, f"R={R} {tun}")
            if R == 1:
                assert (ref[2] != 0).any()
    # an isolated vertex as a single-source cluster
    iso = np.nonzero(deg == 0)[0]
    if iso.size:
        cp1 = np.array([0, 1], np.int32)
        src1 = iso[:1].astype(np.int32)
        assert_same(gpu_cbfs(rp, col, cp1, src1, 1), oracle.cbfs(orp, ocol, cp1, src1, R=1), "isolated")
        # an isolated source next to a connected one in one range-owned push
        # round (a frontier list of no arcs beside a list with arcs)
        cp2 = np.array([0, 2], np.int32)
        src2 = np.array([centers[0], iso[0]], np.int32)
        hub = P.Tuning(mode=1, alpha=-1.0, hub_arcs=1)
        assert_same(gpu_cbfs(rp, col, cp2, src2, 1, hub), oracle.cbfs(orp, ocol, cp2, src2, R=1), "isolated, hub push")


@pytest.mark.parametrize("tun", [None, dict(force_pull=1, gamma=1e-9), dict(alpha=-1.0), dict(mode=1, group_words=16),
                                 dict(mode=2, concurrent_groups=3), dict(mode=2, group_words=1, concurrent_groups=5),
                                 dict(field_bits=8)],
                         ids=["default", "pull", "push", "w16", "pers", "pers_w1", "fields8"])
def test_parity_radius_one_violation_two_hops_out(tun):
    """R = 1 with one source exactly two hops from its center: the only offsets
    outside [-1, 1] are +2 at the center and -2 at that source (the encode checks
    the center), next to valid clusters of the same centers; and a source in
    another component, which never reaches the center (found at finalize)."""
    import paper_2410_17226_amd as P
    n, s, d = synth.random_graph(160, 0.03, 23)
    rp, col, _ = P.build_csr(n, s, d, flags=7)
    nv = rp.size - 1
    deg = np.diff(rp)

    def hops_from(c):
        dist = np.full(nv, -1)
        dist[c] = 0
        frontier = [c]
        while frontier:
            nxt = []
            for u in frontier:
                for w in col[rp[u]:rp[u + 1]]:
                    if dist[w] < 0:
                        dist[w] = dist[u] + 1
                        nxt.append(w)
            frontier = nxt
        return dist

    cps, srcs = [0], []
    for c in np.argsort(-deg, kind="stable")[:6]:
        h = hops_from(c)
        nb = col[rp[c]:rp[c + 1]][:8].tolist()
        two = np.nonzero(h == 2)[0]
        far = np.nonzero(h < 0)[0]
        srcs += [int(c)] + nb                       # valid
        cps.append(len(srcs))
        if two.size:
            srcs += [int(c)] + nb + [int(two[0])]   # one source two hops out
            cps.append(len(srcs))
        if far.size:
            srcs += [int(c)] + nb[:2] + [int(far[0])]  # one source the center never reaches
            cps.append(len(srcs))
    cp = np.array(cps, np.int32)
    src = np.array(srcs, np.int32)
    gpu = gpu_cbfs(rp, col, cp, src, 1, tuning_of(tun, 1, int(np.diff(cp).max())))
    ref = oracle.cbfs(rp, col, cp, src, R=1)
    assert (ref[2] == oracle.E_RADIUS).sum() >= 6 and (ref[2] == 0).sum() == 6
    assert_same(gpu, ref, f"two hops out, {tun}")


def test_parity_radius_zero():
    """R = 0: single-source clusters (plain BFS) and a two-source cluster that
    violates the radius, in every direction mode."""
    ours, ref_in = prepare(*synth.rmat_edges(10, 16, seed=21), lambda rp: oracle.top_degree(rp, 6), 1, 1)
    rp, col, _, _ = ours
    centers = oracle.top_degree(rp, 6)
    cp = np.arange(7, dtype=np.int32)
    src = centers.astype(np.int32)
    nb = int(col[rp[centers[0]]])
    cp2 = np.concatenate([cp, [8]]).astype(np.int32)
    src2 = np.concatenate([src, [centers[1], nb if nb != centers[1] else int(col[rp[centers[1]]])]]).astype(np.int32)
    for tun in (None, dict(force_pull=1), dict(alpha=-1.0), dict(mode=2, concurrent_groups=3, group_words=1)):
        gpu = gpu_cbfs(rp, col, cp2, src2, 0, tuning_of(tun))
        ref = oracle.cbfs(rp, col, cp2, src2, R=0)
        assert ref[2][-1] == oracle.E_RADIUS and (ref[2][:-1] == 0).all()
        assert_same(gpu, ref, f"R=0 {tun}")


MIN_TUNINGS = [None, dict(alpha=-1.0), dict(force_pull=1), dict(mode=1, force_pull=1, gamma=1e-9),
               dict(mode=1, group_words=16), dict(mode=2, concurrent_groups=4, group_words=1),
               dict(mode=1, alpha=-1.0, hub_arcs=1), dict(field_bits=64)]
MIN_IDS = ["default", "push", "pull", "pull_wave", "w16", "persistent", "hub_push", "unpacked"]


def min_cases():
    out = []
    for seed in range(2):
        out.append(("gnp", lambda seed=seed: synth.random_graph(150, 0.04, seed + 40)))
        out.append(("tree", lambda seed=seed: synth.random_tree(150, seed + 40)))
    out.append(("grid", lambda: synth.grid_edges(25, 0.1, seed=4)))
    out.append(("rmat10", lambda: synth.rmat_edges(10, 16, seed=9)))
    return out


@pytest.mark.parametrize("name,gen", min_cases(), ids=[c[0] for c in min_cases()])
@pytest.mark.parametrize("tun", MIN_TUNINGS, ids=MIN_IDS)
def test_parity_min_relative(name, gen, tun):
    """The paper's own encoding <S_v[0..d], Delta_v> (Section 3.1): balls of
    radius h (diameter at most 2h) declared with d = 2h - 1 (violations),
    2h and 2h + 1, and scattered clusters (violations), bit for bit against
    the oracle, statuses and cleared outputs included."""
    import paper_2410_17226_amd as P
    n, s, d = gen()
    rp, col, _ = P.build_csr(n, s, d)
    orp, ocol, _ = oracle.clean_csr(n, s, d)
    assert np.array_equal(rp, orp) and np.array_equal(col, ocol)
    nv = rp.size - 1
    rng = np.random.default_rng(17)
    for h in (1, 2, 3):
        centers = rng.choice(nv, size=min(6, nv), replace=False).astype(np.int32)
        cp, src = P.select_clusters(rp, col, centers, 64, h)
        extra = rng.choice(nv, size=min(9, nv), replace=False).astype(np.int32)
        cp = np.concatenate([cp, [cp[-1] + extra.size]]).astype(np.int32)
        src = np.concatenate([src, extra]).astype(np.int32)
        for dd in (2 * h - 1, 2 * h, 2 * h + 1):
            gpu = gpu_cbfs(rp, col, cp, src, dd, tuning_of(tun), encoding=P.CBFS_ENCODE_MIN)
            ref = oracle.cbfs_min(orp, ocol, cp, src, dd)
            assert_same(gpu, ref, f"{name} h={h} d={dd}")


def test_parity_min_relative_wide_clusters():
    """Clusters of 150 and 256 sources (2 and 4 words) in the min-relative form."""
    import paper_2410_17226_amd as P
    n, s, d = synth.rmat_edges(11, 16, seed=13)
    rp, col, _ = P.build_csr(n, s, d)
    centers = oracle.top_degree(rp, 3)
    for k in (150, 256):
        cp, src = P.select_clusters(rp, col, centers, k, 1)
        for tun in (None, dict(force_pull=1), dict(alpha=-1.0)):
            gpu = gpu_cbfs(rp, col, cp, src, 2, tuning_of(tun, (k + 63) // 64), encoding=P.CBFS_ENCODE_MIN)
            ref = oracle.cbfs_min(rp, col, cp, src, 2)
            assert (ref[2] == 0).all()
            assert_same(gpu, ref, f"k={k} {tun}")


@pytest.mark.parametrize("tun", TUNINGS, ids=TUNING_IDS)
def test_parity_degenerate_graphs(tun):
    """A single vertex (no arcs at all: empty pull tiles), one edge, and a
    triangle with every vertex a source, in every direction mode."""
    import paper_2410_17226_amd as P
    cases = [(1, [], [0], [0, 1]), (2, [(0, 1)], [0, 1], [0, 2]), (3, [(0, 1), (1, 2), (0, 2)], [1, 0, 2], [0, 3]),
             (2, [(0, 1)], [1, 0], [0, 1, 2])]
    for n, edges, srcs, cptr in cases:
        e = np.array(edges, np.int64).reshape(-1, 2)
        rp, col, _ = P.build_csr(n, e[:, 0], e[:, 1], flags=7)
        orp, ocol, _ = oracle.clean_csr(n, e[:, 0], e[:, 1], flags=7)
        assert np.array_equal(rp, orp) and np.array_equal(col, ocol)
        cp = np.array(cptr, np.int32)
        src = np.array(srcs, np.int32)
        for R in (0, 1):
            gpu = gpu_cbfs(rp, col, cp, src, R, tuning_of(tun))
            ref = oracle.cbfs(rp, col, cp, src, R=R)
            assert_same(gpu, ref, f"n={n} edges={edges} R={R}")


def workload_inputs(name):
    cfg = configs.WORKLOADS[name]
    n, s, d = configs.raw_graph(name)

    def centers_fn(rp):
        if cfg["centers"] == "top_degree":
            return oracle.top_degree(rp, cfg["count"])
        return synth.random_centers(rp.size - 1, cfg["count"], cfg["seed"]).astype(np.int32)
    return cfg, prepare(n, s, d, centers_fn, cfg["k"], cfg["hops"])


@pytest.mark.parametrize("name", ["rmat12_small", "rmat16_batch", "grid128_small", "chunglu16_small", "rmat14"])
@pytest.mark.parametrize("mode", [1, 2])
def test_parity_workloads_small(name, mode):
    import paper_2410_17226_amd as P
    cfg, (ours, ref_in) = workload_inputs(name)
    rp, col, cp, src = ours
    gpu = gpu_cbfs(rp, col, cp, src, cfg["R"], P.Tuning(mode=mode))
    ref = oracle.cbfs(*ref_in, R=cfg["R"])
    assert_same(gpu, ref, name)
    assert (ref[2] == 0).all()
    stats = P.last_run_stats()
    assert stats["device_error"] == 0 and stats["rounds"] > 0


def test_autotuned_knobs_keep_every_bit():
    """The autotuner's choice, and every trial it timed, reproduce the oracle."""
    import paper_2410_17226_amd as P
    torch = _torch()
    cfg, (ours, ref_in) = workload_inputs("rmat16_batch")
    rp, col, cp, src = ours
    rp_d, col_d = torch.from_numpy(rp).cuda(), torch.from_numpy(col).cuda()
    best, trials = P.autotune(rp_d, col_d, cp, src, cfg["R"], sample_clusters=8)
    timed = [t for t in trials if t[1] >= 0]
    assert len(timed) >= 5
    assert min(ms for _, ms, _ in timed) == min(ms for t, ms, _ in timed if t == best)
    ref = oracle.cbfs(*ref_in, R=cfg["R"])
    assert_same(gpu_cbfs(rp, col, cp, src, cfg["R"], best), ref, f"autotuned {best}")
    for t, ms, mode in trials[:6]:
        if ms >= 0:
            assert_same(gpu_cbfs(rp, col, cp, src, cfg["R"], t), ref, f"trial {t}")



PACKED_TUNINGS = [None, dict(force_pull=1, gamma=1e-9), dict(alpha=-1.0), dict(mode=2, concurrent_groups=3),
                  dict(mode=2, group_words=1, concurrent_groups=7), dict(group_words=2, force_pull=1)]


@pytest.mark.parametrize("fb", [8, 16, 32])
@pytest.mark.parametrize("R", [1, 2])
@pytest.mark.parametrize("ti", range(len(PACKED_TUNINGS)))
def test_parity_packed_fields(fb, R, ti):
    """Clusters of at most 32 sources sharing search words (fields of 8, 16 or
    32 bits): clusters that fill their field exactly, smaller ones, a count of
    clusters that leaves the last word partly empty, a cluster whose radius is
    violated next to valid ones, and a cluster that does not reach every
    vertex; outputs word for word against the oracle."""
    torch = _torch()
    import paper_2410_17226_amd as P
    n, s, d = synth.random_graph(300, {8: 0.04, 16: 0.06, 32: 0.13}[fb], 90 + fb + R)
    rp, col, _ = P.build_csr(n, s, d, flags=7)
    nv = rp.size - 1
    rng = np.random.default_rng(fb * 10 + R)
    centers = rng.choice(nv, 13, replace=False).astype(np.int32)
    cp, src = P.select_clusters(rp, col, centers, fb, R)   # balls capped at fb sources: many fill their field
    # one more cluster of scattered sources (a radius violation among valid clusters), then a single source
    extra = rng.choice(np.setdiff1d(np.arange(nv), src), max(2, fb // 2), replace=False).astype(np.int32)
    cp = np.concatenate([cp, [cp[-1] + extra.size, cp[-1] + extra.size + 1]]).astype(np.int32)
    src = np.concatenate([src, extra, [centers[0]]]).astype(np.int32)
    assert np.diff(cp).max() <= fb and (np.diff(cp) == fb).any()
    tun = PACKED_TUNINGS[ti]
    t = P.Tuning(**{**(tun or {}), "field_bits": fb})
    gpu = gpu_cbfs(rp, col, cp, src, R, t)
    ref = oracle.cbfs(rp, col, cp, src, R=R)
    assert_same(gpu, ref, f"fields of {fb} bits, R={R}, {tun}")
