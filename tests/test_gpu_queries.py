"""GPU parity of the landmark-labeling queries (Section 4.2, "Answering Queries
with Clustered Landmarks"; Algorithm "Framework of Landmark Labeling", Query)
at every radius: labels built by the HIP path (cbfs_run_batch, then
cbfs_labels_pack), queries answered by cbfs_query_batch, compared element by
element with the oracle's brute force over all landmarks.

The graphs are G(n, p) graphs, which have odd cycles, so offsets of both
parities occur (on a bipartite graph all offsets of a radius-2 cluster are
even, and pairs such as (-2, +1) never show up)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("R", [0, 1, 2, 3])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_query_batch_any_radius_matches_landmark_oracle(R, seed):
    torch = _torch()
    import paper_2410_17226_amd as P
    n, s, d = synth.random_graph(400, 0.015, 40 + seed)
    rp, col, _ = P.build_csr(n, s, d)
    orp, ocol, _ = oracle.clean_csr(n, s, d)
    assert np.array_equal(rp, orp) and np.array_equal(col, ocol)
    nv = rp.size - 1
    centers = synth.random_centers(nv, 12, seed).astype(np.int32)
    cp, src = P.select_clusters(rp, col, centers, 64, R)
    ocp, osrc = oracle.build_clusters(rp, col, centers, 64, R)
    assert np.array_equal(cp, ocp) and np.array_equal(src, osrc)
    print(f"[queries] R={R} seed={seed} n={nv} m={col.size} clusters={cp.size - 1}", flush=True)
    rp_d, col_d = torch.from_numpy(rp).cuda(), torch.from_numpy(col).cuda()
    dist, masks, st = P.run_batch(rp_d, col_d, cp, src, R)
    assert (st.cpu().numpy() == 0).all()
    dvm, mvm = P.labels_pack(dist, masks, R)
    assert tuple(mvm.shape) == (nv, cp.size - 1, 2 * R)
    qs, qt = synth.query_pairs(nv, 5000, 100 + seed)
    qs[:40] = src[:40] if src.size >= 40 else qs[:40]   # landmark endpoints
    qt[40:60] = qs[40:60]                               # s == t
    got = P.query_batch(dvm, mvm, R, torch.from_numpy(qs).cuda(), torch.from_numpy(qt).cuda())
    torch.cuda.synchronize()
    got = got.cpu().numpy().view(np.uint32)
    want = oracle.query_landmarks(orp, ocol, ocp, osrc, qs, qt)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, f"{bad.size} answers differ, e.g. pair {bad[0]}: {got[bad[0]]} vs {want[bad[0]]}"
    # the labels' own query evaluated by the oracle from the oracle's encode agrees too
    od, om, ost = oracle.cbfs(orp, ocol, ocp, osrc, R=R)
    assert np.array_equal(oracle.query_labels(od, om, qs, qt), want)


@pytest.mark.parametrize("dd", [2, 4])
def test_landmark_labeling_as_the_paper_builds_it(dd):
    """Section 4.2's index: clusters selected by degree with marking within
    floor(d/2) hops (library and oracle selections agree), C-BFS labels with
    R = floor(d/2) built by the HIP path, queries equal to the brute force
    over the same landmarks, never below the exact distance, and exact when
    an endpoint is a landmark."""
    torch = _torch()
    import paper_2410_17226_amd as P
    n, s, d = synth.rmat_edges(12, 16, seed=70 + dd)
    rp, col, _ = P.build_csr(n, s, d)
    orp, ocol, _ = oracle.clean_csr(n, s, d)
    assert np.array_equal(rp, orp) and np.array_equal(col, ocol)
    cp, src = P.select_landmarks(rp, col, 24, 64, dd)
    ocp, osrc = oracle.select_landmarks(orp, ocol, 24, 64, dd)
    assert np.array_equal(cp, ocp) and np.array_equal(src, osrc)
    R = dd // 2
    nv = rp.size - 1
    print(f"[ll] d={dd} n={nv} clusters={cp.size - 1} landmarks={src.size}", flush=True)
    rp_d, col_d = torch.from_numpy(rp).cuda(), torch.from_numpy(col).cuda()
    dist, masks, st = P.run_batch(rp_d, col_d, cp, src, R)
    assert (st.cpu().numpy() == 0).all()
    dvm, mvm = P.labels_pack(dist, masks, R)
    qs, qt = synth.query_pairs(nv, 3000, 7 + dd)
    qs[:30] = src[:30]
    got = P.query_batch(dvm, mvm, R, torch.from_numpy(qs).cuda(), torch.from_numpy(qt).cuda())
    got = got.cpu().numpy().view(np.uint32)
    want = oracle.query_landmarks(orp, ocol, ocp, osrc, qs, qt)
    assert np.array_equal(got, want)
    exact = oracle.pair_distances(orp, ocol, qs, qt)
    assert (got.astype(np.int64) >= exact.astype(np.int64)).all()
    assert np.array_equal(got[:30], exact[:30])


@pytest.mark.parametrize("dd", [2, 3, 4, 5, 6])
def test_min_relative_on_landmark_clusters_of_each_diameter(dd):
    """Clusters of diameter d = 2..6 from the paper's selection, encoded in
    the paper's own form <S_v[0..d], Delta_v>, bit for bit against the oracle."""
    torch = _torch()
    import paper_2410_17226_amd as P
    n, s, d = synth.rmat_edges(12, 16, seed=80)
    rp, col, _ = P.build_csr(n, s, d)
    cp, src = P.select_landmarks(rp, col, 12, 64, dd)
    rp_d, col_d = torch.from_numpy(rp).cuda(), torch.from_numpy(col).cuda()
    print(f"[minrel] d={dd} clusters={cp.size - 1}", flush=True)
    for tun in (None, P.Tuning(force_pull=1), P.Tuning(alpha=-1.0)):
        dist, masks, st = P.run_batch(rp_d, col_d, cp, src, dd, tun, encoding=P.CBFS_ENCODE_MIN)
        od, om, ost = oracle.cbfs_min(rp, col, cp, src, dd)
        assert (ost == 0).all()
        assert np.array_equal(st.cpu().numpy(), ost)
        assert np.array_equal(dist.cpu().numpy().view(np.uint32), od)
        assert np.array_equal(masks.cpu().numpy().view(np.uint64), om)


def _local_graphs():
    """(name, row_ptr, col): R-MAT with hubs (rows longer than a wave), a
    sparse G(n, p) with isolated vertices and small components, a long path
    (deep searches), and an R-MAT whose rows are stored in shuffled order."""
    out = []
    n, s, d = synth.rmat_edges(13, 16, seed=5)
    rp, col, _ = oracle.clean_csr(n, s, d)
    out.append(("rmat13", rp, col))
    n, s, d = synth.random_graph(3000, 0.0006, 6)
    rp, col, _ = oracle.clean_csr(n, s, d, flags=7)
    out.append(("gnp_sparse", rp, col))
    n = 5000
    e = np.array([(i, i + 1) for i in range(n - 1)], np.int64)
    rp, col, _ = oracle.clean_csr(n, e[:, 0], e[:, 1], flags=7)
    out.append(("path", rp, col))
    n, s, d = synth.rmat_edges(12, 8, seed=7)
    rp, col, _ = oracle.clean_csr(n, s, d)
    col = col.copy()
    rng = np.random.default_rng(7)
    for v in range(rp.size - 1):
        rng.shuffle(col[rp[v]:rp[v + 1]])
    out.append(("rmat12_shuffled_rows", rp, col))
    return out


@pytest.mark.parametrize("tau", [1, 2, 63, 64, 65, 200, 512, 2048])
def test_local_search_matches_oracle(tau):
    """Bidirectional local search (Appendix B) bit-exact against the oracle:
    the local answer alone (ans pre-filled with none), on every graph."""
    torch = _torch()
    import paper_2410_17226_amd as P
    for name, rp, col in _local_graphs():
        nv = rp.size - 1
        qs, qt = synth.query_pairs(nv, 1500, tau)
        qs[:20] = qt[:20]                                   # s == t
        deg = np.diff(rp)
        hubs = np.argsort(-deg, kind="stable")[:20].astype(np.int32)
        qs[20:40] = hubs                                    # hub endpoints
        if (deg == 0).any():
            qt[40:50] = np.nonzero(deg == 0)[0][:1]          # an isolated endpoint
        print(f"[local] tau={tau} graph={name} n={nv} m={col.size} q={qs.size}", flush=True)
        rp_d, col_d = torch.from_numpy(rp).cuda(), torch.from_numpy(col).cuda()
        got = P.query_local(rp_d, col_d, torch.from_numpy(qs).cuda(), torch.from_numpy(qt).cuda(), tau)
        torch.cuda.synchronize()
        got = got.cpu().numpy().view(np.uint32)
        want = oracle.local_search(rp, col, qs, qt, tau)
        bad = np.nonzero(got != want)[0]
        assert bad.size == 0, (f"{name} tau={tau}: {bad.size} answers differ, e.g. pair {bad[0]} "
                               f"({qs[bad[0]]}, {qt[bad[0]]}): {got[bad[0]]} vs {want[bad[0]]}")


def test_local_search_combined_with_landmarks():
    """ans = min(landmark answer, local answer): cbfs_query_batch, then
    cbfs_query_local on the same output; never below the true distance."""
    torch = _torch()
    import paper_2410_17226_amd as P
    n, s, d = synth.rmat_edges(12, 16, seed=9)
    rp, col, _ = P.build_csr(n, s, d)
    nv = rp.size - 1
    cp, src = P.select_landmarks(rp, col, 16, 64, 2)
    rp_d, col_d = torch.from_numpy(rp).cuda(), torch.from_numpy(col).cuda()
    dist, masks, st = P.run_batch(rp_d, col_d, cp, src, 1)
    assert (st.cpu().numpy() == 0).all()
    dvm, mvm = P.labels_pack(dist, masks, 1)
    qs, qt = synth.query_pairs(nv, 4000, 9)
    s_d, t_d = torch.from_numpy(qs).cuda(), torch.from_numpy(qt).cuda()
    for tau in (64, 512):
        ans = P.query_batch(dvm, mvm, 1, s_d, t_d)
        landmark = ans.cpu().numpy().view(np.uint32).copy()
        P.query_local(rp_d, col_d, s_d, t_d, tau, out=ans)
        torch.cuda.synchronize()
        got = ans.cpu().numpy().view(np.uint32)
        local = oracle.local_search(rp, col, qs, qt, tau)
        want = np.minimum(oracle.query_landmarks(rp, col, cp, src, qs, qt), local)
        assert np.array_equal(landmark, oracle.query_landmarks(rp, col, cp, src, qs, qt))
        assert np.array_equal(got, want)
        true = oracle.pair_distances(rp, col, qs, qt)
        ok = true != 0xFFFFFFFF
        assert np.all(got[ok] >= true[ok])
        assert np.sum(got != landmark) > 0  # the local search improved some answers


def test_local_search_rejects_bad_tau():
    torch = _torch()
    import paper_2410_17226_amd as P
    rp = torch.tensor([0, 1, 2], dtype=torch.int32, device="cuda")
    col = torch.tensor([1, 0], dtype=torch.int32, device="cuda")
    s = torch.zeros(4, dtype=torch.int32, device="cuda")
    for tau in (0, P.LOCAL_TAU_MAX + 1):
        with pytest.raises(P.CbfsError):
            P.query_local(rp, col, s, s, tau)
    assert P.query_local(rp, col, s[:0], s[:0], 8).numel() == 0


@pytest.mark.parametrize("w", [8, 16, 32, 64])
def test_compact_labels_under_a_budget(w):
    """Compact labels (one-byte distance, w-bit subsets; Section 5.3's storage
    under a memory budget): the packed bytes equal the oracle's outputs packed
    the same way, and queries over them equal the brute force over the
    landmarks."""
    torch = _torch()
    import paper_2410_17226_amd as P
    n, s, d = synth.random_graph(500, 0.012, 60 + w)
    rp, col, _ = P.build_csr(n, s, d)
    nv = rp.size - 1
    cp, src = P.select_landmarks(rp, col, 12, w, 2)
    assert np.diff(cp).max() <= w
    rp_d, col_d = torch.from_numpy(rp).cuda(), torch.from_numpy(col).cuda()
    dist, masks, st = P.run_batch(rp_d, col_d, cp, src, 1)
    assert (st.cpu().numpy() == 0).all()
    d8, mc = P.labels_pack_compact(dist, masks, 1, w)
    od, om, _ = oracle.cbfs(rp, col, cp, src, R=1)
    C = cp.size - 1
    want_d8 = np.where(od == 0xFFFFFFFF, 255, od).astype(np.uint8).T                  # [n][C]
    want_m = np.transpose(om[:, :2, :, 0], (2, 0, 1)).astype(np.uint64)              # [n][C][2]: planes -1, 0
    assert np.array_equal(d8.cpu().numpy(), want_d8)
    got_m = mc.cpu().numpy().view({8: np.uint8, 16: np.uint16, 32: np.uint32, 64: np.uint64}[w]).astype(np.uint64)
    assert np.array_equal(got_m, want_m)
    assert d8.numel() + mc.numel() * mc.element_size() == nv * C * (1 + 2 * w // 8)  # bytes per vertex as budgeted
    qs, qt = synth.query_pairs(nv, 5000, 70 + w)
    qs[:30] = src[:30]
    ans = P.query_batch_compact(d8, mc, 1, w, torch.from_numpy(qs).cuda(), torch.from_numpy(qt).cuda())
    torch.cuda.synchronize()
    assert np.array_equal(ans.cpu().numpy().view(np.uint32), oracle.query_landmarks(rp, col, cp, src, qs, qt))


def test_compact_labels_plain_landmarks_and_errors():
    """Single-vertex landmarks (R = 0, a distance byte only) and the range
    errors: a cluster wider than w, and a distance of 255 or more."""
    torch = _torch()
    import paper_2410_17226_amd as P
    n, s, d = synth.random_graph(500, 0.012, 81)
    rp, col, _ = P.build_csr(n, s, d)
    nv = rp.size - 1
    lm = P.top_degree(rp, 40).astype(np.int32)
    cp = np.arange(lm.size + 1, dtype=np.int32)
    rp_d, col_d = torch.from_numpy(rp).cuda(), torch.from_numpy(col).cuda()
    dist, masks, st = P.run_batch(rp_d, col_d, cp, lm, 0)
    d8, mc = P.labels_pack_compact(dist, masks, 0, 8)
    qs, qt = synth.query_pairs(nv, 3000, 82)
    ans = P.query_batch_compact(d8, mc, 0, 8, torch.from_numpy(qs).cuda(), torch.from_numpy(qt).cuda())
    torch.cuda.synchronize()
    assert np.array_equal(ans.cpu().numpy().view(np.uint32), oracle.query_landmarks(rp, col, cp, lm, qs, qt))
    # a cluster of 20 sources does not fit 8-bit subsets
    cp2, src2 = P.select_landmarks(rp, col, 3, 20, 2)
    assert np.diff(cp2).max() > 8
    dist2, masks2, _ = P.run_batch(rp_d, col_d, cp2, src2, 1)
    with pytest.raises(P.CbfsError) as ei:
        P.labels_pack_compact(dist2, masks2, 1, 8)
    assert ei.value.status == -2
    # a path of 400 vertices: distances beyond one byte
    e = np.array([(i, i + 1) for i in range(399)], np.int64)
    prp, pcol, _ = P.build_csr(400, e[:, 0], e[:, 1])
    pd, pm, _ = P.run_batch(torch.from_numpy(prp).cuda(), torch.from_numpy(pcol).cuda(),
                            np.array([0, 1], np.int32), np.array([0], np.int32), 0)
    with pytest.raises(P.CbfsError) as ei:
        P.labels_pack_compact(pd, pm, 0, 8)
    assert ei.value.status == -2
