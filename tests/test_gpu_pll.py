"""GPU parity of the exact 2-hop distance oracle (pruned landmark labeling in
batches of growing size; the paper's appendix on the exact distance oracle):
labels from cbfs_pll_build equal the oracle's entry for entry, with and
without phase-1 cluster labels, for the paper's batch schedule, for batches of
one root (the sequential method) and for batches run in several chunks; and
cbfs_pll_query answers every sampled pair with its exact distance."""
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


def _graphs():
    out = []
    n, s, d = synth.rmat_edges(12, 8, seed=21)
    out.append(("rmat12", n, s, d, 7))
    n, s, d = synth.random_graph(1500, 0.002, 22)
    out.append(("gnp_sparse", n, s, d, 7))
    n, s, d = synth.grid_edges(40, 0.1, seed=23)
    out.append(("grid40", n, s, d, 7))
    return out


def _setup(torch, P, n, s, d, flags, with_bp):
    rp, col, _ = P.build_csr(n, s, d, flags=flags)
    nv = rp.size - 1
    rp_d, col_d = torch.from_numpy(rp).cuda(), torch.from_numpy(col).cuda()
    bp_gpu = bp_ref = None
    sources = np.zeros(0, np.int32)
    if with_bp:
        cp, sources = P.select_landmarks(rp, col, 4, 32, 2)
        dist, masks, st = P.run_batch(rp_d, col_d, cp, sources, 1)
        assert (st.cpu().numpy() == 0).all()
        dvm, mvm = P.labels_pack(dist, masks, 1)
        bp_gpu = (dvm, mvm, 1)
        od, om, ost = oracle.cbfs(rp, col, cp, sources, R=1)
        bp_ref = (od, om)
    deg = np.diff(rp)
    order = np.lexsort((np.arange(nv), -deg)).astype(np.int32)
    order = order[~np.isin(order, sources)]
    return rp, col, rp_d, col_d, nv, bp_gpu, bp_ref, order


SCHEDULES = [dict(), dict(first=1, growth=1.0, max_batch=1), dict(first=7, growth=1.5, max_batch=40, slots=5)]


@pytest.mark.parametrize("gi", range(3))
@pytest.mark.parametrize("with_bp", [False, True])
@pytest.mark.parametrize("si", range(3))
def test_pll_labels_and_queries_match_oracle(gi, with_bp, si):
    torch = _torch()
    import paper_2410_17226_amd as P
    name, n, s, d, flags = _graphs()[gi]
    sched = SCHEDULES[si]
    if si == 1 and name == "rmat12":
        pytest.skip("one launch per root over 3,000 roots: covered by the smaller graphs")
    rp, col, rp_d, col_d, nv, bp_gpu, bp_ref, order = _setup(torch, P, n, s, d, flags, with_bp)
    cap = 1024
    print(f"[pll] graph={name} n={nv} m={col.size} bp={with_bp} sched={sched} roots={order.size}", flush=True)
    cnt_d, lab_d = P.pll_build(rp_d, col_d, torch.from_numpy(order).cuda(), bp=bp_gpu, label_cap=cap, **sched)
    torch.cuda.synchronize()
    cnt = cnt_d.cpu().numpy()
    lab = lab_d.cpu().numpy().view(np.uint64)
    ocnt, olab = oracle.pll(rp, col, order, bp=bp_ref, first=sched.get("first", 200),
                            growth=sched.get("growth", 1.5), max_batch=sched.get("max_batch", 1000), label_cap=cap)
    assert np.array_equal(cnt, ocnt), f"label sizes differ at {np.nonzero(cnt != ocnt)[0][:5]}"
    for v in range(nv):
        assert np.array_equal(lab[v, :cnt[v]], olab[v, :ocnt[v]]), f"label of vertex {v} differs"
    qs, qt = synth.query_pairs(nv, 4000, 31 + gi)
    qs[:10] = qt[:10]
    ans = P.pll_query(cnt_d, lab_d, torch.from_numpy(qs).cuda(), torch.from_numpy(qt).cuda(), bp=bp_gpu)
    torch.cuda.synchronize()
    ans = ans.cpu().numpy().view(np.uint32)
    exact = oracle.pair_distances(rp, col, qs, qt)
    assert np.array_equal(ans, exact), f"{np.sum(ans != exact)} answers are not the exact distance"
    assert np.array_equal(ans, oracle.pll_query(ocnt, olab, qs, qt, bp=bp_ref))


def test_pll_label_capacity_and_arguments():
    torch = _torch()
    import paper_2410_17226_amd as P
    name, n, s, d, flags = _graphs()[0]
    rp, col, rp_d, col_d, nv, _, _, order = _setup(torch, P, n, s, d, flags, False)
    order_d = torch.from_numpy(order).cuda()
    with pytest.raises(P.CbfsError) as ei:
        P.pll_build(rp_d, col_d, order_d, label_cap=2)
    assert ei.value.status == -6  # CBFS_E_WORKSPACE: a label would exceed its capacity
    for bad in (dict(label_cap=0), dict(label_cap=P.PLL_LABEL_CAP_MAX + 1), dict(growth=0.5)):
        with pytest.raises(P.CbfsError):
            P.pll_build(rp_d, col_d, order_d, **{"label_cap": 64, **bad})


def test_pll_rmat14_full_schedule_matches_oracle():
    """R-MAT 14 (about 12K roots: the paper's batch schedule reaches its cap of
    1,000 roots and runs 16 batches), phase 1 of 8 landmark clusters: labels
    equal the oracle's entry for entry, and 20,000 queries are exact."""
    torch = _torch()
    import paper_2410_17226_amd as P
    n, s, d = synth.rmat_edges(14, 16, seed=41)
    rp, col, rp_d, col_d, nv, _, _, _ = _setup(torch, P, n, s, d, 15, False)
    cp, src = P.select_landmarks(rp, col, 8, 64, 2)
    dist, masks, st = P.run_batch(rp_d, col_d, cp, src, 1)
    dvm, mvm = P.labels_pack(dist, masks, 1)
    od, om, _ = oracle.cbfs(rp, col, cp, src, R=1)
    deg = np.diff(rp)
    order = np.lexsort((np.arange(nv), -deg)).astype(np.int32)
    order = order[~np.isin(order, src)]
    assert len(oracle.pll_batches(order.size)) >= 12
    print(f"[pll] rmat14 n={nv} roots={order.size}", flush=True)
    cnt_d, lab_d = P.pll_build(rp_d, col_d, torch.from_numpy(order).cuda(), bp=(dvm, mvm, 1), label_cap=1024)
    torch.cuda.synchronize()
    cnt = cnt_d.cpu().numpy()
    lab = lab_d.cpu().numpy().view(np.uint64)
    ocnt, olab = oracle.pll(rp, col, order, bp=(od, om), label_cap=1024)
    assert np.array_equal(cnt, ocnt)
    mask = np.arange(1024)[None, :] < cnt[:, None]
    assert np.array_equal(lab[mask], olab[mask])
    qs, qt = synth.query_pairs(nv, 20000, 43)
    ans = P.pll_query(cnt_d, lab_d, torch.from_numpy(qs).cuda(), torch.from_numpy(qt).cuda(), bp=(dvm, mvm, 1))
    torch.cuda.synchronize()
    assert np.array_equal(ans.cpu().numpy().view(np.uint32), oracle.pair_distances(rp, col, qs, qt))
