"""GPU check of ``cbfs_run_batch_static``, the batch entry point that allocates
nothing (its workspace is the library's own device scratch array).

Its outputs must equal ``cbfs_run_batch``'s bit for bit on two calls in a row,
the second with a smaller input (the scratch keeps the first call's contents),
in both launch modes; a batch whose workspace exceeds the scratch is refused
before anything is enqueued.
"""
import numpy as np
import pytest

import synth
from synth import configs

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _workload(name):
    import paper_2410_17226_amd as P
    cfg = configs.WORKLOADS[name]
    n_in, s, d = configs.raw_graph(name)
    rp, col, _ = P.build_csr(n_in, s, d)
    if cfg["centers"] == "top_degree":
        centers = P.top_degree(rp, cfg["count"])
    else:
        centers = synth.random_centers(rp.size - 1, cfg["count"], cfg["seed"]).astype(np.int32)
    cp, src = P.select_clusters(rp, col, centers, cfg["k"], cfg["hops"])
    return rp, col, cp, src, cfg["R"]


def _small_grid(side, count, seed):
    import paper_2410_17226_amd as P
    n_in, s, d = synth.grid_edges(side, 0.05, seed=seed)
    rp, col, _ = P.build_csr(n_in, s, d)
    centers = synth.random_centers(rp.size - 1, count, seed).astype(np.int32)
    cp, src = P.select_clusters(rp, col, centers, 64, 2)
    return rp, col, cp, src, 2


def _same(torch, inputs, tuning, label):
    import paper_2410_17226_amd as P
    rp, col, cp, src, R = inputs
    rp_d, col_d = torch.from_numpy(rp).cuda(), torch.from_numpy(col).cuda()
    ws = P.run_batch_workspace_size(rp_d, col_d, cp, src, R, tuning)
    assert 0 < ws <= P.STATIC_SCRATCH_BYTES, (label, ws)
    print(f"[no_alloc] {label}: n={rp.size - 1} m={col.size} C={cp.size - 1} workspace={ws}", flush=True)
    d1, m1, s1 = P.run_batch_static(rp_d, col_d, cp, src, R, tuning)
    torch.cuda.synchronize()
    d0, m0, s0 = P.run_batch(rp_d, col_d, cp, src, R, tuning)
    torch.cuda.synchronize()
    assert (s0.cpu().numpy() == 0).all()
    assert np.array_equal(s1.cpu().numpy(), s0.cpu().numpy()), label
    assert np.array_equal(d1.cpu().numpy(), d0.cpu().numpy()), label
    assert np.array_equal(m1.cpu().numpy(), m0.cpu().numpy()), label


def test_static_matches_run_batch_host_loop_twice():
    torch = _torch()
    import paper_2410_17226_amd as P
    t = P.Tuning(mode=P.CBFS_MODE_HOST_LOOP)
    _same(torch, _workload("rmat16_batch"), t, "host loop, R-MAT 16, 32 clusters")
    _same(torch, _workload("rmat12_small"), t, "host loop, R-MAT 12, 16 clusters (smaller)")


def test_static_matches_run_batch_persistent_twice():
    torch = _torch()
    import paper_2410_17226_amd as P
    t = P.Tuning(mode=P.CBFS_MODE_PERSISTENT)
    _same(torch, _workload("grid128_small"), t, "persistent, grid 128, 16 clusters")
    _same(torch, _small_grid(48, 6, 3), t, "persistent, grid 48, 6 clusters (smaller)")


def test_static_refuses_a_batch_beyond_its_scratch():
    torch = _torch()
    import paper_2410_17226_amd as P
    rp, col, cp, src, R = _small_grid(512, 16, 5)
    rp_d, col_d = torch.from_numpy(rp).cuda(), torch.from_numpy(col).cuda()
    t = P.Tuning(mode=P.CBFS_MODE_PERSISTENT, field_bits=64)  # one cluster per word: 16 group slots
    assert P.run_batch_workspace_size(rp_d, col_d, cp, src, R, t) > P.STATIC_SCRATCH_BYTES
    with pytest.raises(P.CbfsError) as ei:
        P.run_batch_static(rp_d, col_d, cp, src, R, t)
    assert ei.value.status == -6  # CBFS_E_WORKSPACE, before any launch
