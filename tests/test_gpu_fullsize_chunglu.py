"""GPU check of the Chung-Lu batch at its full size (n = 2^25, average degree
30, about 0.85 billion arcs; 64 clusters of 256 sources, four mask words per
offset), run exactly as ``bench.py --workload chunglu25`` launches it.

An exact oracle comparison would take one BFS per source over 0.85 billion
arcs (minutes per cluster), so sampled clusters are checked with the BFS
certificate in its word-parallel form, which holds exactly when the encoded
distances are the true ones;
the same recipe at 2^16 vertices is compared word for word in
``test_gpu_parity.py``.  The graph cleanup is the library's, checked against the
oracle's cleanup at smaller sizes in ``test_library.py``.
"""
import os
import time

import numpy as np
import pytest

import oracle
import synth
from synth import configs

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

THREADS = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)


def _log(msg):
    print(f"[chunglu25 {time.strftime('%H:%M:%S')}] {msg}", flush=True)


def test_chunglu25_batch_certified():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2410_17226_amd as P
    cfg = configs.WORKLOADS["chunglu25"]
    n_in, s, d = configs.raw_graph("chunglu25")
    rp, col, _ = P.build_csr(n_in, s, d)
    del s, d
    n = rp.size - 1
    centers = P.top_degree(rp, cfg["count"])
    cp, src = P.select_clusters(rp, col, centers, cfg["k"], cfg["hops"])
    ocp, osrc = oracle.build_clusters(rp, col, centers, cfg["k"], cfg["hops"])
    assert np.array_equal(cp, ocp) and np.array_equal(src, osrc)
    assert (np.diff(cp) == 256).all()
    _log(f"n={n} m={col.size} clusters={cp.size - 1}")
    rp_d, col_d = torch.from_numpy(rp).cuda(), torch.from_numpy(col).cuda()
    R = cfg["R"]
    dist, masks, st = P.run_batch(rp_d, col_d, cp, src, R)
    torch.cuda.synchronize()
    _log(f"run_batch done: {P.last_run_stats()}")
    assert (st.cpu().numpy() == 0).all()
    C = cp.size - 1
    for c in (0, C // 2, C - 1):
        gd = dist[c].cpu().numpy().view(np.uint32)
        gm = masks[c].cpu().numpy().view(np.uint64)
        bad = oracle.certificate_words(rp, col, src[cp[c]:cp[c + 1]], R, gd, gm, nthreads=THREADS)
        assert bad == 0, f"cluster {c}: {bad} certificate violations"
        # one component: the center reaches every vertex
        assert gd[src[cp[c]]] == 0 and (gd != 0xFFFFFFFF).all()
        _log(f"cluster {c}: certificate holds")
    del dist, masks, st
    torch.cuda.empty_cache()
