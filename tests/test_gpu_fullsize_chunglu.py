"""GPU check of the Chung-Lu batch at its full size (n = 2^25, average degree
30, about 0.85 billion arcs; 64 clusters of 256 sources, four mask words per
offset), run exactly as ``bench.py --workload chunglu25`` launches it.

An oracle run takes one BFS per source over 0.85 billion arcs (about five
minutes per cluster on 8 cores), so it was run once, by
``tests/golden/make_fullsize_golden.py chunglu25``, for two clusters (the first
and the last): their SHA-256 digests of dist and masks are stored in
``tests/golden/chunglu25_digests.txt`` and the GPU's outputs must hash to the
same values.  A third cluster is checked with the BFS certificate in its
word-parallel form, which holds exactly when the encoded distances are the
true ones.  The same recipe at 2^16 vertices is compared word for word in
``test_gpu_parity.py``.  The graph cleanup is the library's; the stored digests
of the oracle's own cleanup must match its CSR.
"""
import hashlib
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


def _golden(golden_dir):
    meta, rows = {}, {}
    with open(os.path.join(golden_dir, "chunglu25_digests.txt")) as f:
        for ln in f:
            if ln.startswith("# n="):
                meta = dict(kv.split("=") for kv in ln[2:].split())
            elif not ln.startswith("#"):
                c, k, s_sha, d_sha, m_sha = ln.split()
                rows[int(c)] = (int(k), s_sha, d_sha, m_sha)
    return meta, rows


def _sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def test_chunglu25_batch_exact_and_certified(golden_dir):
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
    meta, gold = _golden(golden_dir)
    assert int(meta["n"]) == n and int(meta["m"]) == col.size
    assert meta["row_ptr_sha256"] == _sha(rp) and meta["col_sha256"] == _sha(col)
    for c, (k, s_sha, d_sha, m_sha) in sorted(gold.items()):
        assert _sha(src[cp[c]:cp[c + 1]]) == s_sha and cp[c + 1] - cp[c] == k
        assert _sha(dist[c].cpu().numpy().view(np.uint32)) == d_sha, f"cluster {c}: dist differs from the oracle's"
        assert _sha(masks[c].cpu().numpy().view(np.uint64)) == m_sha, f"cluster {c}: masks differ from the oracle's"
        _log(f"cluster {c}: digests equal the oracle's")
    for c in (C // 2,):
        gd = dist[c].cpu().numpy().view(np.uint32)
        gm = masks[c].cpu().numpy().view(np.uint64)
        bad = oracle.certificate_words(rp, col, src[cp[c]:cp[c + 1]], R, gd, gm, nthreads=THREADS)
        assert bad == 0, f"cluster {c}: {bad} certificate violations"
        # one component: the center reaches every vertex
        assert gd[src[cp[c]]] == 0 and (gd != 0xFFFFFFFF).all()
        _log(f"cluster {c}: certificate holds")
    del dist, masks, st
    torch.cuda.empty_cache()
