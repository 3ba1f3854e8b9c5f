#!/usr/bin/env python3
"""Writes the stored oracle results of the full-size workloads (test data).

Calls only the oracle (``oracle/``) and the seeded generators (``synth/``):
every stored value is the oracle's, computed on the CPU from the same seeded
raw graph the GPU tests build.

    python tests/golden/make_fullsize_golden.py serve_rmat22
        -> tests/golden/serve_rmat22_pairs.txt
    python tests/golden/make_fullsize_golden.py chunglu25
        -> tests/golden/chunglu25_digests.txt

serve_rmat22: the landmark-labeling query (Section 4.2; Algorithm "Framework
of Landmark Labeling", Query) over the sources of the 128 serving clusters
(top-128 centers of the scale-22 R-MAT rule, each with its 63 lowest-id
neighbours), answered by brute force as the minimum over that landmark set of
delta(x, s) + delta(x, t) (one BFS per distinct landmark), and the exact
delta(s, t) (one BFS from s), for the first 1000 pairs of the benchmark's
query stream plus pairs with a landmark endpoint and pairs with s = t.

chunglu25: SHA-256 digests of the oracle's center-relative outputs (dist
[n] uint32 and masks [2R+1][n][W] uint64, little-endian, that layout) of two
of the 64 clusters of 256 sources, plus digests of the cleaned CSR.
"""
from __future__ import annotations

import argparse
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402
from synth import configs  # noqa: E402

# the benchmark's query stream: synth.query_pairs(n, 1_000_000, seed of the
# rmat22 workload + 5), of which the first QPAIRS pairs are stored
QSTREAM = 1_000_000
QPAIRS = 1000
CHUNGLU_CLUSTERS = (0, 63)


def _log(msg):
    print(f"[golden {time.strftime('%H:%M:%S')}] {msg}", flush=True)


def sha(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def graph(name):
    n_in, s, d = configs.raw_graph(name)
    rp, col, _ = oracle.clean_csr(n_in, s, d)
    del s, d
    _log(f"{name}: n={rp.size - 1} m={col.size}")
    return rp, col


def serve_rmat22(threads):
    cfg = configs.WORKLOADS["serve_rmat22"]
    rp, col = graph("serve_rmat22")
    n = rp.size - 1
    centers = oracle.top_degree(rp, cfg["count"])
    cp, src = oracle.build_clusters(rp, col, centers, cfg["k"], cfg["hops"])
    landmarks = np.unique(src).astype(np.int32)
    _log(f"{cp.size - 1} clusters, {src.size} sources, {landmarks.size} distinct landmarks")
    qs, qt = synth.query_pairs(n, QSTREAM, configs.WORKLOADS["rmat22"]["seed"] + 5)
    qs, qt = qs[:QPAIRS].copy(), qt[:QPAIRS].copy()
    kind = ["stream"] * QPAIRS
    # a landmark endpoint (the answer is then exact) and s = t pairs
    es, et = synth.query_pairs(n, 32, 91)
    ls = src[np.arange(24) * 331 % src.size]
    qs = np.concatenate([qs, ls, es[24:32]]).astype(np.int32)
    qt = np.concatenate([qt, et[:24], es[24:32]]).astype(np.int32)
    kind += ["landmark_s"] * 24 + ["same"] * 8
    t = time.time()
    ans = oracle.query_landmarks(rp, col, np.array([0, landmarks.size], np.int32), landmarks, qs, qt,
                                 nthreads=threads)
    _log(f"landmark answers in {time.time() - t:.1f} s")
    t = time.time()
    delta = oracle.pair_distances(rp, col, qs, qt, nthreads=threads)
    _log(f"pair distances in {time.time() - t:.1f} s")
    assert (ans.astype(np.int64) >= delta.astype(np.int64)).all()
    out = os.path.join(HERE, "serve_rmat22_pairs.txt")
    with open(out, "w") as f:
        f.write("# Landmark-labeling query answers of the oracle on the serve_rmat22 workload (R-MAT scale 22,\n")
        f.write("# labels of the top-128 clusters, R = 1): ans = min over the clusters' sources x of\n")
        f.write("# delta(x,s)+delta(x,t) (Section 4.2, Algorithm \"Framework of Landmark Labeling\", Query),\n")
        f.write("# delta = delta(s,t) by plain BFS.  Written by tests/golden/make_fullsize_golden.py serve_rmat22\n")
        f.write(f"# n={n} m={col.size} row_ptr_sha256={sha(rp)} col_sha256={sha(col)}\n")
        f.write(f"# sources_sha256={sha(src)}\n")
        f.write("# kind s t ans delta\n")
        for j in range(qs.size):
            f.write(f"{kind[j]} {qs[j]} {qt[j]} {ans[j]} {delta[j]}\n")
    _log(f"wrote {out}")


def chunglu25(threads):
    cfg = configs.WORKLOADS["chunglu25"]
    rp, col = graph("chunglu25")
    n = rp.size - 1
    centers = oracle.top_degree(rp, cfg["count"])
    cp, src = oracle.build_clusters(rp, col, centers, cfg["k"], cfg["hops"])
    R = cfg["R"]
    lines = []
    for c in CHUNGLU_CLUSTERS:
        t = time.time()
        S = src[cp[c]:cp[c + 1]]
        od, om, st = oracle.cbfs(rp, col, np.array([0, S.size], np.int32), S, R=R, nthreads=threads)
        assert st[0] == 0
        lines.append(f"{c} {S.size} {sha(S)} {sha(od[0])} {sha(om[0])}")
        _log(f"cluster {c}: {S.size} sources in {time.time() - t:.1f} s")
        del od, om
    out = os.path.join(HERE, "chunglu25_digests.txt")
    with open(out, "w") as f:
        f.write("# SHA-256 digests of the oracle's center-relative C-BFS outputs on the chunglu25 workload\n")
        f.write("# (Chung-Lu beta 2.1, n = 2^25, average degree 30; clusters of 256 sources, R = 1):\n")
        f.write("# dist [n] uint32 and masks [2R+1][n][W] uint64 (W = 4), little-endian.\n")
        f.write("# Written by tests/golden/make_fullsize_golden.py chunglu25\n")
        f.write(f"# n={n} m={col.size} row_ptr_sha256={sha(rp)} col_sha256={sha(col)}\n")
        f.write("# cluster k sources_sha256 dist_sha256 masks_sha256\n")
        for ln in lines:
            f.write(ln + "\n")
    _log(f"wrote {out}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", choices=["serve_rmat22", "chunglu25"])
    ap.add_argument("--threads", type=int, default=0)
    a = ap.parse_args()
    {"serve_rmat22": serve_rmat22, "chunglu25": chunglu25}[a.which](a.threads)


if __name__ == "__main__":
    main()
