#!/usr/bin/env python3
"""Benchmark of the batched Cluster-BFS hot path on one MI355X.

Workload: the seeded R-MAT graph of scale 22, edge factor 16, quadrant
probabilities (0.57, 0.19, 0.19, 0.05), symmetrized, deduplicated, self-loops
removed, largest component kept (~2.39M vertices, ~128.3M arcs, int32 CSR);
256 radius-1 clusters whose centers are the 256 highest-degree vertices (ties
by id), each center plus its 63 lowest-id neighbours.  Synthetic stand-in for
the paper's real social/web graphs.

One step = one cbfs_run_batch over all 256 clusters (every output written),
with the graph, outputs and workspace already resident in device memory.
Reported: source-GTEPS = sum_c k_c * m / step time; the roofline of the
dominant kernel; the plain form (one cluster per call, same kernels); the CPU
oracle on a bounded sample of the same workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "source-GTEPS (sources×edges/s) + %HBM roofline; batched vs plain; query p50/p99"
KERNEL_SOURCES = ["cbfs_device.h", "cbfs_round.h", "cbfs_kernels.hip", "cbfs_kernels.h"]
WORKLOAD_NAMES = {
    "rmat22": ("rmat22_batch256", "R-MAT scale 22 ef 16 (0.57,0.19,0.19,0.05)"),
    "rmat14": ("rmat14_one_cluster", "R-MAT scale 14 ef 16 (0.57,0.19,0.19,0.05)"),
    "grid4096": ("grid4096_batch128", "4096x4096 4-neighbour grid, 5% of edges deleted"),
    "chunglu25": ("chunglu25_batch64", "Chung-Lu beta 2.1, n 2^25, average degree 30"),
}


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2410_17226_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(n, m, stats, C, k_w, R):
    """Compulsory HBM bytes of one batch (the per-group model of the design):
    per frontier appearance of a vertex its row-pointer pair (8 B), its arcs
    (4 B each), and its own state words read/written (24 B per word); the
    outputs written once (dist 4 B + 2R+1 planes of k_w words per cluster and
    vertex); and the per-group state clear (16 B per word and vertex)."""
    W = stats["group_words"]
    fv, fa = stats["frontier_vertices"], stats["frontier_arcs"]
    traversal = 8 * fv + 4 * fa
    own_state = 24 * W * fv
    outputs = C * n * (4 + 8 * k_w * (2 * R + 1))
    init = stats["groups"] * n * 16 * W
    return traversal + own_state + outputs + init


def pull_launch_bytes(n, m, stats, C, k_w, R):
    """Compulsory HBM bytes of one pull launch, averaged over a batch's pull
    launches: the dense pass (arcs 4m, row pointers 4(n+1), frontier bitmap
    n/8, every vertex's own state words 8Wn), the vertex phase fused into the
    launch (24 B per state word of each F_i vertex: own set and seen set read,
    seen set written, as in the batch model), and the outputs, attributed to
    pull rounds in proportion of their frontier vertices."""
    W = stats["group_words"]
    pulls = max(1, stats["pull_rounds"])
    fv_pull = stats.get("pull_frontier_vertices", 0)
    fv = max(1, stats["frontier_vertices"])
    dense_pass = 4 * m + 4 * (n + 1) + n // 8 + 8 * W * n
    outputs = C * n * (4 + 8 * k_w * (2 * R + 1))
    return int(dense_pass + (24 * W * fv_pull + outputs * fv_pull / fv) / pulls)


def load_traffic(kind: str, workload: str):
    """Measured HBM bytes per launch from committed rocprofv3 counter runs,
    only if they were taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"{kind}_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_hash") != kernel_hash():
        return None
    return rec.get("bytes_per_launch")


def golden_pairs(n, m):
    """Oracle answers (tests/golden/serve_rmat22_pairs.txt, written by the
    golden script from the oracle) of the first queries of the serving stream,
    if they were made for this graph."""
    path = os.path.join(ROOT, "tests", "golden", "serve_rmat22_pairs.txt")
    if not os.path.exists(path):
        return None
    meta, ans = {}, []
    with open(path) as f:
        for ln in f:
            if ln.startswith("# n="):
                meta = dict(kv.split("=") for kv in ln[2:].split())
            elif ln.startswith("stream "):
                ans.append(int(ln.split()[3]))
    if int(meta.get("n", -1)) != n or int(meta.get("m", -1)) != m:
        return None
    return np.array(ans, dtype=np.uint32)


def median_call_ms(fn, reps, warm=2):
    import torch
    st = torch.cuda.current_stream()
    for _ in range(warm):
        fn(st)
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        fn(st)
        b.record(st)
        b.synchronize()
        times.append(a.elapsed_time(b))
    return float(np.median(times))


def diameter_table(P, torch, rp, col, rp_d, col_d, m):
    """Time of C-BFS in the paper's own encoding for clusters of diameter
    d = 2..6 (each: the highest-degree free vertex and the 63 highest-degree
    free vertices within floor(d/2) hops, Section 4.2), relative to d = 2."""
    rows = []
    for d in range(2, 7):
        cp, src = P.select_landmarks(rp, col, 64, 64, d)
        one = np.array([0, cp[1]], np.int32)
        out1 = P.run_batch(rp_d, col_d, one, src[: cp[1]], d, encoding=P.CBFS_ENCODE_MIN)
        t1 = median_call_ms(lambda st: P.run_batch(rp_d, col_d, one, src[: cp[1]], d, out=out1, stream=st,
                                                   encoding=P.CBFS_ENCODE_MIN), 7)
        st1 = out1[2].cpu().numpy()
        outb = P.run_batch(rp_d, col_d, cp, src, d, encoding=P.CBFS_ENCODE_MIN)
        tb = median_call_ms(lambda st: P.run_batch(rp_d, col_d, cp, src, d, out=outb, stream=st,
                                                   encoding=P.CBFS_ENCODE_MIN), 3, warm=1)
        ok = bool((st1 == 0).all() and (outb[2].cpu().numpy() == 0).all())
        ksum = int(cp[-1])
        rows.append({"d": d, "one_cluster_ms": round(t1, 3), "batch_clusters": int(cp.size - 1), "batch_ms": round(tb, 2),
                     "batch_source_gteps": round(ksum * m / (tb * 1e-3) / 1e9, 1), "status_ok": ok})
        del outb, out1
    base1, baseb = rows[0]["one_cluster_ms"], rows[0]["batch_ms"]
    for r in rows:
        r["one_cluster_rel"] = round(r["one_cluster_ms"] / base1, 3)
        r["batch_rel"] = round(r["batch_ms"] / baseb, 3)
    return rows


def ll_distortion(P, torch, rp, col, rp_d, col_d, pairs=4096, seed=91, local_taus=(), budget=0):
    """Landmark labeling as Section 4.2 builds it (clusters of 64 selected by
    degree with marking, d = 2, star labels with offsets -1 and 0) for several
    label counts; distortion of the query answer against exact distances from
    a GPU batch of single-source searches (radius 0).  With ``local_taus``,
    the 128-cluster labels are also combined with the bidirectional local
    search of Appendix B for each tau; with ``budget``, the memory-budget
    comparison of plain landmarks and clusters of 8 .. 64 sources."""
    import synth
    n = rp.size - 1
    qs, qt = synth.query_pairs(n, pairs, seed)
    exact = np.empty(pairs, np.int64)
    for lo in range(0, pairs, 512):  # exact distances, 512 single-source searches at a time
        hi = min(pairs, lo + 512)
        one = np.arange(hi - lo + 1, dtype=np.int32)
        ex_d, ex_m, ex_st = P.run_batch(rp_d, col_d, one, qs[lo:hi], 0)
        exact[lo:hi] = ex_d.cpu().numpy().view(np.uint32)[np.arange(hi - lo), qt[lo:hi]]
        assert (ex_st.cpu().numpy() == 0).all()
        del ex_d, ex_m
    qs_d, qt_d = torch.from_numpy(qs).to(rp_d.device), torch.from_numpy(qt).to(rp_d.device)
    out = []
    for r in (16, 64, 128):
        cp, src = P.select_landmarks(rp, col, r, 64, 2)
        dist, masks, st = P.run_batch(rp_d, col_d, cp, src, 1)
        dvm, mvm = P.labels_pack(dist, masks, 1)
        ans = P.query_batch(dvm, mvm, 1, qs_d, qt_d).cpu().numpy().view(np.uint32).astype(np.int64)
        pos = exact > 0
        ratio = ans[pos] / exact[pos]
        row = {"clusters": int(cp.size - 1), "landmarks": int(cp[-1]), "pairs": int(pos.sum()),
               "label_bytes_per_vertex": int((dvm.numel() * 4 + mvm.numel() * 8) // n),
               "mean_distortion": round(float(ratio.mean()), 4), "max_distortion": round(float(ratio.max()), 3),
               "exact_fraction": round(float((ans[pos] == exact[pos]).mean()), 4),
               "bound_holds": bool((ans >= exact).all())}
        if r == 128 and local_taus:
            row["local_search"] = local_search_table(P, torch, rp_d, col_d, dvm, mvm, qs_d, qt_d, exact, local_taus)
        out.append(row)
        del dist, masks, dvm, mvm
    if budget:
        out.append({"memory_budget_bytes_per_vertex": budget,
                    "rows": ll_budget_table(P, torch, rp, col, rp_d, col_d, qs_d, qt_d, exact, budget)})
    return out


def ll_budget_table(P, torch, rp, col, rp_d, col_d, qs_d, qt_d, exact, budget=1024, timed_queries=1 << 20):
    """Section 5.3's landmark-labeling comparison under a memory budget of
    `budget` bytes per vertex: plain landmarks (one distance byte each, the
    highest-degree vertices) against clusters of w = 8, 16, 32, 64 sources
    (Section 4.2's selection, d = 2, stored as one distance byte and two w-bit
    subsets: budget / (1 + w / 4) clusters).  Per configuration: device time of
    the index (C-BFS batch + compact packing), error of the answers on the
    sampled pairs, and the device query rate."""
    import synth
    n = rp.size - 1
    st = torch.cuda.current_stream()
    ts, tt = synth.query_pairs(n, timed_queries, 95)
    ts_d, tt_d = torch.from_numpy(ts).to(rp_d.device), torch.from_numpy(tt).to(rp_d.device)
    out_d = torch.empty(timed_queries, dtype=torch.int32, device=rp_d.device)
    pos = exact > 0
    rows = []
    for w in (0, 8, 16, 32, 64):
        if w == 0:
            lm = P.top_degree(rp, budget).astype(np.int32)
            cp, src, R, wq = np.arange(lm.size + 1, dtype=np.int32), lm, 0, 8
        else:
            cp, src = P.select_landmarks(rp, col, budget // (1 + w // 4), w, 2)
            R, wq = 1, w
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        dist, masks, stat = P.run_batch(rp_d, col_d, cp, src, R)
        d8, mc = P.labels_pack_compact(dist, masks, R, wq)
        e1.record(st)
        torch.cuda.synchronize()
        build_ms = e0.elapsed_time(e1)
        assert (stat.cpu().numpy() == 0).all()
        del dist, masks
        C = cp.size - 1
        a = P.query_batch_compact(d8, mc, R, wq, qs_d, qt_d).cpu().numpy().view(np.uint32).astype(np.int64)
        times = []
        for _ in range(3):
            q0, q1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            q0.record(st)
            P.query_batch_compact(d8, mc, R, wq, ts_d, tt_d, out=out_d, stream=st)
            q1.record(st)
            q1.synchronize()
            times.append(q0.elapsed_time(q1))
        rows.append({"w": w if w else "plain", "clusters": int(C), "landmarks": int(cp[-1]),
                     "bytes_per_vertex": int(C * (1 if w == 0 else 1 + w // 4)),
                     "index_ms": round(build_ms, 2),
                     "error_pct": round(float((a[pos] / exact[pos]).mean() - 1.0) * 100, 3),
                     "exact_fraction": round(float((a[pos] == exact[pos]).mean()), 4),
                     "bound_holds": bool((a >= exact).all()),
                     "device_qps": round(timed_queries / (float(np.median(times)) * 1e-3), 1)})
        print(f"[bench] budget {budget} B/vertex: {rows[-1]}", file=sys.stderr, flush=True)
        del d8, mc
    return rows


def local_search_table(P, torch, rp_d, col_d, dvm, mvm, qs_d, qt_d, exact, taus, timed_queries=1 << 17):
    """Appendix B's trade-off: the landmark answer combined (by a minimum) with
    a bidirectional local search of tau vertices per side.  Distortion over
    the sampled pairs against exact distances, and the device time of
    cbfs_query_batch + cbfs_query_local over uniform random pairs."""
    import synth
    n = rp_d.numel() - 1
    ts, tt = synth.query_pairs(n, timed_queries, 93)
    ts_d, tt_d = torch.from_numpy(ts).to(rp_d.device), torch.from_numpy(tt).to(rp_d.device)
    out_d = torch.empty(timed_queries, dtype=torch.int32, device=rp_d.device)
    st = torch.cuda.current_stream()
    pos = exact > 0
    close = pos & (exact <= 3)
    rows = []
    for tau in [0] + list(taus):
        ans = P.query_batch(dvm, mvm, 1, qs_d, qt_d)
        if tau:
            P.query_local(rp_d, col_d, qs_d, qt_d, tau, out=ans)
        a = ans.cpu().numpy().view(np.uint32).astype(np.int64)
        ratio = a[pos] / exact[pos]
        times = []
        for _ in range(3):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            P.query_batch(dvm, mvm, 1, ts_d, tt_d, out=out_d, stream=st)
            if tau:
                P.query_local(rp_d, col_d, ts_d, tt_d, tau, out=out_d, stream=st)
            e1.record(st)
            e1.synchronize()
            times.append(e0.elapsed_time(e1))
        ms = float(np.median(times))
        rows.append({"tau": tau, "mean_distortion": round(float(ratio.mean()), 4),
                     "exact_fraction": round(float((a[pos] == exact[pos]).mean()), 4),
                     "close_pairs": int(close.sum()),
                     "close_mean_distortion": round(float((a[close] / exact[close]).mean()), 4) if close.any() else None,
                     "bound_holds": bool((a >= exact).all()),
                     "device_qps": round(timed_queries / (ms * 1e-3), 1),
                     "us_per_query_amortized": round(ms * 1e3 / timed_queries, 4)})
        print(f"[bench] local search: {rows[-1]}", file=sys.stderr, flush=True)
    return rows


def pll_table(P, torch, dev, scale=16, clusters=16, label_cap=2048, pairs=512, cpu=True):
    """The exact distance oracle of the paper's appendix on an R-MAT graph:
    phase 1 = C-BFS labels of `clusters` landmark clusters (Section 4.2's
    selection, 64 sources, d = 2), phase 2 = pruned BFS from every other vertex
    in batches of 200 * 1.5^i (at most 1000).  Device times of both phases,
    label sizes, the device query rate over 10^6 random pairs, and exactness on
    sampled pairs against a GPU batch of single-source searches; with `cpu`,
    the oracle's phase 2 on the same input, timed on the host."""
    import synth
    n_in, s, d = synth.rmat_edges(scale, 16, seed=77)
    rp, col, _ = P.build_csr(n_in, s, d)
    n, m = rp.size - 1, col.size
    rp_d, col_d = torch.from_numpy(rp).to(dev), torch.from_numpy(col).to(dev)
    st = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    cp, src = P.select_landmarks(rp, col, clusters, 64, 2)
    ev[0].record(st)
    dist, masks, stat = P.run_batch(rp_d, col_d, cp, src, 1)
    dvm, mvm = P.labels_pack(dist, masks, 1)
    ev[1].record(st)
    deg = np.diff(rp)
    order = np.lexsort((np.arange(n), -deg)).astype(np.int32)
    order = order[~np.isin(order, src)]
    order_d = torch.from_numpy(order).to(dev)
    bp = (dvm, mvm, 1)
    P.pll_build(rp_d, col_d, order_d, bp=bp, label_cap=label_cap)  # warm-up
    ev[2].record(st)
    cnt_d, lab_d = P.pll_build(rp_d, col_d, order_d, bp=bp, label_cap=label_cap)
    ev[3].record(st)
    torch.cuda.synchronize()
    assert (stat.cpu().numpy() == 0).all()
    cnt = cnt_d.cpu().numpy()
    qn = 1_000_000
    qs, qt = synth.query_pairs(n, qn, 78)
    qs_d, qt_d = torch.from_numpy(qs).to(dev), torch.from_numpy(qt).to(dev)
    ans_d = torch.empty(qn, dtype=torch.int32, device=dev)
    P.pll_query(cnt_d, lab_d, qs_d, qt_d, bp=bp, out=ans_d)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    P.pll_query(cnt_d, lab_d, qs_d, qt_d, bp=bp, out=ans_d)
    e1.record(st)
    torch.cuda.synchronize()
    q_ms = e0.elapsed_time(e1)
    # exactness on sampled pairs: exact distances from a batch of single-source searches
    one = np.arange(pairs + 1, dtype=np.int32)
    ex_d, _, ex_st = P.run_batch(rp_d, col_d, one, qs[:pairs], 0)
    exact = ex_d.cpu().numpy().view(np.uint32)[np.arange(pairs), qt[:pairs]]
    got = ans_d[:pairs].cpu().numpy().view(np.uint32)
    out = {"graph": f"R-MAT scale {scale} ef 16", "n": int(n), "m_arcs": int(m), "phase1_clusters": int(cp.size - 1),
           "phase1_sources": int(cp[-1]), "phase2_roots": int(order.size),
           "batches": len(_pll_batches(order.size)),
           "phase1_ms": round(ev[0].elapsed_time(ev[1]), 3), "phase2_ms": round(ev[2].elapsed_time(ev[3]), 3),
           "labels_per_vertex_mean": round(float(cnt.mean()), 2), "labels_per_vertex_max": int(cnt.max()),
           "index_bytes": int(cnt.sum() * 8 + dvm.numel() * 4 + mvm.numel() * 8),
           "device_qps_1M": round(qn / (q_ms * 1e-3), 1), "exact_on_sampled_pairs": bool(np.array_equal(got, exact)),
           "sampled_pairs": pairs}
    if cpu:
        import oracle
        od, om, _ = oracle.cbfs(rp, col, cp, src, R=1)
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        t = time.time()
        ocnt, olab = oracle.pll(rp, col, order, bp=(od, om), label_cap=label_cap, nthreads=threads)
        cpu_s = time.time() - t
        out["cpu_baseline"] = {"kind": "oracle", "phase2_s": round(cpu_s, 2), "cores": threads,
                               "same_labels_as_gpu": bool(np.array_equal(ocnt, cnt))}
    return out


def _pll_batches(count, first=200, growth=1.5, max_batch=1000):
    out, b, lo = [], first, 0
    while lo < count:
        size = min(b, count - lo)
        out.append(size)
        lo += size
        b = max(1, min(max_batch, int(b * growth)))
    return out


def gather_ceiling(torch, col_d, n, m, reps=5, blocks=4096):
    """Time of one pass that gathers, for every arc of the CSR in CSR order, a row of 64, 128
    or 256 bytes (the pull's arc-phase traffic with none of its other work), measured with the
    probe kernel of ``libcbfs_probe.so``: the floor for a pull round that gathers every arc's set."""
    import ctypes
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2410_17226_amd", "libcbfs_probe.so"))
    lib.cbfs_probe_gather.restype = ctypes.c_int
    lib.cbfs_probe_gather.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]
    assert col_d.dtype == torch.int32 and col_d.is_contiguous() and col_d.numel() == m
    stream = torch.cuda.current_stream()
    out = torch.empty(blocks * 256, dtype=torch.int64, device=col_d.device)
    res = {}
    for row in (64, 128, 256):
        state = torch.ones((n, row // 8), dtype=torch.int64, device=col_d.device)

        def once():
            rc = lib.cbfs_probe_gather(row, col_d.data_ptr(), m, state.data_ptr(), out.data_ptr(), blocks,
                                       stream.cuda_stream)
            if rc != 0:
                raise RuntimeError(f"gather probe launch failed ({rc})")
        once()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            once()
        e1.record(stream)
        torch.cuda.synchronize()
        res[str(row)] = round(e0.elapsed_time(e1) / reps, 3)
        del state
    return {"pass_ms": res, "row_bytes": [64, 128, 256],
            "note": "one pass over all arcs in CSR order gathering a row of each size per arc (probe kernel, "
                    "no other work): the floor for a pull round that gathers every arc's set"}


def rmat14_latency(P, torch, dev):
    """The one-cluster R-MAT scale-14 workload: time of one cbfs_run_batch
    (median of 20 after 3 warm-ups), graph and outputs resident."""
    from synth import configs
    cfg = configs.WORKLOADS["rmat14"]
    n_in, src, dst = configs.raw_graph("rmat14")
    rp, col, _ = P.build_csr(n_in, src, dst)
    cp, s = P.select_clusters(rp, col, P.top_degree(rp, 1), cfg["k"], cfg["hops"])
    rp_d, col_d = torch.from_numpy(rp).to(dev), torch.from_numpy(col).to(dev)
    out = P.run_batch(rp_d, col_d, cp, s, cfg["R"])
    ws = torch.empty(P.run_batch_workspace_size(rp_d, col_d, cp, s, cfg["R"]), dtype=torch.uint8, device=dev)
    st = torch.cuda.current_stream()
    for _ in range(3):
        P.run_batch(rp_d, col_d, cp, s, cfg["R"], out=out, workspace=ws, stream=st)
    times = []
    for _ in range(20):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        P.run_batch(rp_d, col_d, cp, s, cfg["R"], out=out, workspace=ws, stream=st)
        b.record(st)
        b.synchronize()
        times.append(a.elapsed_time(b))
    ms = float(np.median(times))
    k = int(cp[-1])
    return {"workload": "rmat14_one_cluster", "n": int(rp.size - 1), "m_arcs": int(col.size), "sources": k,
            "median_ms": round(ms, 4), "source_gteps": round(k * col.size / (ms * 1e-3) / 1e9, 2),
            "stats": P.last_run_stats()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--mode", type=int, default=0, help="0 auto, 1 host loop, 2 persistent")
    ap.add_argument("--group-words", type=int, default=0)
    ap.add_argument("--slots", type=int, default=0)
    ap.add_argument("--alpha", type=float, default=0.0, help="push/pull threshold (0 = library default)")
    ap.add_argument("--beta", type=float, default=0.0, help="pull/push threshold (0 = library default)")
    ap.add_argument("--gamma", type=float, default=0.0, help="wave-form threshold (0 = library default)")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-clusters", type=int, default=6, help="clusters in the CPU oracle sample")
    ap.add_argument("--no-query", action="store_true")
    ap.add_argument("--no-gather-ceiling", action="store_true", help="skip the gather-probe floor of the pull")
    ap.add_argument("--workload", default="rmat22", choices=["rmat22", "grid4096", "chunglu25", "rmat14"],
                    help="batch workload (the default is the headline one)")
    ap.add_argument("--no-rmat14", action="store_true", help="skip the one-cluster R-MAT 14 latency figure")
    ap.add_argument("--serve-queries", type=int, default=1_000_000, help="queries served per offered rate")
    ap.add_argument("--diameters", action="store_true",
                    help="also time clusters of diameter d = 2..6 in the paper's own encoding <S_v[0..d], Delta_v> "
                         "(landmark selection of Section 4.2), one cluster per call and a 64-cluster batch")
    ap.add_argument("--ll", action="store_true",
                    help="also measure landmark-labeling distortion (clusters selected as in Section 4.2) against "
                         "exact distances computed on the GPU")
    ap.add_argument("--ll-budget", type=int, default=1024,
                    help="with --ll: bytes per vertex for the plain / w = 8..64 comparison (0 = skip)")
    ap.add_argument("--local-taus", default="128,256,512,1024,2048",
                    help="with --ll: local search sizes (vertices per side) combined with the 128-cluster labels")
    ap.add_argument("--pll", type=int, default=0, metavar="SCALE",
                    help="also build the exact 2-hop oracle (pruned landmark labeling) on an R-MAT graph of this scale")
    ap.add_argument("--pll-cap", type=int, default=2048, help="label capacity per vertex of the exact oracle")
    ap.add_argument("--tune", action="store_true",
                    help="autotune the launch knobs on the first 16 clusters before timing (untimed)")
    ap.add_argument("--copy-only", type=int, default=0,
                    help="only run one device-to-device copy of this many bytes (counter calibration)")
    ap.add_argument("--gather-only", type=int, default=0,
                    help="only run one gather of this many random 64-byte rows out of a 4 GiB table "
                         "(counter calibration for scattered 64-byte reads)")
    args = ap.parse_args()
    if args.gather_only:
        import torch
        rows = 1 << 26  # 4 GiB of 64-byte rows: far beyond every cache
        table = torch.ones((rows, 8), dtype=torch.int64, device="cuda")
        g = torch.Generator(device="cuda")
        g.manual_seed(7)
        idx = torch.randint(0, rows, (args.gather_only,), device="cuda", generator=g)
        torch.cuda.synchronize()
        out = table.index_select(0, idx)
        torch.cuda.synchronize()
        print(json.dumps({"gather_rows": args.gather_only, "row_bytes": 64, "index_bytes": 8,
                          "distinct_rows": int(torch.unique(idx).numel()), "check": int(out[:, 0].sum())}))
        return
    if args.copy_only:
        import torch
        x = torch.empty(args.copy_only, dtype=torch.uint8, device="cuda")
        y = torch.empty_like(x)
        x.fill_(1)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": args.copy_only}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; a batch of clusters would shard "
                                   "across GPUs by cluster groups with a replicated CSR and no communication "
                                   "during the search, which is not built", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import paper_2410_17226_amd as P
    import synth
    from synth import configs

    cfg = configs.WORKLOADS[args.workload]
    t0 = time.time()
    n_in, src, dst = configs.raw_graph(args.workload)
    rp, col, _ = P.build_csr(n_in, src, dst)
    del src, dst
    n, m = rp.size - 1, col.size
    if cfg["centers"] == "top_degree":
        centers = P.top_degree(rp, cfg["count"])
    else:
        centers = synth.random_centers(n, cfg["count"], cfg["seed"]).astype(np.int32)
    cptr, sources = P.select_clusters(rp, col, centers, cfg["k"], cfg["hops"])
    R = cfg["R"]
    C = cptr.size - 1
    ksum = int(cptr[-1])
    k_w = (int(np.diff(cptr).max()) + 63) // 64
    setup_s = time.time() - t0
    print(f"[bench] graph n={n} m={m} clusters={C} sources={ksum} setup {setup_s:.1f}s", file=sys.stderr,
          flush=True)

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    rp_d = torch.from_numpy(rp).to(dev)
    col_d = torch.from_numpy(col).to(dev)
    tuning = P.Tuning(mode=args.mode, group_words=args.group_words, concurrent_groups=args.slots,
                      alpha=args.alpha, beta=args.beta, gamma=args.gamma)
    tuned = None
    if args.tune:
        t0 = time.time()
        tuning, trials = P.autotune(rp_d, col_d, cptr, sources, R, start=tuning, sample_clusters=16)
        tuned = {"chosen": vars(tuning), "trials": len(trials), "seconds": round(time.time() - t0, 2),
                 "best_trial_ms": round(min(ms for _, ms, _ in trials if ms >= 0), 2)}
        print(f"[bench] autotune: {tuned}", file=sys.stderr, flush=True)
        for t, ms, mode in trials:
            print(f"[bench]   trial mode={mode} {vars(t)} {ms:.2f} ms", file=sys.stderr, flush=True)
    dist = torch.empty((C, n), dtype=torch.int32, device=dev)
    masks = torch.empty((C, 2 * R + 1, n, k_w), dtype=torch.int64, device=dev)
    status = torch.empty(C, dtype=torch.int32, device=dev)
    ws_bytes = P.run_batch_workspace_size(rp_d, col_d, cptr, sources, R, tuning)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    out = (dist, masks, status)

    for _ in range(args.warmup):
        P.run_batch(rp_d, col_d, cptr, sources, R, tuning, out=out, workspace=ws)
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    wall0 = time.time()
    ev0.record(stream)
    for k in range(args.steps):
        marks[k].record(stream)
        P.run_batch(rp_d, col_d, cptr, sources, R, tuning, out=out, workspace=ws, stream=stream)
    marks[args.steps].record(stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.time() - wall0
    step_ms = ev0.elapsed_time(ev1) / args.steps
    per_step = [marks[k].elapsed_time(marks[k + 1]) for k in range(args.steps)]
    median_ms = float(np.median(per_step))
    # one more step with every kernel launch bracketed by HIP events on the
    # library's stream, for the per-kernel attribution of the roofline
    P.profile_enable(True)
    P.run_batch(rp_d, col_d, cptr, sources, R, tuning, out=out, workspace=ws, stream=stream)
    prof = P.profile_read()
    P.profile_enable(False)
    stats = P.last_run_stats()
    prof_steps = 1
    assert (status.cpu().numpy() == 0).all(), "a cluster reported a radius violation"
    gteps = ksum * m / (step_ms * 1e-3) / 1e9
    print(f"[bench] batched: {step_ms:.2f} ms/step ({wall / args.steps * 1e3:.2f} wall) GTEPS={gteps:.1f} "
          f"stats={stats} prof={prof}", file=sys.stderr, flush=True)

    # roofline of the dominant kernel
    kind, (launches, total_ms) = max(prof.items(), key=lambda kv: kv[1][1])
    avg_ms = total_ms / max(1, launches)
    B_alg_step = algorithmic_bytes(n, m, stats, C, k_w, R)
    if kind == "persistent":
        per_launch = B_alg_step * prof_steps / launches
        unit_note = "one batch (all groups) per launch"
    elif kind == "pull":
        per_launch = pull_launch_bytes(n, m, stats, C, k_w, R)
        unit_note = ("one dense pass over the CSR, the frontier bitmap and the group state, plus the fused "
                     "vertex phase of F_i (24 B per state word of each frontier vertex) and its share of the "
                     "outputs, averaged over the batch's pull launches")
    else:
        per_launch = B_alg_step * prof_steps / launches
        unit_note = "batch bytes spread over the launches"
    achieved = per_launch / (avg_ms * 1e-3) / 1e9
    traffic = load_traffic(kind, args.workload)
    roofline = {"bound": "hbm", "kernel": kind, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "bytes_per_launch": int(per_launch), "avg_launch_ms": round(avg_ms, 3), "launches": launches,
                "units": unit_note, "step_algorithmic_bytes": int(B_alg_step),
                "step_frac": round(B_alg_step / (step_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}

    if not args.no_gather_ceiling:
        roofline["gather_ceiling"] = gather_ceiling(torch, col_d, n, m)
        print(f"[bench] gather ceiling: {roofline['gather_ceiling']['pass_ms']}", file=sys.stderr, flush=True)

    # plain form: one cluster per call, same kernels and defaults
    plain = None
    if not args.no_plain:
        # outputs of their own, so the batch's labels stay intact for the query legs
        one = (torch.empty_like(dist[:1]), torch.empty_like(masks[:1]), torch.empty_like(status[:1]))
        torch.cuda.synchronize()
        ev0.record(stream)
        for ci in range(C):
            cp1 = np.array([0, cptr[ci + 1] - cptr[ci]], np.int32)
            P.run_batch(rp_d, col_d, cp1, sources[cptr[ci]:cptr[ci + 1]], R, tuning, out=one, workspace=ws,
                        stream=stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        plain_ms = ev0.elapsed_time(ev1)
        plain = {"value": round(ksum * m / (plain_ms * 1e-3) / 1e9, 2), "ms": round(plain_ms, 2),
                 "calls": C, "batched_speedup": round(plain_ms / step_ms, 2)}
        # the compulsory bytes of searching every cluster on its own (one
        # cluster per level loop, as the plain calls do), delivered by the
        # batch; the per-call frontier counts come from an untimed second pass
        equiv = 0
        for ci in range(C):
            cp1 = np.array([0, cptr[ci + 1] - cptr[ci]], np.int32)
            P.run_batch(rp_d, col_d, cp1, sources[cptr[ci]:cptr[ci + 1]], R, tuning, out=one, workspace=ws,
                        stream=stream)
            equiv += algorithmic_bytes(n, m, P.last_run_stats(), 1, k_w, R)
        roofline["cluster_equivalent"] = {
            "bytes": int(equiv), "frac": round(equiv / (step_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "plain_frac": round(equiv / (plain_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "note": "sum over clusters of the batch model's bytes with each cluster in a group of its own, "
                    "divided by the batch's step time (frac) and by the plain calls' time (plain_frac)"}
        print(f"[bench] plain: {plain}", file=sys.stderr, flush=True)

    # CPU oracle on a bounded sample (the first clusters), also checked against the GPU
    cpu = None
    if not args.no_cpu:
        import oracle
        nc = args.cpu_clusters
        cps = cptr[: nc + 1]
        srcs = sources[: cps[-1]]
        P.run_batch(rp_d, col_d, cptr, sources, R, tuning, out=out, workspace=ws)
        torch.cuda.synchronize()
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        t = time.time()
        od, om, ost = oracle.cbfs(rp, col, cps, srcs, R=R, nthreads=threads)
        cpu_s = time.time() - t
        same = bool(np.array_equal(dist[:nc].cpu().numpy().view(np.uint32), od) and
                    np.array_equal(masks[:nc].cpu().numpy().view(np.uint64), om))
        cpu = {"value": round(int(cps[-1]) * m / cpu_s / 1e9, 3), "unit": "GTEPS", "cores": threads,
               "kind": "oracle", "sample": f"first {nc} clusters ({int(cps[-1])} sources, one BFS each) "
                                           f"of the same workload, {cpu_s:.1f} s",
               "gpu_matches_sample": same}
        # the same oracle on one thread, over the first 24 sources of the first cluster
        k1 = int(min(24, cptr[1]))
        t = time.time()
        od1, om1, _ = oracle.cbfs(rp, col, np.array([0, k1], np.int32), sources[:k1], R=R, W=k_w, nthreads=1)
        cpu1_s = time.time() - t
        cpu["one_thread"] = {"value": round(k1 * m / cpu1_s / 1e9, 3), "unit": "GTEPS", "cores": 1,
                             "sample": f"first {k1} sources of the first cluster, {cpu1_s:.1f} s"}
        del od1, om1
        print(f"[bench] cpu: {cpu}", file=sys.stderr, flush=True)

    # serving: labels of the first 128 clusters (the top-128 centers) kept on
    # the device; Poisson streams of uniform s-t queries at fixed rates
    query = None
    if not args.no_query and args.workload == "rmat22":
        from paper_2410_17226_amd import server
        CQ = min(128, C)
        dvm, mvm = P.labels_pack(dist[:CQ], masks[:CQ], R)
        torch.cuda.synchronize()
        qn = 1_000_000
        qs, qt = synth.query_pairs(n, qn, cfg["seed"] + 5)
        qs_d, qt_d = torch.from_numpy(qs).to(dev), torch.from_numpy(qt).to(dev)
        ans_d = torch.empty(qn, dtype=torch.int32, device=dev)
        P.query_batch(dvm, mvm, R, qs_d, qt_d, out=ans_d)
        torch.cuda.synchronize()
        ev0.record(stream)
        P.query_batch(dvm, mvm, R, qs_d, qt_d, out=ans_d, stream=stream)
        ev1.record(stream)
        torch.cuda.synchronize()
        kernel_ms = ev0.elapsed_time(ev1)
        query = {"clusters": CQ, "landmarks": int(cptr[CQ]), "label_bytes": int(dvm.numel() * 4 + mvm.numel() * 8),
                 "device_qps_1M_batch": round(qn / (kernel_ms * 1e-3), 1), "rates": []}
        gold = golden_pairs(n, m) if CQ == 128 else None
        ex = server.GpuExecutor(dvm, mvm, R, max_batch=1 << 16, lanes=4)
        count = min(args.serve_queries, qn)
        one_batch = ans_d[:count].cpu().numpy().view(np.uint32)
        for rate in (1e5, 1e6, 1e7):
            arr = synth.poisson_arrivals(rate, count, int(rate))
            rep = server.serve(ex, qs[:count], qt[:count], arr)
            same = bool(np.array_equal(rep.answers, one_batch))
            summ = rep.summary()
            summ.update({"offered_qps": rate, "same_as_one_batch": same})
            if gold is not None:
                g = min(gold.size, count)
                summ["same_as_oracle_first"] = g if bool(np.array_equal(rep.answers[:g], gold[:g])) else -1
            query["rates"].append({k: (round(v, 2) if isinstance(v, float) else v) for k, v in summ.items()})
            print(f"[bench] serve {rate:.0e} QPS: {summ}", file=sys.stderr, flush=True)
        del dvm, mvm

    dtab = diameter_table(P, torch, rp, col, rp_d, col_d, m) if args.diameters else None
    if dtab:
        print(f"[bench] diameters: {dtab}", file=sys.stderr, flush=True)
    taus = [int(x) for x in args.local_taus.split(",") if x.strip()]
    ll = ll_distortion(P, torch, rp, col, rp_d, col_d, local_taus=taus, budget=args.ll_budget) if args.ll else None
    if ll:
        print(f"[bench] landmark labeling: {ll}", file=sys.stderr, flush=True)
    pll = pll_table(P, torch, dev, scale=args.pll, label_cap=args.pll_cap, cpu=not args.no_cpu) if args.pll else None
    if pll:
        print(f"[bench] exact oracle: {pll}", file=sys.stderr, flush=True)
    r14 = None
    if not args.no_rmat14 and args.workload == "rmat22":
        r14 = rmat14_latency(P, torch, dev)
        print(f"[bench] rmat14: {r14}", file=sys.stderr, flush=True)

    line = {
        "metric": METRIC, "value": round(gteps, 2), "unit": "GTEPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(step_ms, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": WORKLOAD_NAMES[args.workload][0], "graph": WORKLOAD_NAMES[args.workload][1],
                   "n": n, "m_arcs": m, "clusters": C, "sources_per_cluster": int(cfg["k"]), "radius": R,
                   "group_words": stats["group_words"], "mode": stats["mode"], "slots": stats["slots"],
                   "parallelism": "single GPU"},
        "roofline": roofline, "cpu_baseline": cpu, "plain": plain, "query": query, "autotune": tuned,
        "run_stats": stats, "median_ms_per_step": round(median_ms, 3),
        "per_step_ms": [round(x, 3) for x in per_step], "rmat14": r14,
    }
    if dtab:
        line["diameters"] = dtab
    if ll:
        line["landmark_labeling"] = ll
    if pll:
        line["exact_oracle"] = pll
    if stats["mode"] == 2 or args.workload == "grid4096":
        line["levels_per_s"] = round(stats["rounds"] / (step_ms * 1e-3), 1)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
