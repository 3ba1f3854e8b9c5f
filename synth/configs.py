"""The seeded workloads, as plain data (no arithmetic of the method).

Each workload names a raw-graph generator with its parameters and master seed,
a center rule (``top_degree`` = the top-``count`` vertices by cleaned degree,
ties by ascending id; ``random`` = ``count`` distinct uniform ids drawn from
the cleaned graph with the clusters substream), the sources per cluster ``k``
(center + lowest-id vertices within ``hops``), and the offset radius ``R``.

The first five entries are the benchmark workloads; the ``*_small`` entries are
the same recipes at sizes an oracle finishes in seconds.
"""
from __future__ import annotations

WORKLOADS = {
    "rmat14": dict(graph="rmat", scale=14, edge_factor=16, abc=(0.57, 0.19, 0.19), seed=14,
                   centers="top_degree", count=1, k=64, hops=1, R=1),
    "rmat22": dict(graph="rmat", scale=22, edge_factor=16, abc=(0.57, 0.19, 0.19), seed=22,
                   centers="top_degree", count=256, k=64, hops=1, R=1),
    "grid4096": dict(graph="grid", side=4096, delete_frac=0.05, seed=4096,
                     centers="random", count=128, k=64, hops=2, R=2),
    "chunglu25": dict(graph="chung_lu", n=1 << 25, beta=2.1, avg_deg=30.0, seed=25,
                      centers="top_degree", count=64, k=256, hops=1, R=1),
    "serve_rmat22": dict(graph="rmat", scale=22, edge_factor=16, abc=(0.57, 0.19, 0.19), seed=22,
                         centers="top_degree", count=128, k=64, hops=1, R=1,
                         query_seed=5, rates=(1e5, 1e6, 1e7)),
    # same recipes, oracle-sized
    "rmat12_small": dict(graph="rmat", scale=12, edge_factor=16, abc=(0.57, 0.19, 0.19), seed=12,
                         centers="top_degree", count=16, k=64, hops=1, R=1),
    "rmat16_batch": dict(graph="rmat", scale=16, edge_factor=16, abc=(0.57, 0.19, 0.19), seed=16,
                         centers="top_degree", count=32, k=64, hops=1, R=1),
    "grid128_small": dict(graph="grid", side=128, delete_frac=0.05, seed=128,
                          centers="random", count=16, k=64, hops=2, R=2),
    "chunglu16_small": dict(graph="chung_lu", n=1 << 16, beta=2.1, avg_deg=30.0, seed=16,
                            centers="top_degree", count=4, k=256, hops=1, R=1),
}


def raw_graph(name_or_cfg):
    """Raw (n, src, dst) edge list of a workload, before cleanup."""
    from . import rmat_edges, grid_edges, chung_lu_edges
    cfg = WORKLOADS[name_or_cfg] if isinstance(name_or_cfg, str) else name_or_cfg
    g = cfg["graph"]
    if g == "rmat":
        a, b, c = cfg["abc"]
        return rmat_edges(cfg["scale"], cfg["edge_factor"], a, b, c, seed=cfg["seed"])
    if g == "grid":
        return grid_edges(cfg["side"], cfg["delete_frac"], seed=cfg["seed"])
    if g == "chung_lu":
        return chung_lu_edges(cfg["n"], cfg["beta"], cfg["avg_deg"], seed=cfg["seed"])
    raise ValueError(g)
