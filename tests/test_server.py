"""Continuous-batching server: scheduling logic on the CPU with a fake executor
whose answers come from the oracle's label query, and the GPU executor
against the brute-force landmark oracle."""
import time

import numpy as np
import pytest

import oracle
import synth
from paper_2410_17226_amd import server


class FakeExecutor:
    """Lanes that finish `delay` seconds after submission; answers from a
    CPU function of (s, t)."""

    def __init__(self, answer_fn, lanes=3, capacity=64, delay=0.002):
        self.lanes, self.capacity, self.delay = lanes, capacity, delay
        self.answer_fn = answer_fn
        self._ready = [None] * lanes
        self._args = [None] * lanes
        self.submitted = []

    def submit(self, lane, s, t):
        assert self._ready[lane] is None, "lane reused before its batch finished"
        assert s.size <= self.capacity
        self._ready[lane] = time.perf_counter() + self.delay
        self._args[lane] = (s.copy(), t.copy())
        self.submitted.append(s.size)

    def done(self, lane):
        return self._ready[lane] is not None and time.perf_counter() >= self._ready[lane]

    def fetch(self, lane):
        s, t = self._args[lane]
        self._ready[lane] = None
        return self.answer_fn(s, t)


@pytest.fixture(scope="module")
def labels():
    n, s, d = synth.rmat_edges(10, 8, seed=31)
    rp, col, _ = oracle.clean_csr(n, s, d)
    cp, src = oracle.build_clusters(rp, col, oracle.top_degree(rp, 6), 64, 1)
    dist, masks, st = oracle.cbfs(rp, col, cp, src, R=1)
    assert (st == 0).all()
    return rp, col, cp, src, dist, masks


def test_serve_matches_alone_and_batches_continuously(labels):
    rp, col, cp, src, dist, masks = labels
    nv = rp.size - 1
    qs, qt = synth.query_pairs(nv, 3000, 4)
    arrivals = synth.poisson_arrivals(2e5, qs.size, 4)   # ~15 ms of arrivals
    fn = lambda a, b: oracle.query_labels(dist, masks, a, b)  # noqa: E731
    ex = FakeExecutor(fn, lanes=3, capacity=128, delay=0.003)
    rep = server.serve(ex, qs, qt, arrivals)
    alone = np.array([fn(qs[i:i + 1], qt[i:i + 1])[0] for i in range(qs.size)], dtype=np.uint32)
    assert np.array_equal(rep.answers, alone)
    assert np.array_equal(rep.answers, oracle.query_landmarks(rp, col, cp, src, qs, qt))
    assert rep.max_in_flight > 1            # later arrivals were admitted while earlier batches ran
    assert max(ex.submitted) <= 128 and sum(ex.submitted) == qs.size
    assert np.all(rep.latency_s >= 0)
    summ = rep.summary()
    assert summ["queries"] == qs.size and summ["p99_us"] >= summ["p50_us"] > 0


def test_serve_single_lane_and_late_arrivals(labels):
    rp, col, cp, src, dist, masks = labels
    nv = rp.size - 1
    qs, qt = synth.query_pairs(nv, 200, 9)
    arrivals = np.linspace(0, 0.02, qs.size)
    fn = lambda a, b: oracle.query_labels(dist, masks, a, b)  # noqa: E731
    ex = FakeExecutor(fn, lanes=1, capacity=16, delay=0.0005)
    rep = server.serve(ex, qs, qt, arrivals, idle_sleep=0.0005)
    assert np.array_equal(rep.answers, fn(qs, qt))
    assert rep.max_in_flight == 1
    # nothing completes before it arrives
    assert np.all(rep.latency_s >= 0)


class CountingExecutor(FakeExecutor):
    """Records the queries on the device at every submission."""

    def __init__(self, *a, **k):
        super().__init__(*a, **k)
        self.on_device = 0
        self.peak = 0
        self._sizes = [0] * self.lanes

    def submit(self, lane, s, t):
        super().submit(lane, s, t)
        self._sizes[lane] = s.size
        self.on_device += s.size
        self.peak = max(self.peak, self.on_device)

    def fetch(self, lane):
        self.on_device -= self._sizes[lane]
        return super().fetch(lane)


def test_serve_memory_budget_bounds_queries_in_flight(labels):
    """Admission by memory: with room for 100 queries on the device, no more
    than 100 are ever in flight, batches are cut to fit, and every answer is
    still the one the request gets alone."""
    rp, col, cp, src, dist, masks = labels
    nv = rp.size - 1
    qs, qt = synth.query_pairs(nv, 2000, 21)
    arrivals = synth.poisson_arrivals(5e5, qs.size, 21)
    fn = lambda a, b: oracle.query_labels(dist, masks, a, b)  # noqa: E731
    ex = CountingExecutor(fn, lanes=4, capacity=64, delay=0.002)
    rep = server.serve(ex, qs, qt, arrivals, max_in_flight_queries=100)
    assert not rep.rejected.any()
    assert np.array_equal(rep.answers, fn(qs, qt))
    assert ex.peak <= 100 and rep.max_in_flight_queries <= 100
    assert rep.max_in_flight >= 2          # two batches fit side by side
    assert sum(ex.submitted) == qs.size and max(ex.submitted) <= 64


def test_serve_sheds_load_beyond_the_backlog(labels):
    """Overload (arrivals far faster than the lanes drain): requests that find
    the backlog full are rejected at arrival and get no answer; every admitted
    request is answered correctly; rejections appear only under overload."""
    rp, col, cp, src, dist, masks = labels
    nv = rp.size - 1
    qs, qt = synth.query_pairs(nv, 3000, 22)
    arrivals = np.linspace(0.0, 0.003, qs.size)       # 1e6 QPS offered
    fn = lambda a, b: oracle.query_labels(dist, masks, a, b)  # noqa: E731
    ex = FakeExecutor(fn, lanes=1, capacity=32, delay=0.002)  # drains about 16K QPS
    rep = server.serve(ex, qs, qt, arrivals, max_backlog=50)
    ok = ~rep.rejected
    assert rep.rejected.sum() > qs.size // 2
    assert np.array_equal(rep.answers[ok], fn(qs[ok], qt[ok]))
    assert np.all(np.isnan(rep.latency_s[rep.rejected])) and np.all(rep.latency_s[ok] >= 0)
    assert sum(ex.submitted) == ok.sum()
    summ = rep.summary()
    assert summ["rejected"] == int(rep.rejected.sum()) and summ["answered"] == int(ok.sum())
    # the same stream at a rate the lane keeps up with sheds nothing
    slow = np.linspace(0.0, 0.6, 200)
    rep2 = server.serve(FakeExecutor(fn, lanes=1, capacity=32, delay=0.002), qs[:200], qt[:200], slow,
                        max_backlog=50, idle_sleep=0.0005)
    assert not rep2.rejected.any() and np.array_equal(rep2.answers, fn(qs[:200], qt[:200]))


@pytest.mark.gpu
def test_gpu_server_matches_oracle_and_alone():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2410_17226_amd as P
    n, s, d = synth.rmat_edges(12, 16, seed=12)
    rp, col, _ = P.build_csr(n, s, d)
    cp, src = P.select_clusters(rp, col, P.top_degree(rp, 16), 64, 1)
    rp_d, col_d = torch.from_numpy(rp).cuda(), torch.from_numpy(col).cuda()
    dist, masks, st = P.run_batch(rp_d, col_d, cp, src, 1)
    dvm, mvm = P.labels_pack(dist, masks, 1)
    torch.cuda.synchronize()
    nv = rp.size - 1
    qs, qt = synth.query_pairs(nv, 20000, 5)
    arrivals = synth.poisson_arrivals(1e6, qs.size, 5)
    ex = server.GpuExecutor(dvm, mvm, 1, max_batch=4096, lanes=4)
    rep = server.serve(ex, qs, qt, arrivals)
    want = oracle.query_landmarks(rp, col, cp, src, qs, qt)
    assert np.array_equal(rep.answers, want)
    # the same query alone gives the same answer
    for i in range(0, qs.size, 997):
        one = P.query_batch(dvm, mvm, 1, torch.from_numpy(qs[i:i + 1]).cuda(), torch.from_numpy(qt[i:i + 1]).cuda())
        assert int(one.cpu().numpy().view(np.uint32)[0]) == int(rep.answers[i])
    # a tight memory budget admits fewer lanes and still answers the same
    ex1 = server.GpuExecutor(dvm, mvm, 1, max_batch=4096, lanes=4, memory_budget=4096 * 12)
    assert ex1.lanes == 1
    rep1 = server.serve(ex1, qs, qt, arrivals)
    assert np.array_equal(rep1.answers, want)
