"""Continuous-batching server for s-t distance queries over Cluster-BFS labels.

Landmark-labeling queries (Section 4.2, "Answering Queries with Clustered
Landmarks") are answered by ``cbfs_query_batch`` from device-resident,
vertex-major labels.  This module is the request loop around it:

* requests arrive open-loop (each carries its scheduled arrival time);
* the server keeps ``lanes`` execution lanes, each owning a device buffer of
  ``max_batch`` queries and its own stream; the number of lanes is what the
  memory budget admits;
* whenever a lane is free, the requests that have arrived (up to
  ``max_batch``) are admitted into it as one batch: host-to-device copy, query
  kernel and device-to-host copy are enqueued on the lane's stream, and the
  loop goes on admitting new arrivals into other lanes while earlier batches
  are still on the device (continuous batching);
* admission by memory, per request: every query in flight holds
  ``bytes_per_query`` bytes of device memory (its s, t and answer), and a
  batch is admitted only while the queries in flight fit the memory budget
  (``max_in_flight_queries``); a batch that does not fit waits, or is cut to
  what fits;
* overload: an arrived request that finds ``max_backlog`` requests already
  waiting for admission is rejected at once (load shedding), flagged in
  ``ServeReport.rejected``, and gets no answer;
* a batch's completion is observed by polling its event; every request's
  latency is completion time minus scheduled arrival time.

Each answer depends only on its own (s, t) and the labels, so it is the same
whether the request runs alone or mixed with others in any batch.

The scheduling logic is independent of the device: it talks to an executor
with ``lanes``, ``capacity``, ``submit(lane, s, t)``, ``done(lane)`` and
``fetch(lane)``.  ``GpuExecutor`` is the HIP one.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np


class GpuExecutor:
    """Lanes of device buffers and streams over device-resident labels.

    ``memory_budget`` (bytes of device memory for query buffers) bounds both
    the lanes allocated (each holds ``max_batch`` queries) and, through
    ``max_in_flight_queries``, the queries the server keeps in flight."""

    bytes_per_query = 4 + 4 + 4  # s, t, answer (int32 each)

    def __init__(self, dist_vm, mask_vm, radius: int, max_batch: int = 65536, lanes: int = 4,
                 memory_budget: int | None = None):
        import torch
        from . import _binding as B
        self._torch = torch
        self._B = B
        self.dist_vm, self.mask_vm, self.radius = dist_vm, mask_vm, int(radius)
        dev = dist_vm.device
        per_lane = max_batch * self.bytes_per_query
        if memory_budget is not None:
            lanes = max(1, min(lanes, int(memory_budget) // per_lane))
        self.lanes = lanes
        self.capacity = max_batch
        self.max_in_flight_queries = lanes * max_batch if memory_budget is None else \
            max(1, min(lanes * max_batch, int(memory_budget) // self.bytes_per_query))
        self._s_h = [torch.empty(max_batch, dtype=torch.int32, pin_memory=True) for _ in range(lanes)]
        self._t_h = [torch.empty(max_batch, dtype=torch.int32, pin_memory=True) for _ in range(lanes)]
        self._a_h = [torch.empty(max_batch, dtype=torch.int32, pin_memory=True) for _ in range(lanes)]
        self._s_d = [torch.empty(max_batch, dtype=torch.int32, device=dev) for _ in range(lanes)]
        self._t_d = [torch.empty(max_batch, dtype=torch.int32, device=dev) for _ in range(lanes)]
        self._a_d = [torch.empty(max_batch, dtype=torch.int32, device=dev) for _ in range(lanes)]
        self._streams = [torch.cuda.Stream(device=dev) for _ in range(lanes)]
        self._events = [torch.cuda.Event() for _ in range(lanes)]
        self._count = [0] * lanes

    def submit(self, lane: int, s: np.ndarray, t: np.ndarray):
        torch = self._torch
        q = s.size
        self._s_h[lane][:q].numpy()[:] = s
        self._t_h[lane][:q].numpy()[:] = t
        st = self._streams[lane]
        with torch.cuda.stream(st):
            self._s_d[lane][:q].copy_(self._s_h[lane][:q], non_blocking=True)
            self._t_d[lane][:q].copy_(self._t_h[lane][:q], non_blocking=True)
            self._B.query_batch(self.dist_vm, self.mask_vm, self.radius, self._s_d[lane][:q], self._t_d[lane][:q],
                                out=self._a_d[lane][:q], stream=st)
            self._a_h[lane][:q].copy_(self._a_d[lane][:q], non_blocking=True)
            self._events[lane].record(st)
        self._count[lane] = q

    def done(self, lane: int) -> bool:
        return self._events[lane].query()

    def fetch(self, lane: int) -> np.ndarray:
        self._events[lane].synchronize()
        return self._a_h[lane][: self._count[lane]].numpy().view(np.uint32).copy()


@dataclass
class ServeReport:
    answers: np.ndarray          # uint32 per request (meaningless where rejected)
    latency_s: np.ndarray        # completion - arrival per request (nan where rejected)
    batches: int
    wall_s: float
    max_in_flight: int           # batches on the device at once
    batch_sizes: list = field(default_factory=list)
    rejected: np.ndarray | None = None    # bool per request: shed at arrival
    max_in_flight_queries: int = 0        # queries on the device at once

    def summary(self) -> dict:
        ok = ~self.rejected if self.rejected is not None else np.ones(self.latency_s.size, bool)
        lat = self.latency_s[ok]
        out = {
            "queries": int(self.latency_s.size), "answered": int(lat.size),
            "rejected": int(self.latency_s.size - lat.size), "batches": self.batches,
            "achieved_qps": float(lat.size / self.wall_s), "wall_s": float(self.wall_s),
            "max_in_flight": self.max_in_flight, "max_in_flight_queries": self.max_in_flight_queries,
            "mean_batch": float(np.mean(self.batch_sizes)) if self.batch_sizes else 0.0,
        }
        if lat.size:
            out.update({"p50_us": float(np.percentile(lat, 50) * 1e6), "p99_us": float(np.percentile(lat, 99) * 1e6),
                        "p999_us": float(np.percentile(lat, 99.9) * 1e6)})
        return out


def serve(executor, s: np.ndarray, t: np.ndarray, arrivals: np.ndarray, min_batch: int = 1,
          clock=time.perf_counter, idle_sleep: float = 0.0, max_in_flight_queries: int | None = None,
          max_backlog: int | None = None) -> ServeReport:
    """Serve requests i = (s[i], t[i]) arriving at ``arrivals[i]`` seconds
    (non-decreasing, relative to the start) with continuous batching.

    ``max_in_flight_queries`` (default: the executor's, else unlimited) is the
    memory admission limit; ``max_backlog`` (default: unlimited) is the number
    of arrived requests that may wait for admission before new arrivals are
    rejected."""
    s = np.ascontiguousarray(s, dtype=np.int32)
    t = np.ascontiguousarray(t, dtype=np.int32)
    arrivals = np.asarray(arrivals, dtype=np.float64)
    n = s.size
    if max_in_flight_queries is None:
        max_in_flight_queries = getattr(executor, "max_in_flight_queries", None)
    limit = int(max_in_flight_queries) if max_in_flight_queries else None
    answers = np.zeros(n, dtype=np.uint32)
    done_at = np.full(n, np.nan, dtype=np.float64)
    rejected = np.zeros(n, dtype=bool)
    lane_batch = [None] * executor.lanes   # request indices of the batch in each lane
    free = list(range(executor.lanes))
    backlog = deque()   # arrived, not rejected, not yet admitted: ranges [lo, hi) in arrival order
    waiting = 0         # requests in the backlog
    next_arr = 0        # next request not yet arrived
    batches = 0
    in_flight = 0
    in_flight_q = 0
    max_in_flight = 0
    max_q = 0
    sizes = []
    start = clock()
    finished = 0
    while finished < n:
        now = clock() - start
        # completions
        for lane in range(executor.lanes):
            idx = lane_batch[lane]
            if idx is not None and executor.done(lane):
                answers[idx] = executor.fetch(lane)
                done_at[idx] = clock() - start
                finished += idx.size
                in_flight_q -= idx.size
                lane_batch[lane] = None
                free.append(lane)
                in_flight -= 1
        # arrivals: join the backlog while it has room; the rest are shed
        end = int(np.searchsorted(arrivals, now, side="right"))
        if end > next_arr:
            room = end - next_arr if max_backlog is None else max(0, min(end - next_arr, max_backlog - waiting))
            if room:
                backlog.append((next_arr, next_arr + room))
                waiting += room
            if next_arr + room < end:
                rejected[next_arr + room:end] = True
                finished += end - next_arr - room
            next_arr = end
        # admission: the backlog, into free lanes, as memory allows
        while free and waiting:
            room = executor.capacity if limit is None else min(executor.capacity, limit - in_flight_q)
            if room <= 0:
                break  # the in-flight queries hold the whole budget
            take = min(room, waiting)
            if take < min_batch and next_arr < n and in_flight > 0:
                break  # let a little more arrive while the device is busy
            parts, got = [], 0
            while got < take:
                lo, hi = backlog[0]
                k = min(hi - lo, take - got)
                parts.append(np.arange(lo, lo + k, dtype=np.int64))
                got += k
                if lo + k == hi:
                    backlog.popleft()
                else:
                    backlog[0] = (lo + k, hi)
            idx = parts[0] if len(parts) == 1 else np.concatenate(parts)
            waiting -= take
            lane = free.pop()
            executor.submit(lane, s[idx], t[idx])
            lane_batch[lane] = idx
            sizes.append(take)
            batches += 1
            in_flight += 1
            in_flight_q += take
            max_in_flight = max(max_in_flight, in_flight)
            max_q = max(max_q, in_flight_q)
        if idle_sleep and in_flight == 0 and not waiting and next_arr < n and arrivals[next_arr] > now:
            time.sleep(min(idle_sleep, arrivals[next_arr] - now))
    wall = clock() - start
    return ServeReport(answers, done_at - arrivals, batches, wall, max_in_flight, sizes, rejected, max_q)
