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
from dataclasses import dataclass, field

import numpy as np


class GpuExecutor:
    """Lanes of device buffers and streams over device-resident labels."""

    def __init__(self, dist_vm, mask_vm, radius: int, max_batch: int = 65536, lanes: int = 4,
                 memory_budget: int | None = None):
        import torch
        from . import _binding as B
        self._torch = torch
        self._B = B
        self.dist_vm, self.mask_vm, self.radius = dist_vm, mask_vm, int(radius)
        dev = dist_vm.device
        per_lane = max_batch * (4 + 4 + 4)  # s, t, answer
        if memory_budget is not None:
            lanes = max(1, min(lanes, int(memory_budget) // per_lane))
        self.lanes = lanes
        self.capacity = max_batch
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
    answers: np.ndarray
    latency_s: np.ndarray
    batches: int
    wall_s: float
    max_in_flight: int
    batch_sizes: list = field(default_factory=list)

    def summary(self) -> dict:
        lat = self.latency_s
        return {
            "queries": int(lat.size), "batches": self.batches, "achieved_qps": float(lat.size / self.wall_s),
            "p50_us": float(np.percentile(lat, 50) * 1e6), "p99_us": float(np.percentile(lat, 99) * 1e6),
            "p999_us": float(np.percentile(lat, 99.9) * 1e6), "max_in_flight": self.max_in_flight,
            "mean_batch": float(np.mean(self.batch_sizes)) if self.batch_sizes else 0.0,
        }


def serve(executor, s: np.ndarray, t: np.ndarray, arrivals: np.ndarray, min_batch: int = 1,
          clock=time.perf_counter, idle_sleep: float = 0.0) -> ServeReport:
    """Serve requests i = (s[i], t[i]) arriving at ``arrivals[i]`` seconds
    (non-decreasing, relative to the start) with continuous batching."""
    s = np.ascontiguousarray(s, dtype=np.int32)
    t = np.ascontiguousarray(t, dtype=np.int32)
    arrivals = np.asarray(arrivals, dtype=np.float64)
    n = s.size
    answers = np.empty(n, dtype=np.uint32)
    done_at = np.empty(n, dtype=np.float64)
    lane_range = [None] * executor.lanes
    free = list(range(executor.lanes))
    next_req = 0
    batches = 0
    in_flight = 0
    max_in_flight = 0
    sizes = []
    start = clock()
    completed = 0
    while completed < n:
        now = clock() - start
        # completions
        for lane in range(executor.lanes):
            r = lane_range[lane]
            if r is not None and executor.done(lane):
                a, b = r
                answers[a:b] = executor.fetch(lane)
                done_at[a:b] = clock() - start
                completed += b - a
                lane_range[lane] = None
                free.append(lane)
                in_flight -= 1
        # admission: everything that has arrived, into free lanes
        while free and next_req < n and arrivals[next_req] <= now:
            end = int(np.searchsorted(arrivals, now, side="right"))
            end = min(end, next_req + executor.capacity, n)
            if end - next_req < min_batch and end < n and in_flight > 0:
                break  # let a little more arrive while the device is busy
            lane = free.pop()
            executor.submit(lane, s[next_req:end], t[next_req:end])
            lane_range[lane] = (next_req, end)
            sizes.append(end - next_req)
            next_req = end
            batches += 1
            in_flight += 1
            max_in_flight = max(max_in_flight, in_flight)
        if idle_sleep and in_flight == 0 and next_req < n and arrivals[next_req] > now:
            time.sleep(min(idle_sleep, arrivals[next_req] - now))
    wall = clock() - start
    return ServeReport(answers, done_at - arrivals, batches, wall, max_in_flight, sizes)
