"""Serving loop: many independent simulations, admitted by device-memory budget, stepped
together with continuous batching.

Requests arrive over time (Poisson arrivals).  A request is admitted as soon as it has
arrived, a batch slot is free and its workspace fits in the memory budget; its state stays
resident in device memory until it has run its steps.  Every server iteration advances all
admitted requests by one split step each, in one batched launch sequence (one captured
graph per membership), each request with its own CFL time step; requests that finish leave
and free their memory and slot, and waiting ones join at the next iteration.  The plain
mode steps each admitted request on its own (one launch sequence per request), in FP64.

Reported: per-iteration step latency (p50, p99: the time one step of every admitted request
takes), aggregate cell-updates/s over the busy time, queueing delay and completion time per
request.
"""
import time

import numpy as np

from . import cc
from . import workloads as W


class Request:
    def __init__(self, rid, work, arrival, steps):
        self.rid = rid
        self.work = work
        self.arrival = arrival
        self.steps = steps
        self.solver = None
        self.done = 0
        self.dt = None
        self.admitted = None
        self.admit_iter = None
        self.finished = None
        self.result = None


def poisson_arrivals(n, rate, seed=0):
    """Arrival times (s) of n requests with exponential gaps of mean 1/rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def make_requests(n, rate=50.0, steps=500, seed=0, first=0):
    arr = poisson_arrivals(n, rate, seed)
    return [Request(first + k, W.serving_request(first + k), float(arr[k]), steps) for k in range(n)]


def workspace_bytes(work, precision):
    """Device bytes a request holds while admitted: everything its Solver allocates."""
    return cc.Solver.device_bytes(work["grid"], work["body"], precision)


class Server:
    """mode 'batched': FP32 state (FP64 geometry) in one batch; 'plain': FP64 per request."""

    def __init__(self, mode="batched", budget_bytes=2 << 30, slots=64, keep_results=False, time_scale=1.0,
                 cfl=0.8):
        self.mode = mode
        self.cfl = cfl
        self.precision = cc.CC_FP32_GEOM64 if mode == "batched" else cc.CC_FP64
        self.budget = int(budget_bytes)
        self.slots = int(slots)
        self.keep_results = keep_results  # True, False, or a set of request ids
        self.time_scale = time_scale  # arrivals are replayed time_scale times faster
        self.batch = cc.Batch(slots, self.precision) if mode == "batched" else None
        if self.batch is not None:
            # dense tiles for many members at once: 2-row x blocks and 8-row y column walks
            # (every shape computes the same values; these gave the mix's steps a lower mean
            # and p99 latency than the defaults)
            self.batch.set_tiles(1, 5)

    def close(self):
        """Destroys the batch (every request must have been released)."""
        if self.batch is not None:
            self.batch.close()
            self.batch = None

    def _admit(self, r):
        if r.work["cfl"] != self.cfl:
            raise ValueError("every request of a server uses the server's CFL number")
        s = cc.Solver(r.work["grid"], r.work["body"], precision=self.precision)
        s.set_prim(r.work["prim"])
        r.solver = s
        r.dt = s.cfl_dt(self.cfl)
        if self.batch is not None:
            self.batch.add(s)

    def _release(self, r):
        k = self.keep_results
        if k is True or (k and r.rid in k):
            r.result = r.solver.get_u()
        if self.batch is not None:
            self.batch.remove(r.solver)
        r.solver.close()
        r.solver = None

    def run(self, requests):
        """Serves the requests to completion.  On an error every admitted request is
        released (its context leaves the batch and is destroyed) before the error
        propagates, so no device context outlives the call."""
        active = []
        try:
            return self._run(requests, active)
        except BaseException:
            for r in active:
                try:
                    self._release(r)
                except Exception:
                    pass
            raise

    def _run(self, requests, active):
        import torch
        pending = sorted(requests, key=lambda r: r.arrival)
        done = []
        used = 0
        lat = []
        peak = 0
        cell_updates = 0
        busy = 0.0
        t0 = time.perf_counter()
        while pending or active:
            now = (time.perf_counter() - t0) * self.time_scale
            # admission: arrived, a free slot, and room in the budget (arrival order)
            while pending and pending[0].arrival <= now and len(active) < self.slots:
                r = pending[0]
                need = workspace_bytes(r.work, self.precision)
                if used + need > self.budget:
                    break
                pending.pop(0)
                used += need
                r.need = need
                r.admitted = now
                r.admit_iter = len(lat)  # server iterations run before this request joined
                self._admit(r)
                active.append(r)
            if not active:
                if pending:  # idle until the next arrival
                    time.sleep(max(0.0, (pending[0].arrival - now) / self.time_scale))
                continue
            peak = max(peak, len(active))
            # one split step of every admitted request
            s0 = time.perf_counter()
            if self.batch is not None:
                self.batch.step([r.dt for r in active])
                nxt, st2 = self.batch.last_dt(self.cfl)
                for r, d, st in zip(active, nxt, st2):
                    if (st & ~1) or not (d > 0):  # bit 0 is only reported
                        raise RuntimeError(f"request {r.rid}: device status {st}")
                    r.dt = d
            else:
                for r in active:
                    r.solver.step(r.dt)
                for r in active:
                    r.dt = r.solver.cfl_dt(self.cfl)
                torch.cuda.synchronize()
            s1 = time.perf_counter()
            lat.append(s1 - s0)
            busy += s1 - s0
            for r in active:
                r.done += 1
                cell_updates += r.work["grid"]["nx"] * r.work["grid"]["ny"]
            for r in [r for r in active if r.done >= r.steps]:
                r.finished = (time.perf_counter() - t0) * self.time_scale
                self._release(r)
                used -= r.need
                active.remove(r)
                done.append(r)
        wall = time.perf_counter() - t0
        lat = np.array(lat) * 1e3
        waits = np.array([r.admitted - r.arrival for r in done])
        return {
            "mode": self.mode,
            "requests": len(done),
            "iterations": len(lat),
            "cell_updates": int(cell_updates),
            "busy_s": busy,
            "wall_s": wall,
            "cell_updates_per_s": cell_updates / busy if busy > 0 else 0.0,
            "step_latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                                "mean": float(lat.mean())},
            "queue_wait_s": {"p50": float(np.percentile(waits, 50)), "p99": float(np.percentile(waits, 99))},
            "max_concurrent": peak,
        }
