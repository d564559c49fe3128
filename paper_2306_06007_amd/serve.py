"""Continuous-batching request loop for HVOX transforms on one GPU.

Requests (a synthesis or an analysis job on its own baselines and sky mesh)
arrive over time.  The server keeps a FIFO of arrived requests and admits the
head whenever a slot is free and its device-memory footprint fits the HBM
budget; admitted requests are planned on host worker threads (the C planner
runs without the Python GIL) and run on their own HIP stream, so the work of
several requests overlaps on the device while new ones keep arriving.
Completion is observed through a per-request event; its memory and slot are
released at once and the next requests are admitted.  Plans are cached by
geometry, so repeated requests on the same baselines and mesh reuse the
resident plan (coordinates, chunk order, tables) and skip planning.

Latency is measured from a request's arrival time to the moment its
completion is observed.
"""
from __future__ import annotations

import collections
import hashlib
import threading
import time
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

from .hvox import Plan, footprint_bound


@dataclass
class Result:
    rid: int
    direction: str
    arrival_s: float
    admit_s: float
    done_s: float
    output: object = None
    n_vis: int = 0
    n_pix: int = 0

    @property
    def latency_s(self) -> float:
        return self.done_s - self.arrival_s


def percentile(values, q):
    if len(values) == 0:
        return float("nan")
    return float(np.percentile(np.asarray(values, dtype=float), q))


# ---------------------------------------------------------------------------
# executors
# ---------------------------------------------------------------------------
class GpuExecutor:
    """Runs requests on the current GPU: one HIP stream per slot, host planning
    on worker threads, a plan cache keyed by geometry."""

    def __init__(self, eps=1e-4, dtype="f32", slots=4, planners=4, workspace_bytes=1 << 30,
                 cache_size=8, plan_opts=None):
        import torch
        self.torch = torch
        self.eps, self.dtype = eps, dtype
        self.streams = [torch.cuda.Stream() for _ in range(slots)]
        self.pool = ThreadPoolExecutor(max_workers=planners)
        self.workspace_bytes = float(workspace_bytes)
        self.plan_opts = dict(plan_opts or {})
        self.cache_size = cache_size
        self.cache = collections.OrderedDict()      # key -> Plan
        self.in_use = collections.Counter()         # key -> requests currently using the plan
        self.lock = threading.Lock()
        self.plan_seconds = []                      # host + device time of every plan built

    @property
    def slots(self):
        return len(self.streams)

    def footprint(self, req) -> float:
        return footprint_bound(req.uvw.shape[0], req.xyz.shape[0], self.dtype, self.workspace_bytes)

    @staticmethod
    def _key(req):
        h = hashlib.sha1()
        h.update(np.ascontiguousarray(req.uvw).tobytes())
        h.update(np.ascontiguousarray(req.xyz).tobytes())
        return h.hexdigest()

    def _plan(self, req, stream):
        key = self._key(req)
        with self.lock:
            plan = self.cache.get(key)
            if plan is not None:
                self.cache.move_to_end(key)
                self.in_use[key] += 1
                return key, plan
        t0 = time.perf_counter()
        plan = Plan(req.uvw, req.xyz, self.eps, self.dtype, stream=stream, workspace_bytes=self.workspace_bytes,
                    **self.plan_opts)
        with self.lock:
            self.plan_seconds.append(time.perf_counter() - t0)
        with self.lock:
            if key in self.cache:               # planned concurrently by another worker
                plan.free()
                plan = self.cache[key]
            else:
                self.cache[key] = plan
            self.in_use[key] += 1
            self._evict()
        return key, plan

    def _evict(self):
        while len(self.cache) > self.cache_size:
            victim = next((k for k in self.cache if self.in_use[k] == 0), None)
            if victim is None:
                break
            self.cache.pop(victim).free()

    def _run(self, req, slot):
        torch = self.torch
        stream = self.streams[slot]
        key, plan = self._plan(req, stream)
        cd = plan.complex_dtype
        with torch.cuda.stream(stream):
            x = torch.as_tensor(req.data).to("cuda", cd, non_blocking=False)
            out = plan.synthesis(x, stream=stream) if req.direction == "synthesis" else plan.analysis(x, stream=stream)
            ev = torch.cuda.Event()
            ev.record(stream)
        return key, out, ev

    def submit(self, req, slot):
        return self.pool.submit(self._run, req, slot)

    def done(self, handle) -> bool:
        if not handle.done():
            return False
        _, _, ev = handle.result()
        return ev.query()

    def finish(self, handle):
        key, out, ev = handle.result()
        ev.synchronize()
        res = out.cpu().numpy()
        with self.lock:
            self.in_use[key] -= 1
            self._evict()
        return res

    def close(self):
        self.pool.shutdown(wait=True)
        with self.lock:
            for p in self.cache.values():
                p.free()
            self.cache.clear()


class FakeExecutor:
    """CPU stand-in with the executor interface: a request 'runs' for a
    modelled time on a worker thread and returns the supplied function's
    result.  Used to test admission and accounting without a GPU."""

    def __init__(self, slots=2, seconds_per_term=1e-9, compute=None, footprint_per_point=64.0):
        self._slots = slots
        self.pool = ThreadPoolExecutor(max_workers=slots)
        self.seconds_per_term = seconds_per_term
        self.compute = compute
        self.footprint_per_point = footprint_per_point
        self.concurrent = 0
        self.max_concurrent = 0
        self.lock = threading.Lock()

    @property
    def slots(self):
        return self._slots

    def footprint(self, req) -> float:
        return self.footprint_per_point * (req.uvw.shape[0] + req.xyz.shape[0])

    def _run(self, req):
        with self.lock:
            self.concurrent += 1
            self.max_concurrent = max(self.max_concurrent, self.concurrent)
        time.sleep(self.seconds_per_term * req.uvw.shape[0] * req.xyz.shape[0])
        out = self.compute(req) if self.compute else None
        with self.lock:
            self.concurrent -= 1
        return out

    def submit(self, req, slot):
        return self.pool.submit(self._run, req)

    def done(self, handle) -> bool:
        return handle.done()

    def finish(self, handle):
        return handle.result()

    def close(self):
        self.pool.shutdown(wait=True)


# ---------------------------------------------------------------------------
# server
# ---------------------------------------------------------------------------
@dataclass
class Server:
    executor: object
    hbm_budget_bytes: float = 64e9
    poll_s: float = 2e-4
    log: list = field(default_factory=list)

    def run(self, requests, keep_outputs=True):
        """Replay ``requests`` (objects with rid, arrival_s, direction, uvw, xyz,
        data) in real time; return their Results in request order."""
        ex = self.executor
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival_s))
        waiting = collections.deque()
        free_slots = list(range(ex.slots))
        inflight = []                    # (req, slot, handle, footprint, admit_s)
        used = 0.0
        results = {}
        t0 = time.perf_counter()
        while pending or waiting or inflight:
            now = time.perf_counter() - t0
            progressed = False
            while pending and pending[0].arrival_s <= now:
                waiting.append(pending.popleft())
            for item in list(inflight):
                req, slot, handle, fp, admit_s = item
                if ex.done(handle):
                    out = ex.finish(handle)
                    done_s = time.perf_counter() - t0
                    inflight.remove(item)
                    free_slots.append(slot)
                    used -= fp
                    results[req.rid] = Result(req.rid, req.direction, req.arrival_s, admit_s, done_s,
                                              out if keep_outputs else None, req.uvw.shape[0], req.xyz.shape[0])
                    progressed = True
            while waiting and free_slots:
                req = waiting[0]
                fp = ex.footprint(req)
                if used + fp > self.hbm_budget_bytes and inflight:
                    break                # wait for memory to free up (FIFO: no overtaking)
                waiting.popleft()
                slot = free_slots.pop(0)
                used += fp
                admit_s = time.perf_counter() - t0
                inflight.append((req, slot, ex.submit(req, slot), fp, admit_s))
                self.log.append((admit_s, req.rid, len(inflight), used))
                progressed = True
            if not progressed:
                if pending and not waiting and not inflight:
                    time.sleep(max(0.0, min(pending[0].arrival_s - (time.perf_counter() - t0), 0.01)))
                else:
                    time.sleep(self.poll_s)
        return [results[r.rid] for r in sorted(requests, key=lambda r: r.rid)]


def summarize(results) -> dict:
    lat = [r.latency_s for r in results]
    span = max(r.done_s for r in results) - min(r.arrival_s for r in results)
    units = sum(r.n_vis + r.n_pix for r in results)
    return {"requests": len(results), "p50_latency_s": percentile(lat, 50), "p99_latency_s": percentile(lat, 99),
            "mean_latency_s": float(np.mean(lat)), "makespan_s": span,
            "throughput_vis_pix_per_s": units / span if span > 0 else float("nan")}
