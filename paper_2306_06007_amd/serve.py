"""Continuous-batching request loop for HVOX transforms on one GPU.

Requests (a synthesis or an analysis job on its own baselines and sky mesh)
arrive over time.  Every arrival is planned at once on a host worker thread
(the C planner runs without the Python GIL and without device memory: a
host-only plan, whose ``device_bytes`` is the memory its device part will
hold).  The server keeps a FIFO of arrived requests and admits the head as
soon as it is planned, a slot is free and its plan fits the HBM budget next to
the plans already resident (idle cached plans are evicted to make room); the
admitted request's plan is uploaded if it is not resident, and the call runs
on the slot's own HIP stream, so the work of several requests overlaps on the
device while new ones keep arriving.  Completion is observed through a
per-request event; its slot is released at once and the next requests are
admitted.  Plans are cached by geometry, so repeated requests on the same
baselines and mesh reuse the resident plan (coordinates, chunk order,
tables).  A plan owns one workspace, so calls on one plan are serialised: a
call waits (on the device) for the previous call on the same plan, whatever
slot made it.  Plan memory comes from PyTorch's caching allocator through the
library's allocation hooks, so steady-state serving makes no hipMalloc /
hipFree calls.

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

from .hvox import Plan


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
@dataclass
class _Entry:
    """A cached plan: host part first, device part once admitted."""
    plan: object = None
    planning: object = None          # Future of the host planning
    bytes: float = 0.0               # device bytes (bound before the upload, exact after)
    on_device: bool = False          # device part exists, or memory is reserved for it
    users: int = 0                   # admitted requests not yet finished
    lock: threading.Lock = field(default_factory=threading.Lock)
    last_event: object = None        # event after the last call enqueued on the plan


class GpuExecutor:
    """Runs requests on the current GPU: one HIP stream per slot, host planning
    on worker threads, admission by the plans' device bytes, a plan cache keyed
    by geometry."""

    def __init__(self, eps=1e-4, dtype="f32", slots=4, planners=4, workspace_bytes=1 << 30,
                 cache_size=8, plan_opts=None, deterministic=False):
        import torch
        self.torch = torch
        self.eps, self.dtype = eps, dtype
        self.streams = [torch.cuda.Stream() for _ in range(slots)]
        self.pool = ThreadPoolExecutor(max_workers=planners)
        self.workspace_bytes = float(workspace_bytes)
        self.plan_opts = dict(plan_opts or {})
        self.deterministic = deterministic
        self.cache_size = cache_size
        self.entries = collections.OrderedDict()     # key -> _Entry
        self.lock = threading.Lock()
        self.plan_seconds = []                       # host planning time of every plan built
        self.upload_seconds = []                     # device part of every plan uploaded
        self.evictions = 0

    @property
    def slots(self):
        return len(self.streams)

    @staticmethod
    def _key(req):
        h = hashlib.sha1()
        h.update(np.ascontiguousarray(req.uvw).tobytes())
        h.update(np.ascontiguousarray(req.xyz).tobytes())
        return h.hexdigest()

    def _host_plan(self, req):
        t0 = time.perf_counter()
        plan = Plan(req.uvw, req.xyz, self.eps, self.dtype, host_only=True, workspace_bytes=self.workspace_bytes,
                    deterministic=self.deterministic, **self.plan_opts)
        with self.lock:
            self.plan_seconds.append(time.perf_counter() - t0)
        return plan

    # -- the server's interface
    def prepare(self, req):
        """Start host planning of the request's plan (shared by requests of one
        geometry); returns the token the other calls take."""
        key = self._key(req)
        with self.lock:
            e = self.entries.get(key)
            if e is None:
                e = _Entry()
                e.planning = self.pool.submit(self._host_plan, req)
                self.entries[key] = e
            e.users += 1             # held from arrival: a planned entry is never evicted under a request
        return key

    def prepared(self, key) -> bool:
        return self.entries[key].planning.done()

    def _bytes(self, e):
        if e.plan is None:
            e.plan = e.planning.result()
            e.bytes = float(e.plan.info()["device_bytes"])
        return e.bytes

    def resident_bytes(self) -> float:
        with self.lock:
            return sum(e.bytes for e in self.entries.values() if e.on_device)

    def admit(self, key, budget, force=False) -> bool:
        """Reserve device memory for the request's plan unless it is resident:
        idle cached plans are evicted (least recently used first) until the
        resident plans plus this one fit ``budget``; ``force`` admits anyway
        (nothing else is in flight, so it would never fit otherwise)."""
        with self.lock:
            e = self.entries[key]
            self.entries.move_to_end(key)
            need = self._bytes(e)
            if e.on_device:
                return True
            resident = sum(x.bytes for x in self.entries.values() if x.on_device)
            for k in list(self.entries):
                if resident + need <= budget:
                    break
                x = self.entries[k]
                if x.on_device and x.users == 0 and k != key:
                    resident -= x.bytes
                    self._drop(k)
            if resident + need > budget and not force:
                return False
            e.on_device = True
            return True

    def _drop(self, key):
        x = self.entries.pop(key)
        if x.plan is not None:
            x.plan.free()
        self.evictions += 1

    def _run(self, key, req, slot):
        torch = self.torch
        stream = self.streams[slot]
        e = self.entries[key]
        with e.lock:                                 # one host-side enqueue at a time per plan
            plan = e.plan
            if plan.host_only:
                t0 = time.perf_counter()
                plan.upload(stream=stream)
                with self.lock:
                    self.upload_seconds.append(time.perf_counter() - t0)
                    e.bytes = float(plan.info()["device_bytes"])
            with torch.cuda.stream(stream):
                x = torch.as_tensor(req.data).to("cuda", plan.complex_dtype, non_blocking=False)
                if e.last_event is not None:
                    stream.wait_event(e.last_event)  # the previous call on this plan, on any stream
                out = (plan.synthesis(x, stream=stream) if req.direction == "synthesis"
                       else plan.analysis(x, stream=stream))
                ev = torch.cuda.Event()
                ev.record(stream)
            e.last_event = ev
        return key, out, ev

    def submit(self, key, req, slot):
        return self.pool.submit(self._run, key, req, slot)

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
            self.entries[key].users -= 1
            self._trim()
        return res

    def _trim(self):
        # keep at most cache_size idle resident plans
        idle = [k for k, x in self.entries.items() if x.users == 0]
        for k in idle[:max(0, len(idle) - self.cache_size)]:
            self._drop(k)

    def close(self):
        self.pool.shutdown(wait=True)
        with self.lock:
            for x in self.entries.values():
                if x.plan is None and x.planning is not None:
                    x.plan = x.planning.result()
                if x.plan is not None:
                    x.plan.free()
            self.entries.clear()


class FakeExecutor:
    """CPU stand-in with the executor interface: a request 'runs' for a
    modelled time on a worker thread and returns the supplied function's
    result; its footprint is a modelled number of bytes per point.  Used to
    test admission and accounting without a GPU."""

    def __init__(self, slots=2, seconds_per_term=1e-9, compute=None, footprint_per_point=64.0):
        self._slots = slots
        self.pool = ThreadPoolExecutor(max_workers=slots)
        self.seconds_per_term = seconds_per_term
        self.compute = compute
        self.footprint_per_point = footprint_per_point
        self.concurrent = 0
        self.max_concurrent = 0
        self.used = 0.0
        self.reqs = {}
        self.lock = threading.Lock()

    @property
    def slots(self):
        return self._slots

    def prepare(self, req):
        self.reqs[req.rid] = req
        return req.rid

    def prepared(self, key) -> bool:
        return True

    def footprint(self, req) -> float:
        return self.footprint_per_point * (req.uvw.shape[0] + req.xyz.shape[0])

    def resident_bytes(self) -> float:
        return self.used

    def admit(self, key, budget, force=False) -> bool:
        fp = self.footprint(self.reqs[key])
        if self.used + fp > budget and not force:
            return False
        self.used += fp
        return True

    def _run(self, req):
        with self.lock:
            self.concurrent += 1
            self.max_concurrent = max(self.max_concurrent, self.concurrent)
        time.sleep(self.seconds_per_term * req.uvw.shape[0] * req.xyz.shape[0])
        out = self.compute(req) if self.compute else None
        with self.lock:
            self.concurrent -= 1
        return req.rid, out

    def submit(self, key, req, slot):
        return self.pool.submit(self._run, req)

    def done(self, handle) -> bool:
        return handle.done()

    def finish(self, handle):
        rid, out = handle.result()
        self.used -= self.footprint(self.reqs[rid])
        return out

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
        data) in real time; return their Results in request order.  The log
        records (admit time, rid, requests in flight, resident device bytes)
        at every admission."""
        ex = self.executor
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival_s))
        waiting = collections.deque()    # (req, token): arrived, planning started, not admitted
        free_slots = list(range(ex.slots))
        inflight = []                    # (req, slot, handle, admit_s)
        results = {}
        t0 = time.perf_counter()
        while pending or waiting or inflight:
            now = time.perf_counter() - t0
            progressed = False
            while pending and pending[0].arrival_s <= now:
                req = pending.popleft()
                waiting.append((req, ex.prepare(req)))
            for item in list(inflight):
                req, slot, handle, admit_s = item
                if ex.done(handle):
                    out = ex.finish(handle)
                    done_s = time.perf_counter() - t0
                    inflight.remove(item)
                    free_slots.append(slot)
                    results[req.rid] = Result(req.rid, req.direction, req.arrival_s, admit_s, done_s,
                                              out if keep_outputs else None, req.uvw.shape[0], req.xyz.shape[0])
                    progressed = True
            while waiting and free_slots:
                req, tok = waiting[0]
                if not ex.prepared(tok):
                    break                # FIFO: the head is still being planned
                if not ex.admit(tok, self.hbm_budget_bytes, force=not inflight):
                    break                # wait for memory to free up (no overtaking)
                waiting.popleft()
                slot = free_slots.pop(0)
                admit_s = time.perf_counter() - t0
                inflight.append((req, slot, ex.submit(tok, req, slot), admit_s))
                self.log.append((admit_s, req.rid, len(inflight), ex.resident_bytes()))
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
