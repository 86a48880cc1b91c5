"""Serving: continuous batching of gridding / degridding jobs on one GPU.

Jobs of uneven visibility counts and grid sizes arrive at any time.  The
request loop admits them in arrival order as execution slots (one HIP
stream and host thread each) and HBM budget free up, so jobs that arrive
while others are on the GPU start as soon as they fit and their kernels
overlap on the device.  CF tables (the CFCache of the PreCompute
component) stay resident between jobs and are evicted least recently used
when the budget binds.  Latency is measured from arrival to completion
(results back on the host); stats() reports throughput with p50 / p99.

`Scheduler` holds the admission logic only (no threads, no GPU) so that it
can be driven by a simulated clock; `Server` runs it with threads and an
executor (the GPU one by default).
"""

import collections
import threading
import time
from concurrent.futures import Future
from dataclasses import dataclass, field
from typing import Any, Callable, Optional

import numpy as np


@dataclass
class Job:
    """One request.  `cf_key` names the CF table the job needs (jobs with
    equal keys share it); `cf_bytes` is that table's size; `bytes` is the
    job's own device footprint (data, grid, plan, scratch)."""
    job_id: int
    op: str                      # "grid" | "degrid"
    cf_key: Any
    bytes: int
    cf_bytes: int
    payload: Any = None          # executor-specific inputs
    n_vis: int = 0
    t_arrival: float = 0.0
    t_admit: Optional[float] = None
    t_done: Optional[float] = None
    slot: Optional[int] = None
    error: Optional[str] = None
    result: Any = None
    cf_cold: bool = False        # this job brought its CF into residency


class Scheduler:
    """Admission by HBM footprint in arrival order, slot accounting and CF
    residency.  All methods are called with the caller's clock."""

    def __init__(self, hbm_budget, n_slots):
        self.budget = int(hbm_budget)
        self.free_slots = list(range(n_slots))
        self.queue = collections.deque()
        self.running = {}
        self.used = 0
        self.peak_used = 0
        self.cf = collections.OrderedDict()     # key -> [bytes, refs]  (LRU order)
        self.done = []
        self.rejected = []

    def submit(self, job, now):
        job.t_arrival = now if job.t_arrival is None else job.t_arrival
        need = job.bytes + job.cf_bytes
        if need > self.budget:
            job.error = "job needs %d bytes, budget is %d" % (need, self.budget)
            job.t_done = now
            self.rejected.append(job)
            return False
        self.queue.append(job)
        return True

    def _cf_need(self, job):
        return 0 if job.cf_key in self.cf else job.cf_bytes

    def _evict_for(self, need):
        """Drop unreferenced CFs, least recently used first, until `need`
        bytes fit; returns True when they do."""
        for key in list(self.cf.keys()):
            if self.used + need <= self.budget:
                break
            b, refs = self.cf[key]
            if refs == 0:
                del self.cf[key]
                self.used -= b
        return self.used + need <= self.budget

    def admit(self, now):
        """Admit queued jobs in arrival order while a slot is free and the
        head job fits (after evicting idle CFs).  Returns [(job, new_cf)]."""
        out = []
        while self.queue and self.free_slots:
            job = self.queue[0]
            need = job.bytes + self._cf_need(job)
            if self.used + need > self.budget and not self._evict_for(need):
                break
            self.queue.popleft()
            new_cf = job.cf_key not in self.cf
            if new_cf:
                self.cf[job.cf_key] = [job.cf_bytes, 0]
                self.used += job.cf_bytes
            self.cf[job.cf_key][1] += 1
            self.cf.move_to_end(job.cf_key)
            self.used += job.bytes
            self.peak_used = max(self.peak_used, self.used)
            job.slot = self.free_slots.pop(0)
            job.t_admit = now
            self.running[job.job_id] = job
            out.append((job, new_cf))
        return out

    def complete(self, job, now, error=None):
        self.running.pop(job.job_id)
        self.used -= job.bytes
        ent = self.cf.get(job.cf_key)
        if ent is not None:
            ent[1] -= 1
        self.free_slots.append(job.slot)
        self.free_slots.sort()
        job.t_done = now
        job.error = error
        self.done.append(job)

    def drop_cf(self, key):
        """Forget a CF whose build failed (no references may remain)."""
        ent = self.cf.get(key)
        if ent is not None and ent[1] == 0:
            self.used -= ent[0]
            del self.cf[key]

    def idle(self):
        return not self.queue and not self.running


def latency_stats(jobs, t0=None, t1=None):
    ok = [j for j in jobs if j.error is None and j.t_done is not None]
    lat = np.array([j.t_done - j.t_arrival for j in ok]) if ok else np.zeros(0)
    nvis = sum(j.n_vis for j in ok)
    if t0 is None:
        t0 = min((j.t_arrival for j in jobs), default=0.0)
    if t1 is None:
        t1 = max((j.t_done for j in ok), default=t0)
    span = max(t1 - t0, 1e-12)
    return {
        "jobs_done": len(ok),
        "jobs_failed": sum(1 for j in jobs if j.error is not None),
        "p50_s": float(np.percentile(lat, 50)) if lat.size else None,
        "p99_s": float(np.percentile(lat, 99)) if lat.size else None,
        "mean_s": float(lat.mean()) if lat.size else None,
        "throughput_vis_per_s": nvis / span,
        "throughput_jobs_per_s": len(ok) / span,
        "span_s": span,
    }


class Server:
    """Threaded request loop around Scheduler.

    executor: object with run(job, slot) -> result and prepare_cf(job, slot)
    (called once when a job brings a CF into residency, on that job's slot,
    before run) and release_cf(key).  Exceptions fail only the job that
    raised them."""

    def __init__(self, executor, hbm_budget, n_slots=4, clock=time.perf_counter):
        self.exe = executor
        self.sched = Scheduler(hbm_budget, n_slots)
        self.clock = clock
        self.lock = threading.Condition()
        self.futures = {}
        self.cf_ready = {}          # key -> threading.Event
        self.stop = False
        self.slot_q = [collections.deque() for _ in range(n_slots)]
        self.threads = [threading.Thread(target=self._slot_loop, args=(i,), daemon=True)
                        for i in range(n_slots)]
        self.loop = threading.Thread(target=self._request_loop, daemon=True)
        for t in self.threads:
            t.start()
        self.loop.start()

    # -- API -------------------------------------------------------------
    def submit(self, job):
        fut = Future()
        with self.lock:
            job.t_arrival = self.clock()
            self.futures[job.job_id] = fut
            if not self.sched.submit(job, job.t_arrival):
                fut.set_exception(RuntimeError(job.error))
            self.lock.notify_all()
        return fut

    def drain(self, timeout=None):
        t_end = None if timeout is None else time.time() + timeout
        with self.lock:
            while not self.sched.idle():
                left = None if t_end is None else t_end - time.time()
                if left is not None and left <= 0:
                    raise TimeoutError("server did not drain")
                self.lock.wait(timeout=left if left is not None else 1.0)

    def close(self):
        with self.lock:
            self.stop = True
            self.lock.notify_all()
        self.loop.join()
        for t in self.threads:
            t.join()

    def stats(self):
        with self.lock:
            jobs = list(self.sched.done) + list(self.sched.rejected)
            s = latency_stats(jobs)
            cold = [j for j in jobs if j.cf_cold]
            warm = [j for j in jobs if not j.cf_cold]
            s["cold"] = {k: latency_stats(cold)[k] for k in ("jobs_done", "p50_s", "p99_s")}
            s["warm"] = {k: latency_stats(warm)[k] for k in ("jobs_done", "p50_s", "p99_s")}
            s["peak_hbm_bytes"] = self.sched.peak_used
            s["hbm_budget"] = self.sched.budget
            s["resident_cfs"] = len(self.sched.cf)
            return s

    # -- internals -------------------------------------------------------
    def _request_loop(self):
        with self.lock:
            while not self.stop:
                for job, new_cf in self.sched.admit(self.clock()):
                    job.cf_cold = new_cf
                    if new_cf:
                        self.cf_ready[job.cf_key] = threading.Event()
                    self.slot_q[job.slot].append((job, new_cf))
                self.lock.notify_all()
                self.lock.wait(timeout=0.05)

    def _slot_loop(self, i):
        while True:
            with self.lock:
                while not self.slot_q[i] and not self.stop:
                    self.lock.wait(timeout=0.05)
                if self.stop and not self.slot_q[i]:
                    return
                job, new_cf = self.slot_q[i].popleft()
                ready = self.cf_ready.get(job.cf_key)
            err = None
            try:
                if new_cf:
                    try:
                        self.exe.prepare_cf(job, i)
                    finally:
                        ready.set()
                else:
                    ready.wait()
                    if not self.exe.has_cf(job.cf_key):
                        raise RuntimeError("CF %r is not available" % (job.cf_key,))
                job.result = self.exe.run(job, i)
            except Exception as e:      # fail this job only
                err = "%s: %s" % (type(e).__name__, e)
            with self.lock:
                self.sched.complete(job, self.clock(), err)
                if err and new_cf and not self.exe.has_cf(job.cf_key):
                    self.sched.drop_cf(job.cf_key)
                for key in [k for k in list(self.cf_ready) if k not in self.sched.cf]:
                    self.cf_ready.pop(key, None)
                    self.exe.release_cf(key)
                fut = self.futures.pop(job.job_id)
                self.lock.notify_all()
            if err:
                fut.set_exception(RuntimeError(err))
            else:
                fut.set_result(job)


class GPUExecutor:
    """Runs jobs with the gfx950 library, one torch stream per slot.

    Job payload: dict(grid_spec, cf_spec, uvw, freq, chan_plane, vis,
    weight, grid) with host numpy arrays; results come back as host arrays
    (the grid for "grid" jobs, the visibilities for "degrid" jobs)."""

    def __init__(self, n_slots, precision, device="cuda"):
        import torch
        from . import lr
        self.torch, self.lr = torch, lr
        self.p = precision
        self.dev = device
        self.streams = [torch.cuda.Stream(device=device) for _ in range(n_slots)]
        self.cfs = {}
        self.cf_events = {}
        self.cplx = torch.complex128 if precision == lr.LR_F64 else torch.complex64
        self.real = torch.float64 if precision == lr.LR_F64 else torch.float32

    def has_cf(self, key):
        return key in self.cfs

    def prepare_cf(self, job, slot):
        torch, lr = self.torch, self.lr
        pl = job.payload
        s = self.streams[slot]
        with torch.cuda.stream(s):
            cf = lr.CF(pl["grid_spec"], dict(pl["cf_spec"]), device=self.dev, stream=s)
            ev = torch.cuda.Event()
            ev.record(s)
        self.cfs[job.cf_key] = cf
        self.cf_events[job.cf_key] = ev

    def release_cf(self, key):
        self.cfs.pop(key, None)
        self.cf_events.pop(key, None)

    def run(self, job, slot):
        torch, lr = self.torch, self.lr
        pl = job.payload
        s = self.streams[slot]
        cf = self.cfs[job.cf_key]
        with torch.cuda.stream(s):
            s.wait_event(self.cf_events[job.cf_key])
            uvw = torch.as_tensor(pl["uvw"]).to(self.dev, non_blocking=True)
            wt = torch.as_tensor(pl["weight"]).to(self.dev, dtype=self.real, non_blocking=True)
            g = pl["grid_spec"]
            v = lr.Vis(uvw, pl["freq"], pl["chan_plane"], None, weight=wt, npol=g.npol)
            if job.op == "grid":
                v.vis = torch.as_tensor(pl["vis"]).to(self.dev, dtype=self.cplx, non_blocking=True)
                grid = torch.empty((g.nplane, g.npol, g.ny, g.nx), dtype=self.cplx,
                                   device=self.dev)
                lr.lr_grid_overwrite(cf, v, self.p, grid, stream=s)
                out = grid.cpu()
            else:
                grid = torch.as_tensor(pl["grid"]).to(self.dev, dtype=self.cplx,
                                                      non_blocking=True)
                v.vis = torch.empty(tuple(pl["weight"].shape), dtype=self.cplx, device=self.dev)
                lr.lr_degrid(cf, v, self.p, grid, stream=s)
                out = v.vis.cpu()
            s.synchronize()
        return out.numpy()


def job_bytes(nrow, nchan, npol, n_grid, precision_bytes=8):
    """Device footprint of one job: uvw, visibilities, weights, grid, the
    binning plan and the presum scratch (an upper bound)."""
    pairs = nrow * nchan
    vis = pairs * npol * precision_bytes
    wt = pairs * npol * precision_bytes // 2
    grid = n_grid * n_grid * npol * precision_bytes
    plan = pairs * 160 + (1 << 20)
    scratch = pairs * npol * precision_bytes
    return int(24 * nrow + 2 * vis + wt + grid + plan + scratch)


def cf_bytes(n_w, h_min, h_max, O, elem_bytes=8, n_fg=1):
    h = [h_min + (2 * (h_max - h_min) * k + n_w - 1) // (2 * (n_w - 1)) for k in range(n_w)] \
        if n_w > 1 else [h_min]
    return int(n_fg * sum((O + 1) ** 2 * (2 * x + 1) ** 2 for x in h) * elem_bytes + 65536)
