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
    equal keys share it); `cf_bytes` is that table's size and
    `cf_build_bytes` the transient scratch its build takes (charged to the
    job that brings the table in).  A degrid job names the model grid it
    reads with `model_key` (jobs with equal keys share one resident copy)
    and its size `model_bytes`.  `bytes` is the job's own device footprint
    (data, output, plan, scratch)."""
    job_id: int
    op: str                      # "grid" | "degrid"
    cf_key: Any
    bytes: int
    cf_bytes: int
    payload: Any = None          # executor-specific inputs
    n_vis: int = 0
    t_arrival: float = 0.0
    model_key: Any = None
    model_bytes: int = 0
    cf_build_bytes: int = 0
    t_admit: Optional[float] = None
    t_done: Optional[float] = None
    slot: Optional[int] = None
    error: Optional[str] = None
    result: Any = None
    cf_cold: bool = False        # this job brought its CF into residency
    model_cold: bool = False     # this job brought its model grid into residency
    charged: int = 0             # bytes charged to the job itself while it runs


class Scheduler:
    """Admission by HBM footprint in arrival order, slot accounting and the
    residency of shared device objects (CF tables and model grids), which
    stay resident while idle and are evicted least recently used when the
    budget binds.  All methods are called with the caller's clock."""

    def __init__(self, hbm_budget, n_slots):
        self.budget = int(hbm_budget)
        self.free_slots = list(range(n_slots))
        self.queue = collections.deque()
        self.running = {}
        self.used = 0
        self.peak_used = 0
        self.res = collections.OrderedDict()    # (kind, key) -> [bytes, refs]  (LRU order)
        self.evicted = []                       # (kind, key) dropped since the last take
        self.done = []
        self.rejected = []

    @property
    def cf(self):
        return {k[1]: v for k, v in self.res.items() if k[0] == "cf"}

    @property
    def models(self):
        return {k[1]: v for k, v in self.res.items() if k[0] == "model"}

    @staticmethod
    def resources(job):
        r = [(("cf", job.cf_key), job.cf_bytes)]
        if job.model_key is not None:
            r.append((("model", job.model_key), job.model_bytes))
        return r

    def _charge(self, job, new):
        return job.bytes + (job.cf_build_bytes if ("cf", job.cf_key) in new else 0)

    def submit(self, job, now):
        job.t_arrival = now if job.t_arrival is None else job.t_arrival
        need = job.bytes + job.cf_build_bytes + sum(b for _, b in self.resources(job))
        if need > self.budget:
            job.error = "job needs %d bytes, budget is %d" % (need, self.budget)
            job.t_done = now
            self.rejected.append(job)
            return False
        self.queue.append(job)
        return True

    def _evict_for(self, need, keep):
        """Drop idle resources other than `keep`, least recently used first,
        until `need` more bytes fit; returns True when they do."""
        for key in list(self.res.keys()):
            if self.used + need <= self.budget:
                break
            b, refs = self.res[key]
            if refs == 0 and key not in keep:
                del self.res[key]
                self.used -= b
                self.evicted.append(key)
        return self.used + need <= self.budget

    def take_evicted(self):
        out, self.evicted = self.evicted, []
        return out

    def admit(self, now):
        """Admit queued jobs in arrival order while a slot is free and the
        head job fits (after evicting idle resources).  Returns [(job,
        new_cf)]; job.model_cold tells whether its model grid is new."""
        out = []
        while self.queue and self.free_slots:
            job = self.queue[0]
            res = self.resources(job)
            new = {k for k, _ in res if k not in self.res}
            need = self._charge(job, new) + sum(b for k, b in res if k in new)
            if self.used + need > self.budget and not self._evict_for(need, {k for k, _ in res}):
                break
            self.queue.popleft()
            for k, b in res:
                if k in new:
                    self.res[k] = [b, 0]
                    self.used += b
                self.res[k][1] += 1
                self.res.move_to_end(k)
            job.charged = self._charge(job, new)
            self.used += job.charged
            self.peak_used = max(self.peak_used, self.used)
            job.slot = self.free_slots.pop(0)
            job.t_admit = now
            job.model_cold = ("model", job.model_key) in new
            self.running[job.job_id] = job
            out.append((job, ("cf", job.cf_key) in new))
        return out

    def complete(self, job, now, error=None):
        self.running.pop(job.job_id)
        self.used -= job.charged
        for k, _ in self.resources(job):
            ent = self.res.get(k)
            if ent is not None:
                ent[1] -= 1
        self.free_slots.append(job.slot)
        self.free_slots.sort()
        job.t_done = now
        job.error = error
        self.done.append(job)

    def drop(self, kind, key):
        """Forget a resource whose preparation failed (no references may
        remain)."""
        ent = self.res.get((kind, key))
        if ent is not None and ent[1] == 0:
            self.used -= ent[0]
            del self.res[(kind, key)]

    def drop_cf(self, key):
        self.drop("cf", key)

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

    executor: object with run(job, slot) -> result, prepare_cf(job, slot)
    (called once when a job brings a CF into residency, on that job's slot,
    before run), has_cf(key) and release_cf(key); for jobs with a model
    grid also prepare_model(job, slot), has_model(key) and
    release_model(key).  Exceptions fail only the job that raised them."""

    def __init__(self, executor, hbm_budget, n_slots=4, clock=time.perf_counter):
        self.exe = executor
        self.sched = Scheduler(hbm_budget, n_slots)
        self.clock = clock
        self.lock = threading.Condition()
        self.futures = {}
        self.ready = {}             # (kind, key) -> threading.Event
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
            s["resident_models"] = len(self.sched.models)
            s["model_uploads"] = sum(1 for j in jobs if j.model_cold)
            errs = collections.Counter(j.error[:160] for j in jobs if j.error is not None)
            s["errors"] = dict(errs.most_common(5))
            waits = [j.t_admit - j.t_arrival for j in jobs if j.t_admit is not None]
            s["admission_wait_p50_s"] = float(np.percentile(waits, 50)) if waits else None
            s["admission_wait_p99_s"] = float(np.percentile(waits, 99)) if waits else None
            return s

    # -- internals -------------------------------------------------------
    def _release(self, keys):
        for kind, key in keys:
            self.ready.pop((kind, key), None)
            if kind == "cf":
                self.exe.release_cf(key)
            else:
                self.exe.release_model(key)

    def _request_loop(self):
        with self.lock:
            while not self.stop:
                admitted = self.sched.admit(self.clock())
                # evictions first: a key evicted and brought back within the
                # same batch keeps the event its new preparation registers
                self._release(self.sched.take_evicted())
                for job, new_cf in admitted:
                    job.cf_cold = new_cf
                    if new_cf:
                        self.ready[("cf", job.cf_key)] = threading.Event()
                    if job.model_cold:
                        self.ready[("model", job.model_key)] = threading.Event()
                    self.slot_q[job.slot].append((job, new_cf))
                self.lock.notify_all()
                self.lock.wait(timeout=0.05)

    def _prepare(self, kind, key, fresh, make, present):
        """Make (fresh) or wait for (shared) one resident resource."""
        ev = self.ready.get((kind, key))
        if fresh:
            try:
                make()
            finally:
                ev.set()
        else:
            ev.wait()
            if not present(key):
                raise RuntimeError("%s %r is not available" % (kind, key))

    def _slot_loop(self, i):
        while True:
            with self.lock:
                while not self.slot_q[i] and not self.stop:
                    self.lock.wait(timeout=0.05)
                if self.stop and not self.slot_q[i]:
                    return
                job, new_cf = self.slot_q[i].popleft()
            err = None
            try:
                self._prepare("cf", job.cf_key, new_cf, lambda: self.exe.prepare_cf(job, i),
                              self.exe.has_cf)
                if job.model_key is not None:
                    self._prepare("model", job.model_key, job.model_cold,
                                  lambda: self.exe.prepare_model(job, i), self.exe.has_model)
                job.result = self.exe.run(job, i)
            except Exception as e:      # fail this job only
                err = "%s: %s" % (type(e).__name__, e)
            with self.lock:
                self.sched.complete(job, self.clock(), err)
                if err:
                    if new_cf and not self.exe.has_cf(job.cf_key):
                        self.sched.drop("cf", job.cf_key)
                        self._release([("cf", job.cf_key)])
                    if job.model_cold and not self.exe.has_model(job.model_key):
                        self.sched.drop("model", job.model_key)
                        self._release([("model", job.model_key)])
                fut = self.futures.pop(job.job_id)
                self.lock.notify_all()
            if err:
                fut.set_exception(RuntimeError(err))
            else:
                fut.set_result(job)


class GPUExecutor:
    """Runs jobs with the gfx950 library, one torch stream per slot.

    Job payload: dict(grid_spec, cf_spec, uvw, freq, chan_plane, vis,
    weight, grid): host arrays in the device's element types, best as
    tensors in pinned memory, so that the host-to-device copies run on the
    slot's stream beside other slots' kernels.  A degrid job with a
    model_key reads the resident copy of its model grid, uploaded once from
    payload['grid'] by the job that brings it in; without one it uploads
    payload['grid'] itself.  Results come back as host arrays (grid jobs:
    the grid; degrid jobs: the visibilities) through pinned memory."""

    def __init__(self, n_slots, precision, device="cuda"):
        import torch
        from . import lr
        self.torch, self.lr = torch, lr
        self.p = precision
        self.dev = device
        self.streams = [torch.cuda.Stream(device=device) for _ in range(n_slots)]
        self.cfs = {}
        self.cf_events = {}
        self.models = {}
        self.model_events = {}
        self.cplx = torch.complex128 if precision == lr.LR_F64 else torch.complex64
        self.real = torch.float64 if precision == lr.LR_F64 else torch.float32

    def has_cf(self, key):
        return key in self.cfs

    def has_model(self, key):
        return key in self.models

    def _dev(self, a, dtype):
        t = a if isinstance(a, self.torch.Tensor) else self.torch.as_tensor(a)
        return t.to(self.dev, dtype=dtype, non_blocking=True)

    def prepare_cf(self, job, slot):
        torch, lr = self.torch, self.lr
        pl = job.payload
        s = self.streams[slot]
        with torch.cuda.stream(s):
            cf = lr.CF(pl["grid_spec"], dict(pl["cf_spec"]), device=self.dev, stream=s)
            ev = torch.cuda.Event()
            ev.record(s)
        # the build's scratch goes back once the build has run: only the
        # table stays resident
        ev.synchronize()
        cf._work = None
        self.cfs[job.cf_key] = cf
        self.cf_events[job.cf_key] = ev

    def release_cf(self, key):
        self.cfs.pop(key, None)
        self.cf_events.pop(key, None)

    def prepare_model(self, job, slot):
        torch = self.torch
        s = self.streams[slot]
        with torch.cuda.stream(s):
            g = self._dev(job.payload["grid"], self.cplx)
            ev = torch.cuda.Event()
            ev.record(s)
        self.models[job.model_key] = g
        self.model_events[job.model_key] = ev

    def release_model(self, key):
        self.models.pop(key, None)
        self.model_events.pop(key, None)

    def run(self, job, slot):
        torch, lr = self.torch, self.lr
        pl = job.payload
        s = self.streams[slot]
        cf = self.cfs[job.cf_key]
        with torch.cuda.stream(s):
            s.wait_event(self.cf_events[job.cf_key])
            uvw = self._dev(pl["uvw"], torch.float64)
            wt = self._dev(pl["weight"], self.real)
            g = pl["grid_spec"]
            v = lr.Vis(uvw, pl["freq"], pl["chan_plane"], None, weight=wt, npol=g.npol)
            if job.op == "grid":
                v.vis = self._dev(pl["vis"], self.cplx)
                grid = torch.empty((g.nplane, g.npol, g.ny, g.nx), dtype=self.cplx,
                                   device=self.dev)
                lr.lr_grid_overwrite(cf, v, self.p, grid, stream=s)
                dev_out = grid
            else:
                if job.model_key is not None:
                    s.wait_event(self.model_events[job.model_key])
                    grid = self.models[job.model_key]
                else:
                    grid = self._dev(pl["grid"], self.cplx)
                v.vis = torch.empty(tuple(wt.shape), dtype=self.cplx, device=self.dev)
                lr.lr_degrid(cf, v, self.p, grid, stream=s)
                dev_out = v.vis
            try:
                out = torch.empty(dev_out.shape, dtype=dev_out.dtype, pin_memory=True)
            except RuntimeError:
                # pinned memory exhausted (results the caller still holds):
                # a pageable copy, slower but bounded by host memory only
                out = None
            if out is not None:
                out.copy_(dev_out, non_blocking=True)
                s.synchronize()
            else:
                s.synchronize()
                out = dev_out.cpu()
        return out.numpy()


_ROUND = 2 << 20      # the caching allocator's segment granule for large blocks


def _r(b):
    return (int(b) + _ROUND - 1) // _ROUND * _ROUND


def job_footprint(op, grid_spec, cf_spec, nrow, nchan, npol, precision, resident_model=False):
    """Device bytes GPUExecutor.run allocates for one job, each tensor
    rounded up to 2 MiB: uvw, weights, the visibilities (input of a grid
    job, output of a degrid job), the output grid of a grid job (or the
    model grid of a degrid job without a resident one), and the library's
    workspace (with the transient binning plan) from lr_workspace_bytes."""
    from . import lr
    cplx = 16 if precision == lr.LR_F64 else 8
    n = int(nrow) * int(nchan) * int(npol)
    grid = int(grid_spec.nplane) * npol * int(grid_spec.nx) * int(grid_spec.ny) * cplx
    opc = lr.LR_OP_GRID if op == "grid" else lr.LR_OP_DEGRID
    ws = lr.workspace_bytes_for(opc, grid_spec, cf_spec, nrow, nchan, npol, precision)
    b = _r(24 * nrow) + _r(n * cplx // 2) + _r(n * cplx) + _r(ws)
    if op == "grid" or not resident_model:
        b += _r(grid)
    return b


def cf_footprint(grid_spec, cf_spec):
    """(bytes of the resident CF blob, transient workspace of its build),
    each rounded up to 2 MiB."""
    from . import lr
    blob = lr.cf_bytes_for(grid_spec, cf_spec)
    work = lr.workspace_bytes_for(lr.LR_OP_CF_BUILD, grid_spec, cf_spec, 0, 0, 0,
                                  cf_spec["storage"])
    return _r(blob), _r(work)


def model_footprint(grid_spec, precision):
    from . import lr
    cplx = 16 if precision == lr.LR_F64 else 8
    return _r(int(grid_spec.nplane) * grid_spec.npol * grid_spec.nx * grid_spec.ny * cplx)
