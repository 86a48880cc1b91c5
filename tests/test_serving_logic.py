"""Serving logic on the CPU: the admission scheduler under a simulated clock
and the threaded request loop with a fake executor (no GPU)."""

import heapq
import threading
import time

import numpy as np
import pytest

from paper_2508_17187_amd.serving import Job, Scheduler, Server, latency_stats


def simulate(jobs, budget, n_slots, duration, fail_ids=()):
    """Event-driven run: arrivals at job.t_arrival, completion after
    duration(job).  Returns the scheduler and a trace of (time, used)."""
    s = Scheduler(budget, n_slots)
    ev = [(j.t_arrival, 0, j.job_id, j) for j in jobs]
    heapq.heapify(ev)
    trace = []
    order = []
    while ev:
        t, kind, _, j = heapq.heappop(ev)
        if kind == 0:
            s.submit(j, t)
        else:
            s.complete(j, t, "injected" if j.job_id in fail_ids else None)
        for job, new_cf in s.admit(t):
            order.append(job.job_id)
            heapq.heappush(ev, (t + duration(job), 1, job.job_id, job))
        trace.append((t, s.used, len(s.running)))
        assert s.used <= s.budget
        assert len(s.running) <= n_slots
    return s, trace, order


def stream(n, rate=20.0, seed=0):
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1 / rate, n))
    jobs = []
    for i in range(n):
        nvis = int(10 ** rng.uniform(4, 7.3))
        ng = int(rng.choice([512, 1024, 2048, 4096]))
        nw = int(rng.integers(1, 65))
        key = (ng, nw)
        # footprints of the right order: ~60 B per visibility plus the grid;
        # a table of 441 offsets x S^2 taps per plane
        cfb = 8 * 441 * 1883 * nw if nw > 1 else 8 * 101 * 101 * 49
        jobs.append(Job(i, "grid" if rng.random() < 0.5 else "degrid", key,
                        60 * nvis + 32 * ng * ng, cfb, n_vis=nvis, t_arrival=float(t[i])))
    return jobs


def test_budget_slots_and_arrival_order_hold():
    jobs = stream(256)
    budget = 16 << 30
    s, trace, order = simulate(jobs, budget, 4, lambda j: 2e-8 * j.n_vis + 0.05)
    assert len(s.done) == 256 and not s.rejected
    assert order == sorted(order)                 # admitted in arrival order
    assert max(u for _, u, _ in trace) <= budget
    assert max(r for _, _, r in trace) == 4      # the slots are all used
    st = latency_stats(s.done)
    assert st["p99_s"] >= st["p50_s"] > 0


def test_jobs_arriving_during_others_are_admitted_as_resources_free():
    # slot-bound: three long jobs, then a short one arrives while they run
    jobs = [Job(i, "grid", ("k", i), 100, 10, n_vis=1, t_arrival=0.0) for i in range(3)]
    jobs.append(Job(3, "grid", ("k", 3), 100, 10, n_vis=1, t_arrival=0.5))
    dur = {0: 3.0, 1: 1.0, 2: 2.0, 3: 0.1}
    s, _, _ = simulate(jobs, 1000, 3, lambda j: dur[j.job_id])
    j3 = [j for j in s.done if j.job_id == 3][0]
    assert j3.t_admit == pytest.approx(1.0)      # the first slot to free up
    # memory-bound: the late job waits for bytes, not slots
    jobs = [Job(0, "grid", "a", 600, 0, t_arrival=0.0),
            Job(1, "grid", "a", 600, 0, t_arrival=0.1)]
    s, _, _ = simulate(jobs, 1000, 4, lambda j: 2.0)
    j1 = [j for j in s.done if j.job_id == 1][0]
    assert j1.t_admit == pytest.approx(2.0)


def test_resident_cf_is_shared_and_evicted_lru_when_budget_binds():
    s = Scheduler(1000, 4)
    a = Job(0, "grid", "A", 100, 300, t_arrival=0)
    b = Job(1, "grid", "A", 100, 300, t_arrival=0)
    s.submit(a, 0), s.submit(b, 0)
    adm = s.admit(0)
    assert [n for _, n in adm] == [True, False]   # one CF for both
    assert s.used == 500
    s.complete(a, 1), s.complete(b, 1)
    assert s.used == 300 and "A" in s.cf          # stays resident when idle
    c = Job(2, "grid", "B", 100, 700, t_arrival=2)
    s.submit(c, 2)
    adm = s.admit(2)
    assert adm and "A" not in s.cf and s.used == 800   # A evicted for B


def test_model_grids_stay_resident_and_build_scratch_is_charged_once():
    s = Scheduler(2000, 4)
    # two degrid jobs on one model grid and one CF: one copy of each; the CF
    # build's scratch is charged to the job that brings the table in only
    a = Job(0, "degrid", "A", 100, 300, model_key="M", model_bytes=400, cf_build_bytes=50)
    b = Job(1, "degrid", "A", 100, 300, model_key="M", model_bytes=400, cf_build_bytes=50)
    s.submit(a, 0), s.submit(b, 0)
    adm = s.admit(0)
    assert [n for _, n in adm] == [True, False]
    assert a.model_cold and not b.model_cold
    assert a.charged == 150 and b.charged == 100
    assert s.used == 300 + 400 + 150 + 100
    s.complete(a, 1), s.complete(b, 1)
    assert s.used == 700 and "M" in s.models and "A" in s.cf     # idle, still resident
    # a job needing 1500 more bytes evicts idle resources, least recently
    # used first, until it fits: the CF goes, the model grid stays
    c = Job(2, "grid", "B", 1000, 500)
    s.submit(c, 2)
    assert s.admit(2) and s.used == 400 + 1500
    assert s.take_evicted() == [("cf", "A")] and "M" in s.models


def test_a_jobs_own_idle_resources_are_not_evicted_to_make_room_for_it():
    s = Scheduler(1000, 4)
    a = Job(0, "degrid", "A", 100, 300, model_key="M", model_bytes=300)
    s.submit(a, 0)
    s.admit(0)
    s.complete(a, 1)                                  # A and M idle: 600 used
    b = Job(1, "degrid", "A", 300, 300, model_key="M", model_bytes=300)
    s.submit(b, 1)
    assert s.admit(1)                                 # 600 + 300 fits without eviction
    assert s.used == 900 and not s.take_evicted()
    s.complete(b, 2)
    c = Job(2, "degrid", "A", 500, 300, model_key="M", model_bytes=300)
    s.submit(c, 2)
    assert not s.admit(2)                             # would need its own A or M evicted
    assert s.used == 600 and "A" in s.cf and "M" in s.models


def test_oversized_job_is_rejected_alone_and_failures_are_isolated():
    jobs = stream(40, seed=3)
    big = Job(99, "grid", "huge", 10 << 40, 0, t_arrival=0.2)
    s, _, _ = simulate(jobs + [big], 16 << 30, 4, lambda j: 0.01, fail_ids={5, 6})
    assert [j.job_id for j in s.rejected] == [99]
    failed = sorted(j.job_id for j in s.done if j.error)
    assert failed == [5, 6]
    assert len([j for j in s.done if not j.error]) == 38
    assert s.used == sum(e[0] for e in s.cf.values())   # only resident CFs remain


class FakeExecutor:
    """Sleeps for a duration proportional to the job; optional failures."""

    def __init__(self, fail=()):
        self.fail = set(fail)
        self.cfs = set()
        self.concurrency = 0
        self.max_concurrency = 0
        self.lock = threading.Lock()

    def has_cf(self, key):
        return key in self.cfs

    def prepare_cf(self, job, slot):
        time.sleep(0.005)
        if job.job_id in self.fail and job.op == "cf":
            raise RuntimeError("cf build failed")
        self.cfs.add(job.cf_key)

    def release_cf(self, key):
        self.cfs.discard(key)

    def run(self, job, slot):
        with self.lock:
            self.concurrency += 1
            self.max_concurrency = max(self.max_concurrency, self.concurrency)
        try:
            time.sleep(0.002 + 1e-9 * job.n_vis)
            if job.job_id in self.fail:
                raise RuntimeError("injected fault")
            return job.job_id * 2
        finally:
            with self.lock:
                self.concurrency -= 1


def test_threaded_server_with_fake_executor():
    exe = FakeExecutor(fail={7})
    srv = Server(exe, hbm_budget=16 << 30, n_slots=4)
    jobs = stream(48, rate=400.0, seed=4)
    futs = []
    for j in jobs:
        futs.append(srv.submit(j))
        time.sleep(0.001)
    srv.drain(timeout=60)
    ok = 0
    for j, f in zip(jobs, futs):
        if j.job_id == 7:
            with pytest.raises(RuntimeError):
                f.result(timeout=1)
        else:
            assert f.result(timeout=1).result == j.job_id * 2
            ok += 1
    st = srv.stats()
    srv.close()
    assert ok == 47 and st["jobs_done"] == 47 and st["jobs_failed"] == 1
    assert exe.max_concurrency > 1                  # work overlapped
    assert st["peak_hbm_bytes"] <= st["hbm_budget"]


def test_cf_evicted_and_brought_back_in_one_batch_is_prepared_again():
    # X and Z resident and idle (X least recently used); A (new CF Y) evicts
    # X, and B, admitted in the same batch, brings X back: B must build it
    # and succeed, as must a later job that shares it
    exe = FakeExecutor()
    srv = Server(exe, hbm_budget=90, n_slots=3)
    mk = lambda i, key: Job(i, "grid", key, 5, 30, n_vis=10)
    srv.submit(mk(0, "X")).result(timeout=5)
    srv.submit(mk(1, "Z")).result(timeout=5)
    with srv.lock:                      # both queued before the loop looks
        fa = srv.submit(mk(2, "Y"))
        fb = srv.submit(mk(3, "X"))
    assert fa.result(timeout=5).result == 4
    assert fb.result(timeout=5).result == 6
    assert srv.submit(mk(4, "X")).result(timeout=5).result == 8
    st = srv.stats()
    srv.close()
    assert st["jobs_failed"] == 0 and st["errors"] == {}
    assert exe.has_cf("X") and exe.has_cf("Y")
