"""Continuous batching on the GPU: jobs of uneven sizes submitted while
others run give the same result in the mix as alone (1e-5 in FP32, 1e-12 in
FP64: only the order of atomic adds differs), CF tables and model grids
stay resident across jobs, and with a budget that admits only two or three
jobs at a time the device memory the jobs allocate (torch's allocator
peak) never exceeds the budget, while every result still equals the job
alone."""

import time

import numpy as np
import pytest

import synth
from oracle.cfbuild import TERM_PS, TERM_W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2508_17187_amd import lr  # noqa: E402
from paper_2508_17187_amd import workload as W  # noqa: E402
from paper_2508_17187_amd.serving import (GPUExecutor, Job, Server, cf_footprint,  # noqa: E402
                                          job_footprint, model_footprint)


def make_jobs(n=16, seed=7, precision=lr.LR_F32, sizes=(64, 96, 128), n_time=(4, 40)):
    rng = np.random.default_rng(seed)
    f64 = precision == lr.LR_F64
    cdt, rdt = (np.complex128, np.float64) if f64 else (np.complex64, np.float32)
    models = {}
    jobs = []
    for i in range(n):
        nx = int(rng.choice(sizes))
        n_w = int(rng.choice([1, 4]))
        wl = synth.tiny_workload(nx=nx, ny=nx, n_w=n_w, h_min=3, h_max=3 if n_w == 1 else 6,
                                 oversample=8, terms=TERM_PS | (TERM_W if n_w > 1 else 0),
                                 n_time=int(rng.integers(*n_time)), nchan=2, cell_arcsec=6.0,
                                 diameter_m=4000.0, cfg_id=200 + i)
        gs = W.grid_spec(wl.grid)
        spec = W.cf_spec(wl.cf, precision)
        op = "grid" if i % 2 == 0 else "degrid"
        g, mkey = None, None
        if op == "degrid":
            # one model grid per grid size, shared by the degrid jobs of that size
            mkey = nx
            if nx not in models:
                models[nx] = (rng.standard_normal((1, 4, nx, nx))
                              + 1j * rng.standard_normal((1, 4, nx, nx))).astype(cdt)
            g = models[nx]
        payload = dict(grid_spec=gs, cf_spec=spec, uvw=wl.obs.uvw, freq=wl.obs.freq_hz,
                       chan_plane=wl.chan_plane, vis=wl.vis.astype(cdt),
                       weight=wl.weight.astype(rdt), grid=g)
        key = (nx, n_w, round(wl.cf.w_max, 6))
        cfb, cfw = cf_footprint(gs, spec)
        jobs.append(Job(i, op, key, job_footprint(op, gs, spec, wl.obs.nrow, 2, 4, precision,
                                                  resident_model=mkey is not None),
                        cfb, payload=payload, n_vis=wl.vis.size, model_key=mkey,
                        model_bytes=model_footprint(gs, precision) if mkey is not None else 0,
                        cf_build_bytes=cfw))
    return jobs


def alone_results(jobs_fn, p, budget):
    out = {}
    for j in jobs_fn():
        exe1 = GPUExecutor(1, p)
        s1 = Server(exe1, hbm_budget=budget, n_slots=1)
        out[j.job_id] = s1.submit(j).result(timeout=60).result
        s1.close()
    return out


@pytest.mark.parametrize("form,tol", [("f32", 1e-5), ("f64", 1e-12)])
def test_results_alone_equal_results_in_the_mix(form, tol):
    p = lr.PRECISIONS[form]
    jobs = make_jobs(precision=p)
    exe = GPUExecutor(4, p)
    budget = 512 << 20
    srv = Server(exe, hbm_budget=budget, n_slots=4)
    futs = []
    for j in jobs:
        futs.append(srv.submit(j))
        time.sleep(0.002)
    srv.drain(timeout=120)
    mix = {j.job_id: f.result(timeout=5).result for j, f in zip(jobs, futs)}
    st = srv.stats()
    srv.close()
    assert st["jobs_done"] == len(jobs) and st["jobs_failed"] == 0
    assert st["peak_hbm_bytes"] <= budget
    assert st["p99_s"] >= st["p50_s"] > 0
    # degrid jobs of one grid size share one resident model grid
    assert st["model_uploads"] == len({j.model_key for j in jobs if j.model_key is not None})
    alone = alone_results(lambda: make_jobs(precision=p), p, budget)
    for j in jobs:
        a, b = mix[j.job_id], alone[j.job_id]
        e = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        assert e <= tol, (j.job_id, j.op, e)


def test_binding_budget_holds_on_the_device_and_results_match_alone():
    p = lr.LR_F32
    mk = lambda: make_jobs(n=12, seed=11, precision=p, sizes=(512, 768), n_time=(200, 400))
    jobs = mk()
    need = max(j.bytes + j.cf_build_bytes + j.cf_bytes + j.model_bytes for j in jobs)
    budget = int(2.5 * need)
    print("largest job %d B, budget %d B" % (need, budget), flush=True)
    exe = GPUExecutor(4, p)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    base = torch.cuda.memory_allocated()
    torch.cuda.reset_peak_memory_stats()
    srv = Server(exe, hbm_budget=budget, n_slots=4)
    futs = [srv.submit(j) for j in jobs]           # all at once: admission must wait
    srv.drain(timeout=300)
    mix = {j.job_id: f.result(timeout=5).result for j, f in zip(jobs, futs)}
    st = srv.stats()
    srv.close()
    torch.cuda.synchronize()
    peak = torch.cuda.max_memory_allocated() - base
    print("allocator peak %d B, scheduler peak %d B, admission wait p99 %.3f s"
          % (peak, st["peak_hbm_bytes"], st["admission_wait_p99_s"]), flush=True)
    assert st["jobs_done"] == len(jobs) and st["jobs_failed"] == 0
    assert peak <= budget
    assert st["admission_wait_p99_s"] > 0
    del exe
    alone = alone_results(mk, p, budget)
    for j in jobs:
        a, b = mix[j.job_id], alone[j.job_id]
        e = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        assert e <= 1e-5, (j.job_id, j.op, e)
