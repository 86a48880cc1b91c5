"""Continuous batching on the GPU: jobs of uneven sizes submitted while
others run give the same result in the mix as alone (1e-5 in FP32, 1e-12 in
FP64: only the order of atomic adds differs), the HBM budget is never
exceeded and CF tables stay resident across jobs."""

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
from paper_2508_17187_amd.serving import GPUExecutor, Job, Server, cf_bytes, job_bytes  # noqa: E402


def make_jobs(n=16, seed=7, precision=lr.LR_F32):
    rng = np.random.default_rng(seed)
    f64 = precision == lr.LR_F64
    cdt, rdt = (np.complex128, np.float64) if f64 else (np.complex64, np.float32)
    jobs = []
    for i in range(n):
        nx = int(rng.choice([64, 96, 128]))
        n_w = int(rng.choice([1, 4]))
        wl = synth.tiny_workload(nx=nx, ny=nx, n_w=n_w, h_min=3, h_max=3 if n_w == 1 else 6,
                                 oversample=8, terms=TERM_PS | (TERM_W if n_w > 1 else 0),
                                 n_time=int(rng.integers(4, 40)), nchan=2, cell_arcsec=6.0,
                                 diameter_m=4000.0, cfg_id=200 + i)
        gs = W.grid_spec(wl.grid)
        spec = W.cf_spec(wl.cf, precision)
        op = "grid" if i % 2 == 0 else "degrid"
        g = None
        if op == "degrid":
            g = (rng.standard_normal((1, 4, nx, nx)) + 1j * rng.standard_normal((1, 4, nx, nx))
                 ).astype(cdt)
        payload = dict(grid_spec=gs, cf_spec=spec, uvw=wl.obs.uvw, freq=wl.obs.freq_hz,
                       chan_plane=wl.chan_plane, vis=wl.vis.astype(cdt),
                       weight=wl.weight.astype(rdt), grid=g)
        key = (nx, n_w, round(wl.cf.w_max, 6))
        eb = 16 if f64 else 8
        jobs.append(Job(i, op, key, job_bytes(wl.obs.nrow, 2, 4, nx, precision_bytes=eb),
                        cf_bytes(n_w, 3, 3 if n_w == 1 else 6, 8, eb), payload=payload,
                        n_vis=wl.vis.size))
    return jobs


@pytest.mark.parametrize("form,tol", [("f32", 1e-5), ("f64", 1e-12)])
def test_results_alone_equal_results_in_the_mix(form, tol):
    p = lr.PRECISIONS[form]
    jobs = make_jobs(precision=p)
    exe = GPUExecutor(4, p)
    budget = 256 << 20
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
    # each job alone, on a fresh one-slot server
    for j in make_jobs(precision=p):
        exe1 = GPUExecutor(1, p)
        s1 = Server(exe1, hbm_budget=budget, n_slots=1)
        alone = s1.submit(j).result(timeout=60).result
        s1.close()
        a, b = mix[j.job_id], alone
        e = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        assert e <= tol, (j.job_id, j.op, e)
