"""GPU: deterministic order (lr_set_deterministic).

With the mode on, repeated gridding calls on the same inputs give
bit-identical grids and sums of weights, also with other work running on
another stream, with a transient instead of an explicit plan and with rows
in time order (column presum) or shuffled (sorted-order gather); the
results match the oracle within the form's tolerance and the default mode
up to rounding order; lr_sumwt gives the same sums bit for bit; and a
serving job's result is bit-identical alone and in the mix.
"""

import copy
import time

import numpy as np
import pytest

import synth
import oracle
from oracle.cfbuild import TERM_A, TERM_PS, TERM_W
from oracle.native import Problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2508_17187_amd import lr  # noqa: E402
from paper_2508_17187_amd import workload as W  # noqa: E402

DEV = "cuda"
PREC = {"f64": lr.LR_F64, "f32": lr.LR_F32}
TOL = {"f64": 1e-12, "f32": 1e-5}


def rel(a, b):
    a = np.asarray(a, np.complex128).ravel()
    b = np.asarray(b, np.complex128).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture
def det():
    prev = lr.set_deterministic(True)
    assert lr.lib().lr_deterministic() == 1
    yield
    lr.set_deterministic(prev)


def workloads():
    # tiles shared by many chunks (Standard kernel, dense), and W + A
    # kernels with pointing offsets on a ragged grid
    a = synth.tiny_workload(n_ant=12, n_time=300, dt_s=60.0, nchan=4, nx=64, ny=64,
                            cell_arcsec=30.0, diameter_m=3000.0, oversample=16, terms=TERM_PS,
                            h_min=3, h_max=3, cfg_id=210)
    b = synth.tiny_workload(n_w=6, h_min=3, h_max=9, oversample=8,
                            terms=TERM_PS | TERM_W | TERM_A, nchan=4, n_time=64, nx=112, ny=72,
                            cell_arcsec=3.0, diameter_m=6000.0, nplane=2,
                            chan_plane=[0, 1, -1, 0], chan_fg=[0, 0, 1, 1],
                            fg_hz=[2.4e9, 3.6e9], cfg_id=211, pointing_sigma=3e-5)
    rng = np.random.default_rng(211)
    b.weight[rng.random(b.weight.shape) < 0.05] = 0.0
    # rows in random order have no period: every group sum takes the
    # sorted-order gather instead of the column presum
    c = copy.deepcopy(a)
    perm = rng.permutation(a.obs.nrow)
    c.obs.uvw, c.obs.ant1, c.obs.ant2 = a.obs.uvw[perm], a.obs.ant1[perm], a.obs.ant2[perm]
    c.vis, c.weight = a.vis[perm], a.weight[perm]
    return {"shared": a, "awp": b, "shuffled": c}


WL = {}


def get(name):
    if not WL:
        WL.update(workloads())
    return WL[name]


def run(cf, v, p, wl, overwrite=True):
    g = W.empty_grid(wl, p)
    if overwrite:
        g.real.fill_(float("nan"))
    sw = torch.zeros((wl.grid.nplane, wl.grid.npol), dtype=torch.float64, device=DEV)
    cnt = torch.zeros(3, dtype=torch.int64, device=DEV)
    (lr.lr_grid_overwrite if overwrite else lr.lr_grid)(cf, v, p, g, sumwt=sw, counters=cnt)
    torch.cuda.synchronize()
    return g.cpu().numpy(), sw.cpu().numpy(), cnt.cpu().numpy()


@pytest.mark.parametrize("name", ["shared", "awp", "shuffled"])
@pytest.mark.parametrize("form", ["f64", "f32"])
def test_repeated_calls_are_bit_identical(det, name, form):
    wl = get(name)
    p = PREC[form]
    cf = W.build_cf(wl, p)
    v = W.device_vis(wl, p)
    v.plan = lr.Plan(cf, v)
    g1, s1, c1 = run(cf, v, p, wl)
    # again, with other work on another stream meanwhile
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        junk = torch.randn((4096, 4096), device=DEV)
        for _ in range(5):
            junk = junk @ junk.T / 4096.0
    g2, s2, c2 = run(cf, v, p, wl)
    torch.cuda.synchronize()
    assert np.array_equal(g1.view(np.uint8), g2.view(np.uint8))
    assert np.array_equal(s1.view(np.uint8), s2.view(np.uint8)) and np.array_equal(c1, c2)
    # a transient plan gives the same bits
    g3, s3, _ = run(cf, W.device_vis(wl, p), p, wl)
    assert np.array_equal(g1.view(np.uint8), g3.view(np.uint8))
    assert np.array_equal(s1.view(np.uint8), s3.view(np.uint8))
    # accumulating into zeros gives the same values as overwriting
    g4, s4, _ = run(cf, v, p, wl, overwrite=False)
    assert np.array_equal(g1, g4)
    # the oracle and the default mode
    ocf = oracle.build_cf(wl.grid, wl.cf)
    pr = Problem.from_workload(wl, ocf)
    assert rel(g1, pr.grid(wl.vis, wl.weight)) <= TOL[form]
    s_ref, c_ref = pr.sumwt(wl.weight)
    assert np.array_equal(c1, c_ref)
    assert np.max(np.abs(s1 - s_ref)) <= 1e-12 * np.abs(s_ref).max()
    lr.set_deterministic(False)
    g5, s5, _ = run(cf, v, p, wl)
    lr.set_deterministic(True)
    assert rel(g1, g5) <= (1e-13 if form == "f64" else 1e-6)
    # lr_sumwt gives the same bits as the gridding call
    sw = torch.zeros_like(torch.as_tensor(s1, device=DEV))
    lr.lr_sumwt(cf, v, p, sw)
    torch.cuda.synchronize()
    assert np.array_equal(sw.cpu().numpy().view(np.uint8), s1.view(np.uint8))


def test_serving_job_alone_and_in_the_mix_bit_identical(det):
    from test_gpu_serving import make_jobs
    from paper_2508_17187_amd.serving import GPUExecutor, Server
    p = lr.LR_F32
    jobs = make_jobs(precision=p)
    srv = Server(GPUExecutor(4, p), hbm_budget=256 << 20, n_slots=4)
    futs = []
    for j in jobs:
        futs.append(srv.submit(j))
        time.sleep(0.002)
    srv.drain(timeout=120)
    mix = {j.job_id: f.result(timeout=5).result for j, f in zip(jobs, futs)}
    srv.close()
    for j in make_jobs(precision=p):
        s1 = Server(GPUExecutor(1, p), hbm_budget=256 << 20, n_slots=1)
        alone = s1.submit(j).result(timeout=60).result
        s1.close()
        assert np.array_equal(mix[j.job_id].view(np.uint8), alone.view(np.uint8)), j.job_id
