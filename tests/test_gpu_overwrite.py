"""GPU: lr_grid_overwrite replaces grid, sumwt and counters with G(vis).

The workload is a ragged grid (112 x 72: tiles of 32 cells overhang both
edges) with two planes, dense enough that some tiles hold more (tile, group)
pairs than one gridder chunk takes, some hold one chunk and some none, so
every tile ownership case is exercised.  Outputs are pre-filled with
garbage; the result must equal the oracle's grid of the same inputs (bars
as for lr_grid), and equal zero + lr_grid.
"""

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
PREC = {"f64": lr.LR_F64, "f32": lr.LR_F32, "f16cf": lr.LR_F32_CF16}
TOL = {"f64": 1e-12, "f32": 1e-5, "f16cf": 3e-3}


def rel(a, b):
    a = np.asarray(a, np.complex128).ravel()
    b = np.asarray(b, np.complex128).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def dense_workload(pointing=0.0, seed_id=93, h_max=7):
    wl = synth.tiny_workload(n_w=6, h_min=3, h_max=h_max, oversample=8,
                             terms=TERM_PS | TERM_W | TERM_A, nchan=4, n_time=64, nx=112,
                             ny=72, cell_arcsec=3.0, diameter_m=6000.0, nplane=2,
                             chan_plane=[0, 1, -1, 0], chan_fg=[0, 0, 1, 1],
                             fg_hz=[2.4e9, 3.6e9], cfg_id=seed_id, pointing_sigma=pointing)
    rng = np.random.default_rng(seed_id)
    wl.weight[rng.random(wl.weight.shape) < 0.05] = 0.0
    return wl


# widest support 15 and 19
@pytest.fixture(scope="module", params=[7, 9], ids=["S15", "S19"])
def dense(request):
    wl = dense_workload(h_max=request.param)
    return wl, oracle.build_cf(wl.grid, wl.cf)


def garbage_outputs(wl, p):
    g = W.empty_grid(wl, p)
    g.real.fill_(float("nan"))
    g.imag.fill_(3.0)
    sw = torch.full((wl.grid.nplane, wl.grid.npol), -5.0, dtype=torch.float64, device=DEV)
    cnt = torch.full((3,), 12345, dtype=torch.int64, device=DEV)
    return g, sw, cnt


@pytest.mark.parametrize("form", ["f64", "f32", "f16cf"])
@pytest.mark.parametrize("use_plan", [False, True])
def test_overwrite_matches_oracle(dense, form, use_plan):
    wl, ocf = dense
    print("overwrite", form, "plan" if use_plan else "transient", flush=True)
    p = PREC[form]
    cf = W.build_cf(wl, p)
    v = W.device_vis(wl, p)
    if use_plan:
        v.plan = lr.Plan(cf, v)
    g, sw, cnt = garbage_outputs(wl, p)
    lr.lr_grid_overwrite(cf, v, p, g, sumwt=sw, counters=cnt)
    torch.cuda.synchronize()
    got = g.cpu().numpy()
    pr = Problem.from_workload(wl, ocf)
    ref = pr.grid(wl.vis, wl.weight)
    s_ref, c_ref = pr.sumwt(wl.weight)
    assert np.all(np.isfinite(got))
    e = rel(got, ref)
    print("overwrite rel-rms", form, e, flush=True)
    assert e <= TOL[form]
    assert np.all(got[ref == 0] == 0)           # cells no footprint reaches
    assert np.array_equal(cnt.cpu().numpy(), c_ref)
    assert np.max(np.abs(sw.cpu().numpy() - s_ref) / np.abs(s_ref).max()) < 1e-12
    # the same as clearing and accumulating
    g2 = W.empty_grid(wl, p)
    lr.lr_grid(cf, v, p, g2)
    torch.cuda.synchronize()
    assert rel(got, g2.cpu().numpy()) <= (1e-14 if form == "f64" else 1e-6)


def test_overwrite_second_call_replaces(dense):
    """A second call with fewer rows into the same buffers leaves nothing of
    the first."""
    wl, ocf = dense
    p = lr.LR_F32
    cf = W.build_cf(wl, p)
    g, sw, cnt = garbage_outputs(wl, p)
    lr.lr_grid_overwrite(cf, W.device_vis(wl, p), p, g, sumwt=sw, counters=cnt)
    half = wl.obs.nrow // 3
    v2 = W.device_vis(wl, p, rows=slice(0, half))
    lr.lr_grid_overwrite(cf, v2, p, g, sumwt=sw, counters=cnt)
    torch.cuda.synchronize()
    import copy
    w2 = copy.deepcopy(wl)
    w2.obs.uvw = wl.obs.uvw[:half]
    w2.obs.ant1 = wl.obs.ant1[:half]
    w2.obs.ant2 = wl.obs.ant2[:half]
    w2.vis = wl.vis[:half]
    w2.weight = wl.weight[:half]
    pr = Problem.from_workload(w2, ocf)
    ref = pr.grid(w2.vis, w2.weight)
    assert rel(g.cpu().numpy(), ref) <= TOL["f32"]
    assert np.array_equal(cnt.cpu().numpy(), pr.sumwt(w2.weight)[1])


def test_overwrite_empty_input_clears(dense):
    wl, _ = dense
    for form in ("f64", "f32"):
        p = PREC[form]
        cf = W.build_cf(wl, p)
        v = W.device_vis(wl, p, rows=slice(0, 0))
        g, sw, cnt = garbage_outputs(wl, p)
        lr.lr_grid_overwrite(cf, v, p, g, sumwt=sw, counters=cnt)
        torch.cuda.synchronize()
        assert g.abs().sum().item() == 0
        assert sw.abs().sum().item() == 0 and cnt.abs().sum().item() == 0
        # every sample flagged: no pairs in any chunk either
        v = W.device_vis(wl, p)
        v.weight.zero_()
        g, sw, cnt = garbage_outputs(wl, p)
        lr.lr_grid_overwrite(cf, v, p, g, sumwt=sw, counters=cnt)
        torch.cuda.synchronize()
        assert g.abs().sum().item() == 0
        assert cnt[1].item() == wl.weight.size


@pytest.mark.parametrize("h_max", [7, 9], ids=["S15", "S19"])
def test_overwrite_pointing_phasor(h_max):
    wl = dense_workload(pointing=3e-5, seed_id=94, h_max=h_max)
    ocf = oracle.build_cf(wl.grid, wl.cf)
    p = lr.LR_F32
    cf = W.build_cf(wl, p)
    v = W.device_vis(wl, p)
    g, sw, cnt = garbage_outputs(wl, p)
    lr.lr_grid_overwrite(cf, v, p, g, sumwt=sw, counters=cnt)
    torch.cuda.synchronize()
    pr = Problem.from_workload(wl, ocf)
    assert rel(g.cpu().numpy(), pr.grid(wl.vis, wl.weight)) <= TOL["f32"]


def test_standard_kernel_tiles_shared_by_many_chunks():
    """Standard kernel (S = 7) on a 64 x 64 grid whose tiles hold over 1024
    (tile, group) pairs, so each is cut into many chunks that add atomically:
    grid, overwrite and PSF against the oracle."""
    wl = synth.tiny_workload(n_ant=12, n_time=300, dt_s=60.0, nchan=4, nx=64, ny=64,
                             cell_arcsec=30.0, diameter_m=3000.0, oversample=16,
                             terms=TERM_PS, h_min=3, h_max=3, cfg_id=95)
    ocf = oracle.build_cf(wl.grid, wl.cf)
    pr = Problem.from_workload(wl, ocf)
    m = pr.map().reshape(-1, 8)
    k = m[m[:, 6] == 1]
    groups = np.unique(np.stack([k[:, 4], k[:, 5], k[:, 1], k[:, 0], k[:, 3], k[:, 2]], 1),
                       axis=0)
    per_tile = {}
    for pv, pu in groups[:, 2:4]:
        for ty in range((pv - 3) // 32, (pv + 3) // 32 + 1):
            for tx in range((pu - 3) // 32, (pu + 3) // 32 + 1):
                per_tile[(ty, tx)] = per_tile.get((ty, tx), 0) + 1
    assert max(per_tile.values()) > 1024          # the case this test is for
    ref = pr.grid(wl.vis, wl.weight)
    for form in ("f64", "f32"):
        p = PREC[form]
        cf = W.build_cf(wl, p)
        v = W.device_vis(wl, p)
        v.plan = lr.Plan(cf, v)
        g = W.empty_grid(wl, p)
        lr.lr_grid(cf, v, p, g)
        g2, sw, cnt = garbage_outputs(wl, p)
        lr.lr_grid_overwrite(cf, v, p, g2, sumwt=sw, counters=cnt)
        torch.cuda.synchronize()
        assert rel(g.cpu().numpy(), ref) <= TOL[form]
        assert rel(g2.cpu().numpy(), ref) <= TOL[form]
    psf_ref, _, _ = pr.psf(wl.weight)
    p = lr.LR_F64
    cf = W.build_cf(wl, p)
    v = W.device_vis(wl, p)
    g = W.empty_grid(wl, p)
    lr.lr_make_psf(cf, v, p, g)
    torch.cuda.synchronize()
    assert rel(g.cpu().numpy(), psf_ref) <= TOL["f64"]
