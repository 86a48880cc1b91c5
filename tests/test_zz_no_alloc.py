"""GPU: lr_grid_static, the gridding entry point that allocates nothing.

Its output is compared with lr_grid's on the same plan, CF and data, on two
calls in a row (the second with fewer rows, so stale contents of the
library's fixed scratch would show), in FP64 and FP32, in the default order
(rounding-order tolerance) and in the deterministic order (bit-identical);
both are also checked against the CPU FP64 oracle.  Host-side errors (no
plan, another form's CF, a plan beyond the fixed scratch) leave the grid
untouched.
"""

import numpy as np
import pytest

import oracle
import synth
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


def _workload():
    return synth.tiny_workload(n_w=5, h_min=3, h_max=8, oversample=8,
                               terms=TERM_PS | TERM_W | TERM_A, nchan=4, n_time=48,
                               nx=112, ny=96, cell_arcsec=3.0, diameter_m=6000.0, cfg_id=231)


def _sub(wl, n_rows):
    """The workload restricted to its first n_rows rows (same grid and CF)."""
    import copy
    s = copy.copy(wl)
    s.obs = copy.copy(wl.obs)
    s.obs.uvw = wl.obs.uvw[:n_rows]
    s.obs.ant1 = wl.obs.ant1[:n_rows]
    s.obs.ant2 = wl.obs.ant2[:n_rows]
    s.vis = wl.vis[:n_rows]
    s.weight = wl.weight[:n_rows]
    return s


@pytest.mark.parametrize("form", ["f64", "f32"])
@pytest.mark.parametrize("deterministic", [False, True])
def test_grid_static_matches_lr_grid(form, deterministic):
    prec = PREC[form]
    wl = _workload()
    ocf = oracle.build_cf(wl.grid, wl.cf)
    cf = W.build_cf(wl, prec)
    prev = lr.set_deterministic(deterministic)
    try:
        nrow = wl.obs.uvw.shape[0]
        # the second call has fewer rows than the first
        for n_rows in (nrow, nrow // 3):
            sub = _sub(wl, n_rows)
            print("lr_grid_static: form=%s det=%s rows=%d" % (form, deterministic, n_rows),
                  flush=True)
            v = W.device_vis(sub, prec)
            plan = lr.Plan(cf, v)
            v = v.with_(plan=plan)
            g_ref = W.empty_grid(sub, prec)
            sw_ref = torch.zeros((1, sub.grid.npol), dtype=torch.float64, device=DEV)
            c_ref = torch.zeros(3, dtype=torch.int64, device=DEV)
            lr.lr_grid(cf, v, prec, g_ref, sw_ref, c_ref)
            g = W.empty_grid(sub, prec)
            sw = torch.zeros_like(sw_ref)
            cnt = torch.zeros_like(c_ref)
            lr.lr_grid_static(cf, v, prec, g, sw, cnt)
            torch.cuda.synchronize()
            got, ref = g.cpu().numpy(), g_ref.cpu().numpy()
            assert np.array_equal(cnt.cpu().numpy(), c_ref.cpu().numpy())
            if deterministic:
                assert np.array_equal(got.view(np.uint8), ref.view(np.uint8))
                assert np.array_equal(sw.cpu().numpy(), sw_ref.cpu().numpy())
            else:
                assert rel(got, ref) <= TOL[form] / 10
                np.testing.assert_allclose(sw.cpu().numpy(), sw_ref.cpu().numpy(), rtol=1e-12)
            pr = Problem.from_workload(sub, ocf)
            want = pr.grid(sub.vis, sub.weight)
            assert rel(got, want) <= TOL[form]
            s_ref, c_ref2 = pr.sumwt(sub.weight)
            assert np.array_equal(cnt.cpu().numpy(), c_ref2)
            np.testing.assert_allclose(sw.cpu().numpy().ravel(), np.asarray(s_ref).ravel(),
                                       rtol=1e-12)
    finally:
        lr.set_deterministic(prev)


def test_grid_static_host_errors():
    prec = lr.LR_F32
    wl = synth.tiny_workload(n_time=8, nchan=2, cfg_id=232)
    cf = W.build_cf(wl, prec)
    v = W.device_vis(wl, prec)
    g = W.empty_grid(wl, prec)
    with pytest.raises(lr.LRError) as e:
        lr.lr_grid_static(cf, v, prec, g)      # no plan
    assert e.value.status == lr.LR_E_ARG
    plan = lr.Plan(cf, v)
    with pytest.raises(lr.LRError) as e:       # CF storage of another form
        lr.lr_grid_static(cf, v.with_(plan=plan), lr.LR_F64, g)
    assert e.value.status in (lr.LR_E_DTYPE, lr.LR_E_ARG)
    torch.cuda.synchronize()
    assert float(g.abs().max()) == 0.0


def test_grid_static_rejects_plans_beyond_its_scratch():
    # about three million one-sample groups: beyond the 2,097,152 groups
    # of 4 FP32 pols the fixed scratch holds
    prec = lr.LR_F32
    gen = torch.Generator(device=DEV)
    gen.manual_seed(233)
    nrow, nchan = 100000, 32
    uvw = ((torch.rand((nrow, 3), generator=gen, device=DEV, dtype=torch.float64) * 2 - 1)
           * torch.tensor([8000.0, 8000.0, 100.0], dtype=torch.float64, device=DEV))
    freq = np.linspace(2.0e9, 4.0e9, nchan)
    wt = torch.ones((nrow, nchan, 4), dtype=torch.float32, device=DEV)
    vis = torch.ones((nrow, nchan, 4), dtype=torch.complex64, device=DEV)
    g = lr.GridSpec(2048, 2048, 4, 1, 0.2 * np.pi / 180 / 3600, 0.2 * np.pi / 180 / 3600)
    cf = lr.lr_cf_build(g, dict(terms=lr.LR_TERM_PS, oversample=100, ps_support=7, n_w=1,
                                w_max=0.0, h_min=3, h_max=3, n_fg=1,
                                fg_hz=np.array([3.0e9]), dish_m=25.0, screen_m=0,
                                storage=prec))
    v = lr.Vis(uvw, freq, vis=vis, weight=wt, npol=4)
    plan = lr.Plan(cf, v)
    assert plan.info()["n_groups"] > 2097152
    grid = torch.zeros((1, 4, 2048, 2048), dtype=torch.complex64, device=DEV)
    with pytest.raises(lr.LRError) as e:
        lr.lr_grid_static(cf, v.with_(plan=plan), prec, grid)
    assert e.value.status == lr.LR_E_RANGE
    torch.cuda.synchronize()
    assert float(grid.abs().max()) == 0.0

