"""GPU: packed plans (lr_plan_pack).

A plan copied into a buffer of its actual size gives the same grid, sums of
weights, counters and degridded visibilities as the plan it came from, bit
for bit (deterministic order for the gridding sums), also after the
original plan and its build buffer are gone; the packed buffer is smaller
than the build buffer.
"""

import gc

import numpy as np
import pytest

import synth
from oracle.cfbuild import TERM_A, TERM_PS, TERM_W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2508_17187_amd import lr  # noqa: E402
from paper_2508_17187_amd import workload as W  # noqa: E402


def _run(cf, v, prec, wl):
    g = W.empty_grid(wl, prec)
    sw = torch.zeros((wl.grid.nplane, wl.grid.npol), dtype=torch.float64, device="cuda")
    cnt = torch.zeros(3, dtype=torch.int64, device="cuda")
    lr.lr_grid(cf, v, prec, g, sw, cnt)
    vd = v.with_(vis=torch.empty_like(v.vis))
    lr.lr_degrid(cf, vd, prec, g)
    torch.cuda.synchronize()
    return g.cpu().numpy(), sw.cpu().numpy(), cnt.cpu().numpy(), vd.vis.cpu().numpy()


@pytest.mark.parametrize("form", ["f64", "f32"])
@pytest.mark.parametrize("pointing", [False, True])
def test_packed_plan_gives_identical_results(form, pointing):
    prec = lr.PRECISIONS[form]
    wl = synth.tiny_workload(n_w=6, h_min=3, h_max=9, oversample=8,
                             terms=TERM_PS | TERM_W | TERM_A, nchan=4, n_time=64, nx=112,
                             ny=72, cell_arcsec=3.0, diameter_m=6000.0, nplane=2,
                             chan_plane=[0, 1, -1, 0], chan_fg=[0, 0, 1, 1],
                             fg_hz=[2.4e9, 3.6e9], pointing_sigma=3e-5 if pointing else 0.0,
                             cfg_id=241)
    cf = W.build_cf(wl, prec)
    v = W.device_vis(wl, prec)
    prev = lr.set_deterministic(True)
    try:
        plan = lr.Plan(cf, v)
        ref = _run(cf, v.with_(plan=plan), prec, wl)
        packed = plan.packed()
        assert packed.buf.numel() < plan.buf.numel()
        assert packed.info() == plan.info()
        del plan
        gc.collect()
        # the build buffer's memory is reused by other work before the
        # packed plan runs
        junk = torch.full((1 << 22,), 7, dtype=torch.int32, device="cuda")
        got = _run(cf, v.with_(plan=packed), prec, wl)
        del junk
    finally:
        lr.set_deterministic(prev)
    for a, b in zip(got, ref):
        assert np.array_equal(np.asarray(a).view(np.uint8), np.asarray(b).view(np.uint8))
