"""Parity at full size (W-projection: 13,478,400 visibilities, 32 w-planes,
2048^2 x 4 grid) in the launch configuration bench.py times (binning plan,
lr_grid_overwrite and lr_degrid; FP64, FP32 and FP16-CF forms), on outputs
the oracle computes one by one:

* degridding: 4000 random (row, channel) samples of the GPU result against
  the oracle degridding the same grid for just those rows;
* gridding: 300 random cells of the GPU grid against the oracle gridding
  every row whose footprint covers one of them (which is all the grid those
  cells receive).
"""

import numpy as np
import pytest

import synth
import oracle
from oracle.native import Problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2508_17187_amd import lr  # noqa: E402
from paper_2508_17187_amd import workload as W  # noqa: E402

TOL = {"f64": 1e-12, "f32": 1e-5, "f16cf": 3e-3}


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def c2():
    wl = synth.config2_wproj(dft_device="cuda")
    say("config2", wl.nsamples)
    m = Problem.from_workload(wl, oracle.build_cf(wl.grid, wl.cf, planes=set())).map()
    return wl, m


def sub_problem(wl, rows, ocf):
    return Problem(wl.obs.uvw[rows], wl.obs.freq_hz, wl.chan_plane, wl.chan_fg, wl.grid.nx,
                   wl.grid.ny, wl.grid.npol, wl.grid.nplane, wl.grid.cell_l, wl.grid.cell_m, ocf)


@pytest.mark.parametrize("form", ["f64", "f32", "f16cf"])
def test_fullsize_degrid_sampled(c2, form):
    wl, m = c2
    p = lr.PRECISIONS[form]
    rng = np.random.default_rng(21)
    shape = (1, 4, wl.grid.ny, wl.grid.nx)
    x = (rng.standard_normal(shape, np.float32) + 1j * rng.standard_normal(shape, np.float32)
         ).astype(np.complex128 if form == "f64" else np.complex64)
    cf = W.build_cf(wl, p)
    v = W.device_vis(wl, p)
    v.plan = lr.Plan(cf, v)
    say("degrid", form, v.plan.info())
    lr.lr_degrid(cf, v, p, torch.as_tensor(x, device="cuda"))
    got = v.vis.cpu().numpy()
    rows = np.sort(rng.choice(wl.obs.nrow, 250, replace=False))
    ks = set((0, int(k)) for k in np.unique(m[rows][..., 4][m[rows][..., 6] == 1]))
    ocf = oracle.build_cf(wl.grid, wl.cf, planes=ks)
    ref = sub_problem(wl, rows, ocf).degrid(x.astype(np.complex128), wl.weight[rows])
    g = got[rows]
    e = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    say("degrid sampled rel-rms", form, e, "samples", ref.size)
    assert e <= TOL[form]


@pytest.mark.parametrize("form", ["f64", "f32", "f16cf"])
def test_fullsize_grid_sampled_cells(c2, form):
    wl, m = c2
    p = lr.PRECISIONS[form]
    cf = W.build_cf(wl, p)
    v = W.device_vis(wl, p)
    v.plan = lr.Plan(cf, v)
    # the gridding call bench.py times: a fresh grid written whole (garbage
    # in the output buffer beforehand must not survive)
    g = torch.full((1, 4, wl.grid.ny, wl.grid.nx), 7.0, dtype=torch.complex128 if form == "f64"
                   else torch.complex64, device="cuda")
    sw = torch.full((1, 4), 5.0, dtype=torch.float64, device="cuda")
    cnt = torch.full((3,), 9, dtype=torch.int64, device="cuda")
    lr.lr_grid_overwrite(cf, v, p, g, sumwt=sw, counters=cnt)
    got = g[0].cpu().numpy()                       # [pol][ny][nx]
    rng = np.random.default_rng(22)
    keep = m[..., 6] == 1
    # pick cells covered by the data: around kept pixels
    kr, kc = np.nonzero(keep)
    sel = rng.choice(kr.size, 300, replace=False)
    h = oracle.half_widths(wl.cf.n_w, wl.cf.h_min, wl.cf.h_max)
    cells = []
    for i in sel:
        mm = m[kr[i], kc[i]]
        hh = int(h[mm[4]])
        cells.append((mm[1] + rng.integers(-hh, hh + 1), mm[0] + rng.integers(-hh, hh + 1)))
    cells = np.array(cells)
    # rows with any kept sample whose footprint covers one of the cells
    pu, pv, kk = m[..., 0], m[..., 1], m[..., 4]
    hk = h[kk]
    cover = np.zeros(keep.shape, bool)
    for cy, cx in cells:
        cover |= keep & (np.abs(pu - cx) <= hk) & (np.abs(pv - cy) <= hk)
    rows = np.nonzero(cover.any(axis=1))[0]
    ks = set((0, int(k)) for k in np.unique(kk[rows][keep[rows]]))
    say("grid", form, "cells", len(cells), "rows", rows.size, "planes", len(ks))
    ocf = oracle.build_cf(wl.grid, wl.cf, planes=ks)
    ref = sub_problem(wl, rows, ocf).grid(wl.vis[rows], wl.weight[rows])[0]
    a = got[:, cells[:, 0], cells[:, 1]]
    b = ref[:, cells[:, 0], cells[:, 1]]
    e = np.linalg.norm(a - b) / np.linalg.norm(b)
    say("grid sampled-cell rel-rms", form, e)
    assert e <= TOL[form]
    # cells no footprint reaches were written as 0, sums and counts replaced
    far = got[:, :8, :8]
    assert np.all(far == 0)
    s_ref, c_ref = Problem.from_workload(wl, oracle.build_cf(wl.grid, wl.cf, planes=set(),
                                                             compact=True)).sumwt(wl.weight)
    assert np.array_equal(cnt.cpu().numpy(), c_ref)
    np.testing.assert_allclose(sw.cpu().numpy(), s_ref, rtol=1e-12)
