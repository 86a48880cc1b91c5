"""GPU: the A-projection image normalisation (Eq. ResIm with the A term on,
Table AWP-CFSETUP A-Projection rows).

lr_ps_taper and lr_pb_image against the oracle's taper and weight image;
dirty and residual images of A+W data with two frequency groups, four
correlations and a cube of two planes (lr_grid_overwrite, rocFFT,
lr_image_normalize_pb) against the oracle's chain on the same inputs; and a
point source half-way down the beam, with beam-attenuated visibilities,
imaged back at its flux.
"""

import numpy as np
import pytest

import oracle
import synth
from oracle.cfbuild import TERM_A, TERM_PS, TERM_W, airy_power
from oracle.conventions import C_LIGHT
from oracle.imaging import centred_fft, centred_ifft, normalise_aw, pb_image, ps_taper
from oracle.native import Problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2508_17187_amd import lr  # noqa: E402
from paper_2508_17187_amd import workload as W  # noqa: E402
from paper_2508_17187_amd.imaging import (aw_normalisation, dirty_image_aw,  # noqa: E402
                                          fg_weight_sums, residual_image_aw)

PREC = {"f64": lr.LR_F64, "f32": lr.LR_F32}
TOL = {"f64": 1e-10, "f32": 1e-5}
PB_MIN = 0.1


def aw_workload():
    return synth.tiny_workload(n_ant=10, diameter_m=500.0, n_time=40, dt_s=300.0, nchan=4,
                               nx=96, ny=96, cell_arcsec=24.0, oversample=8,
                               terms=TERM_PS | TERM_A | TERM_W, n_w=4, h_min=7, h_max=9,
                               nplane=2, chan_plane=[0, 1, 0, 1], chan_fg=[0, 0, 1, 1],
                               fg_hz=[2.6e9, 3.4e9], n_src=4, cfg_id=261)


def oracle_fg_weights(wl):
    g = wl.grid
    out = np.zeros((g.nplane, g.npol, len(wl.cf.fg_hz)))
    for k in range(len(wl.cf.fg_hz)):
        cp = np.where(np.asarray(wl.chan_fg) == k, wl.chan_plane, -1).astype(np.int32)
        pr = Problem(wl.obs.uvw, wl.obs.freq_hz, cp, wl.chan_fg, g.nx, g.ny, g.npol, g.nplane,
                     g.cell_l, g.cell_m, oracle.build_cf(g, wl.cf, planes=set(), compact=True))
        out[:, :, k] = pr.sumwt(wl.weight)[0]
    return out


def oracle_aw_image(wl, ocf, vis):
    g = wl.grid
    pr = Problem.from_workload(wl, ocf)
    grid = pr.grid(vis, wl.weight)
    sw = pr.sumwt(wl.weight)[0]
    pb = pb_image(g.nx, g.ny, g.cell_l, g.cell_m, wl.cf.fg_hz, wl.cf.dish_m,
                  oracle_fg_weights(wl))
    img = centred_ifft(grid)
    return normalise_aw(img, ps_taper(g.nx, 7), ps_taper(g.ny, 7), sw, pb, PB_MIN), pb


def rel_on(a, b, mask):
    return float(np.linalg.norm((a - b)[mask]) / np.linalg.norm(b[mask]))


def test_taper_and_weight_image_match_the_oracle():
    wl = aw_workload()
    cf = W.build_cf(wl, lr.LR_F64)
    g = wl.grid
    for n in (g.nx, 130):
        got = lr.lr_ps_taper(cf, n).cpu().numpy()
        assert np.max(np.abs(got - ps_taper(n, 7))) < 1e-13
    v = W.device_vis(wl, lr.LR_F64)
    fgw = fg_weight_sums(cf, v, lr.LR_F64)
    ref_w = oracle_fg_weights(wl)
    assert np.allclose(fgw.cpu().numpy(), ref_w, rtol=1e-13, atol=0)
    pb = lr.lr_pb_image(cf, fgw).cpu().numpy()
    ref = pb_image(g.nx, g.ny, g.cell_l, g.cell_m, wl.cf.fg_hz, wl.cf.dish_m, ref_w)
    assert np.max(np.abs(pb - ref)) < 1e-13
    assert pb[:, :, g.ny // 2, g.nx // 2] == pytest.approx(1.0, abs=1e-15)
    # no A term: 1 everywhere
    wps = synth.tiny_workload(nx=64, ny=64, cfg_id=262)
    cps = W.build_cf(wps, lr.LR_F64)
    ones = torch.ones((1, 4, 1), dtype=torch.float64, device="cuda")
    assert torch.all(lr.lr_pb_image(cps, ones) == 1.0)


@pytest.mark.parametrize("form", ["f64", "f32"])
def test_dirty_and_residual_images_match_the_oracle(form):
    p = PREC[form]
    wl = aw_workload()
    ocf = oracle.build_cf(wl.grid, wl.cf)
    g = wl.grid
    cf = W.build_cf(wl, p)
    v = W.device_vis(wl, p)
    norm = aw_normalisation(cf, v, p)
    img, _ = dirty_image_aw(cf, v, p, pb_min=PB_MIN, norm=norm)
    ref, pb = oracle_aw_image(wl, ocf, wl.vis)
    inner = np.zeros(ref.shape, bool)
    inner[..., g.ny // 4:3 * g.ny // 4, g.nx // 4:3 * g.nx // 4] = True
    mask = inner & (pb >= PB_MIN)
    assert mask.sum() > 1000
    e = rel_on(img.cpu().numpy(), ref, mask)
    print("AW dirty image rel-RMS", form, e, flush=True)
    assert e <= TOL[form]
    assert np.all(img.cpu().numpy()[pb < PB_MIN] == 0.0)
    # residual against a model of a few pixels (Gamma = 1 / taper^2)
    rdt = torch.float64 if p == lr.LR_F64 else torch.float32
    model = torch.zeros((g.nplane, g.npol, g.ny, g.nx), dtype=rdt, device="cuda")
    for (y, x, f) in ((48, 48, 0.7), (40, 57, 0.3), (55, 41, 0.5)):
        model[:, 0, y, x] = f
        model[:, 3, y, x] = f
    res, _ = residual_image_aw(cf, v, p, model, pb_min=PB_MIN, norm=norm)
    tx, ty = ps_taper(g.nx, 7), ps_taper(g.ny, 7)
    mg = centred_fft(model.double().cpu().numpy() / (ty[:, None] * tx[None, :]))
    pred = Problem.from_workload(wl, ocf).degrid(mg, wl.weight)
    rref, _ = oracle_aw_image(wl, ocf, wl.vis - pred)
    e = rel_on(res.cpu().numpy(), rref, mask)
    print("AW residual image rel-RMS", form, e, flush=True)
    assert e <= TOL[form]


def test_point_source_imaged_back_at_its_flux():
    cell = 20.0 * np.pi / 180 / 3600
    ix, iy = 21, -6
    wl = synth.tiny_workload(n_ant=14, diameter_m=400.0, n_time=48, dt_s=300.0, nchan=2,
                             npol=1, nx=128, ny=128, cell_arcsec=20.0, oversample=8,
                             terms=TERM_PS | TERM_A, h_min=8, h_max=8, f_lo=2.9e9, f_hi=3.1e9,
                             n_src=1, sigma=0.0, cfg_id=251)
    l0, m0 = ix * cell, iy * cell
    b = float(airy_power(np.pi * wl.cf.dish_m * wl.cf.fg_hz[0] * np.hypot(l0, m0) / C_LIGHT))
    f = wl.obs.freq_hz
    u = wl.obs.uvw[:, 0:1] * f[None, :] / C_LIGHT
    v = wl.obs.uvw[:, 1:2] * f[None, :] / C_LIGHT
    wl.vis = (2.0 * b * np.exp(-2j * np.pi * (u * l0 + v * m0)))[..., None]
    wl.weight = np.ones(wl.vis.shape)
    for form in ("f64", "f32"):
        p = PREC[form]
        cf = W.build_cf(wl, p)
        img, _ = dirty_image_aw(cf, W.device_vis(wl, p), p, pb_min=0.05)
        val = float(img[0, 0, 64 + iy, 64 + ix])
        print("point source", form, val, "beam", b, flush=True)
        assert val == pytest.approx(2.0, rel=0.005)
