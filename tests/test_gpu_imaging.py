"""GPU: the image-plane steps around the hot path (Eq. ResIm).

lr_gcf against the oracle's grid correction of the same separable plane;
dirty and residual images (lr_grid_overwrite, rocFFT, lr_image_normalize)
against the oracle's chain on the same inputs (oracle grid or degrid, numpy
FFT, the oracle's correction); a unit point source at the phase centre."""

import numpy as np
import pytest

import synth
import oracle
from oracle.cfbuild import TERM_A, TERM_PS, TERM_W
from oracle.imaging import centred_fft, centred_ifft, gcf_1d, separable_1d
from oracle.native import Problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2508_17187_amd import lr  # noqa: E402
from paper_2508_17187_amd import workload as W  # noqa: E402
from paper_2508_17187_amd.imaging import dirty_image, residual_image  # noqa: E402

PREC = {"f64": lr.LR_F64, "f32": lr.LR_F32, "f16cf": lr.LR_F32_CF16}


def rel(a, b):
    a = np.asarray(a, np.complex128).ravel()
    b = np.asarray(b, np.complex128).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def ps_workload(**kw):
    args = dict(n_ant=8, n_time=24, dt_s=120.0, nchan=3, nx=96, ny=80, cell_arcsec=4.0,
                oversample=20, terms=TERM_PS, h_min=3, h_max=3, cfg_id=97)
    args.update(kw)
    return synth.tiny_workload(**args)


@pytest.mark.parametrize("form,tol", [("f64", 1e-12), ("f32", 1e-6), ("f16cf", 3e-3)])
def test_gcf_matches_oracle(form, tol):
    wl = ps_workload()
    ocf = oracle.build_cf(wl.grid, wl.cf)
    c1 = separable_1d(ocf)
    cf = W.build_cf(wl, PREC[form])
    for n in (wl.grid.nx, wl.grid.ny, 1024):
        got = lr.lr_gcf(cf, n).cpu().numpy()
        ref = gcf_1d(c1, ocf.O, n)
        assert rel(got, ref) <= tol     # complex: offsets -O/2..O/2-1 are not symmetric


def test_gcf_of_the_w0_plane_and_refusals():
    wl = ps_workload(terms=TERM_PS | TERM_W, n_w=4, h_min=3, h_max=5)
    wl.cf.w_max = 2.0e4
    ps = ps_workload()
    ps.cf.screen_m = oracle.build_cf(wl.grid, wl.cf).M
    ocf = oracle.build_cf(ps.grid, ps.cf)
    cf = W.build_cf(wl, lr.LR_F64)
    got = lr.lr_gcf(cf, 96).cpu().numpy()
    assert rel(got, gcf_1d(separable_1d(ocf), ocf.O, 96)) <= 1e-12
    with pytest.raises(lr.LRError) as ei:
        lr.lr_gcf(cf, 96, k=1)
    assert ei.value.status == lr.LR_E_ARG
    with pytest.raises(lr.LRError) as ei:
        lr.lr_gcf(cf, 96, k=9)
    assert ei.value.status == lr.LR_E_RANGE
    aw = ps_workload(terms=TERM_PS | TERM_A)
    with pytest.raises(lr.LRError) as ei:
        lr.lr_gcf(W.build_cf(aw, lr.LR_F64), 96)
    assert ei.value.status == lr.LR_E_ARG


def inner(img):
    """The inner half of each axis, where the correction is well above its
    edge values (dividing by it there magnifies rounding ~1e4 times)."""
    ny, nx = img.shape[-2:]
    return img[..., ny // 4:3 * ny // 4, nx // 4:3 * nx // 4]


def oracle_image(pr, ocf, vis, wt):
    """Re F^dagger G(W V) / (gcf_x gcf_y sumwt) on the CPU."""
    g = pr.grid(vis, wt)
    s, _ = pr.sumwt(wt)
    c1 = separable_1d(ocf)
    gx = gcf_1d(c1, ocf.O, pr.nx).real
    gy = gcf_1d(c1, ocf.O, pr.ny).real
    img = centred_ifft(g).real
    return img / (np.outer(gy, gx)[None, None] * s[:, :, None, None])


@pytest.mark.parametrize("form,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_dirty_image_matches_oracle(form, tol):
    wl = ps_workload()
    ocf = oracle.build_cf(wl.grid, wl.cf)
    pr = Problem.from_workload(wl, ocf)
    ref = oracle_image(pr, ocf, wl.vis, wl.weight)
    p = PREC[form]
    cf = W.build_cf(wl, p)
    img, _ = dirty_image(cf, W.device_vis(wl, p), p)
    e = rel(inner(img.cpu().numpy()), inner(ref))
    print("dirty image", form, e, flush=True)
    assert e <= tol


def test_point_source_at_phase_centre_images_to_unit_peak():
    wl = ps_workload(npol=1, sigma=0.0)
    wl.vis[:] = 1.0
    wl.weight[:] = 1.0
    cf = W.build_cf(wl, lr.LR_F64)
    img, _ = dirty_image(cf, W.device_vis(wl, lr.LR_F64), lr.LR_F64)
    img = img.cpu().numpy()[0, 0]
    peak = img[wl.grid.ny // 2, wl.grid.nx // 2]
    assert abs(peak - 1.0) < 1e-2
    assert np.unravel_index(np.argmax(img), img.shape) == (wl.grid.ny // 2, wl.grid.nx // 2)


@pytest.mark.parametrize("form,tol", [("f64", 1e-11), ("f32", 1e-5)])
def test_residual_image_matches_oracle(form, tol):
    wl = ps_workload()
    ocf = oracle.build_cf(wl.grid, wl.cf)
    pr = Problem.from_workload(wl, ocf)
    g = wl.grid
    rng = np.random.default_rng(98)
    model = np.zeros((g.nplane, g.npol, g.ny, g.nx))
    for _ in range(6):
        model[:, :, rng.integers(g.ny // 4, 3 * g.ny // 4),
              rng.integers(g.nx // 4, 3 * g.nx // 4)] += rng.uniform(0.1, 1.0)
    c1 = separable_1d(ocf)
    gx = gcf_1d(c1, ocf.O, g.nx).real
    gy = gcf_1d(c1, ocf.O, g.ny).real
    pred = pr.degrid(centred_fft(model / np.outer(gy, gx)[None, None]), wl.weight)
    ref = oracle_image(pr, ocf, wl.vis - pred, wl.weight)
    p = PREC[form]
    cf = W.build_cf(wl, p)
    rdt = torch.float64 if p == lr.LR_F64 else torch.float32
    img, _ = residual_image(cf, W.device_vis(wl, p), p,
                            torch.as_tensor(model, dtype=rdt, device="cuda"))
    dirty = oracle_image(pr, ocf, wl.vis, wl.weight)
    e = np.linalg.norm(inner(img.cpu().numpy() - ref)) / np.linalg.norm(inner(dirty))
    print("residual image", form, e, flush=True)
    assert e <= tol
