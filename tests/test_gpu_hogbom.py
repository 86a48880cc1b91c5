"""GPU: Hogbom minor cycle (lr_hogbom) against the oracle's loop.

FP64 is compared bit for bit (the same operations in the same order and the
same tie rule give the same components); FP32 within rounding."""

import numpy as np
import pytest

import synth
import oracle
from oracle.cfbuild import TERM_PS
from oracle.hogbom import hogbom
from oracle.imaging import centred_ifft, gcf_1d, separable_1d
from oracle.native import Problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2508_17187_amd import lr  # noqa: E402

DEV = "cuda"


@pytest.fixture(scope="module")
def dirty_and_psf():
    """Dirty image and PSF of a small point-source observation, made by the
    oracle (Stokes I plane)."""
    wl = synth.tiny_workload(n_ant=10, n_time=40, dt_s=300.0, nchan=2, nx=96, ny=96,
                             cell_arcsec=6.0, oversample=20, terms=TERM_PS, n_src=4,
                             sigma=0.002, cfg_id=99)
    ocf = oracle.build_cf(wl.grid, wl.cf)
    pr = Problem.from_workload(wl, ocf)
    c1 = separable_1d(ocf)
    gx = gcf_1d(c1, ocf.O, wl.grid.nx).real
    gy = gcf_1d(c1, ocf.O, wl.grid.ny).real
    corr = np.outer(gy, gx)
    s, _ = pr.sumwt(wl.weight)
    dirty = centred_ifft(pr.grid(wl.vis, wl.weight))[0, 0].real / corr / s[0, 0]
    psfg, s2, _ = pr.psf(wl.weight)
    psf = centred_ifft(psfg)[0, 0].real / corr / s2[0, 0]
    return np.ascontiguousarray(dirty), np.ascontiguousarray(psf)


def run(dirty, psf, dtype, gain, threshold, niter):
    res = torch.as_tensor(dirty, dtype=dtype, device=DEV).contiguous()
    p = torch.as_tensor(psf, dtype=dtype, device=DEV).contiguous()
    model = torch.zeros_like(res)
    it = lr.lr_hogbom(p, res, model, gain, threshold, niter)
    return model.cpu().numpy(), res.cpu().numpy(), it


def test_fp64_identical_to_oracle(dirty_and_psf):
    dirty, psf = dirty_and_psf
    thr = 0.02 * np.max(np.abs(dirty))
    m_ref, r_ref, it_ref = hogbom(dirty, psf, 0.1, thr, 400)
    m, r, it = run(dirty, psf, torch.float64, 0.1, thr, 400)
    print("hogbom iterations", it, it_ref, flush=True)
    assert it == it_ref and it > 20
    assert np.array_equal(m, m_ref)
    assert np.array_equal(r, r_ref)


def test_fp32_within_rounding(dirty_and_psf):
    dirty, psf = dirty_and_psf
    thr = 0.05 * np.max(np.abs(dirty))
    m_ref, r_ref, it_ref = hogbom(dirty, psf, 0.1, thr, 200)
    m, r, it = run(dirty, psf, torch.float32, 0.1, thr, 200)
    assert abs(it - it_ref) <= 2
    assert abs(m.sum() - m_ref.sum()) <= 1e-3 * abs(m_ref.sum())
    assert np.max(np.abs(r - r_ref)) <= 2e-2 * np.max(np.abs(dirty))


def test_budget_threshold_and_argument_checks(dirty_and_psf):
    dirty, psf = dirty_and_psf
    m, r, it = run(dirty, psf, torch.float64, 0.1, 0.0, 0)
    assert it == 0 and not m.any() and np.array_equal(r, dirty)
    m, r, it = run(dirty, psf, torch.float64, 0.1, 2 * np.max(np.abs(dirty)), 100)
    assert it == 0 and not m.any()
    m, r, it = run(dirty, psf, torch.float64, 1.0, 0.0, 1)
    assert it == 1 and np.count_nonzero(m) == 1
    with pytest.raises(lr.LRError) as ei:
        run(dirty, psf, torch.float64, 0.0, 0.0, 10)
    assert ei.value.status == lr.LR_E_ARG


def test_ragged_image_and_ties():
    """Odd sizes (centre at (ny/2, nx/2) with integer division) and an exact
    tie between two peaks: the lower index is cleaned first on both sides."""
    ny, nx = 37, 52
    rng = np.random.default_rng(11)
    psf = np.zeros((ny, nx))
    psf[ny // 2 - 2:ny // 2 + 3, nx // 2 - 3:nx // 2 + 4] = rng.uniform(0.1, 0.5, (5, 7))
    psf[ny // 2, nx // 2] = 1.0
    dirty = rng.normal(0, 0.01, (ny, nx))
    dirty[3, 50] = 1.0
    dirty[30, 2] = -1.0
    m_ref, r_ref, it_ref = hogbom(dirty, psf, 0.3, 0.05, 60)
    m, r, it = run(dirty, psf, torch.float64, 0.3, 0.05, 60)
    assert it == it_ref
    assert np.array_equal(m, m_ref) and np.array_equal(r, r_ref)
