"""Differentiable degridding on the GPU: the hand-written adjoint (gridding)
as the backward pass, checked by the adjoint identity, by central finite
differences of the quadratic chi^2 (Eq. ImChisq) and against the oracle's
gradient (Eq. ResIm)."""

import numpy as np
import pytest

import synth
import oracle
from oracle.cfbuild import TERM_A, TERM_PS, TERM_W
from oracle.imaging import centred_fft, centred_ifft
from oracle.native import Problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2508_17187_amd import lr  # noqa: E402
from paper_2508_17187_amd import workload as W  # noqa: E402
from paper_2508_17187_amd.autograd import Degrid, DegridOp, chi2  # noqa: E402

DEV = "cuda"


@pytest.fixture(scope="module")
def case():
    wl = synth.tiny_workload(n_w=4, h_min=3, h_max=6, oversample=8,
                             terms=TERM_PS | TERM_W | TERM_A, nchan=3, n_time=10, nx=64, ny=64,
                             cell_arcsec=8.0, diameter_m=4000.0, cfg_id=93,
                             pointing_sigma=2e-5)
    rng = np.random.default_rng(93)
    wl.weight[rng.random(wl.weight.shape) < 0.05] = 0.0
    wl.weight *= rng.uniform(0.5, 1.5, wl.weight.shape)
    return wl


def make_op(wl, p):
    cf = W.build_cf(wl, p)
    v = W.device_vis(wl, p)
    return DegridOp(cf, v, p), v


def test_adjoint_identity_through_autograd(case):
    wl = case
    op, v = make_op(wl, lr.LR_F64)
    rng = np.random.default_rng(1)
    x = torch.as_tensor(rng.standard_normal(op.grid_shape) + 1j * rng.standard_normal(op.grid_shape),
                        device=DEV).requires_grad_(True)
    y = torch.as_tensor(rng.standard_normal(op.shape) + 1j * rng.standard_normal(op.shape),
                        device=DEV)
    dx = Degrid.apply(x, op)
    (gy,) = torch.autograd.grad(dx, x, grad_outputs=y)
    lhs = torch.vdot(dx.detach().flatten(), y.flatten()).item()
    rhs = torch.vdot(x.detach().flatten(), gy.flatten()).item()
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


@pytest.mark.parametrize("form,tol", [("f64", 1e-7), ("f32", 2e-2)])
def test_chi2_gradient_vs_finite_differences(case, form, tol):
    wl = case
    p = lr.PRECISIONS[form]
    op, v = make_op(wl, p)
    rng = np.random.default_rng(2)
    shape = (wl.grid.nplane, wl.grid.npol, wl.grid.ny, wl.grid.nx)
    dt = torch.float64 if p == lr.LR_F64 else torch.float32
    gamma = torch.as_tensor(1.0 + 0.2 * rng.random(shape[-2:]), device=DEV, dtype=dt)
    img = torch.as_tensor(0.01 * rng.standard_normal(shape), device=DEV, dtype=dt)
    img.requires_grad_(True)
    vobs, wt = v.vis, v.weight
    loss = chi2(img, op, vobs, wt, gamma)
    (grad,) = torch.autograd.grad(loss, img)
    eps = 0.05 if form == "f64" else 0.5
    gmax = grad.abs().max().item()
    pix = [tuple(int(a) for a in (0, rng.integers(shape[1]), rng.integers(16, 48),
                                   rng.integers(16, 48))) for _ in range(64)]
    for j in pix:
        e = torch.zeros_like(img)
        e[j] = eps
        with torch.no_grad():
            fd = (chi2(img + e, op, vobs, wt, gamma) - chi2(img - e, op, vobs, wt, gamma)) / (2 * eps)
        assert abs(fd.item() - grad[j].item()) <= tol * gmax, (j, fd.item(), grad[j].item())


def test_gradient_matches_the_oracle(case):
    wl = case
    p = lr.LR_F64
    op, v = make_op(wl, p)
    rng = np.random.default_rng(3)
    shape = (wl.grid.nplane, wl.grid.npol, wl.grid.ny, wl.grid.nx)
    gamma = 1.0 + 0.2 * rng.random(shape[-2:])
    img = 0.01 * rng.standard_normal(shape)
    it = torch.as_tensor(img, device=DEV).requires_grad_(True)
    loss = chi2(it, op, v.vis, v.weight, torch.as_tensor(gamma, device=DEV))
    (grad,) = torch.autograd.grad(loss, it)
    ocf = oracle.build_cf(wl.grid, wl.cf)
    pr = Problem.from_workload(wl, ocf)
    model = pr.degrid(centred_fft(gamma * img), wl.weight)
    r = wl.weight * (wl.vis - model)
    ref = -2 * np.real(gamma * centred_ifft(pr.grid(r, (wl.weight != 0).astype(float))))
    got = grad.cpu().numpy()
    assert np.linalg.norm(got - ref) <= 1e-10 * np.linalg.norm(ref)
