"""Residual and dirty images around the hot path (Eq. ResIm, the step of
UpdateDir after G): grid the (residual) visibilities with
lr_grid_overwrite, take F^dagger of the grid with rocFFT (torch.fft), and
normalise by the grid correction of the kernel's separable plane and the sum
of weights with lr_image_normalize.  The model prediction for the residual
is D F (Gamma I), Gamma = 1 / (gcf_x gcf_y), as in Eq. ImChisq.
"""

import torch

from . import lr
from .autograd import DegridOp, centred_fft2, centred_ifft2


def grid_correction(cf, fg=0, k=0, device="cuda"):
    """(gcf_x [nx], gcf_y [ny]) as FP64 real tensors."""
    g = cf.grid
    gx = lr.lr_gcf(cf, g.nx, fg, k, device=device).real.contiguous()
    gy = lr.lr_gcf(cf, g.ny, fg, k, device=device).real.contiguous()
    return gx, gy


def dirty_image(cf, vis, precision, gcf=None, work=None):
    """Image of vis: Re F^dagger G(W V) / (gcf_x gcf_y sumwt), shape
    [nplane, npol, ny, nx]; returns (image, sumwt)."""
    g = cf.grid
    cdt = torch.complex128 if precision == lr.LR_F64 else torch.complex64
    dev = vis.uvw.device
    grid = torch.empty((g.nplane, g.npol, g.ny, g.nx), dtype=cdt, device=dev)
    sumwt = torch.empty((g.nplane, g.npol), dtype=torch.float64, device=dev)
    lr.lr_grid_overwrite(cf, vis, precision, grid, sumwt=sumwt, work=work)
    img = centred_ifft2(grid).contiguous()
    gx, gy = grid_correction(cf, device=dev) if gcf is None else gcf
    return lr.lr_image_normalize(cf, precision, img, gx, gy, sumwt), sumwt


def predict(cf, vis, precision, model, gcf=None, op=None):
    """Model visibilities D F (Gamma I) of a real model image I [nplane,
    npol, ny, nx] (Eq. VMod, with the grid correction Gamma = 1 / (gcf_x
    gcf_y) of Eq. ImChisq), [nrow, nchan, npol]; flagged samples are 0."""
    gx, gy = grid_correction(cf, device=vis.uvw.device) if gcf is None else gcf
    if op is None:
        op = DegridOp(cf, vis, precision)
    gamma = 1.0 / (gy[:, None] * gx[None, :])
    return op.degrid(centred_fft2((model * gamma).to(op.cdt)))


def residual_image(cf, vis, precision, model, gcf=None, op=None):
    """Image of V - D F (Gamma I) for a real model image I [nplane, npol,
    ny, nx] (Eq. ResIm); returns (image, sumwt).  op: a DegridOp of the
    same data to reuse across major cycles."""
    gx, gy = grid_correction(cf, device=vis.uvw.device) if gcf is None else gcf
    pred = predict(cf, vis, precision, model, gcf=(gx, gy), op=op)
    return dirty_image(cf, vis.with_(vis=(vis.vis - pred).contiguous()), precision,
                       gcf=(gx, gy))
