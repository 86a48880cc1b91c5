"""Residual and dirty images around the hot path (Eq. ResIm, the step of
UpdateDir after G): grid the (residual) visibilities with
lr_grid_overwrite, take F^dagger of the grid with rocFFT (torch.fft), and
normalise by the grid correction of the kernel's separable plane and the sum
of weights with lr_image_normalize.  The model prediction for the residual
is D F (Gamma I), Gamma = 1 / (gcf_x gcf_y), as in Eq. ImChisq.

With A-projection kernels (Table AWP-CFSETUP, A term on) the planes are not
separable: the grid correction is the PS taper the kernels carry
(lr_ps_taper), and the image is also divided by the weight image
(lr_pb_image, from the sums of weights of every frequency group) where it
is at least pb_min (lr_image_normalize_pb).
"""

import numpy as np
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


def fg_weight_sums(cf, vis, precision):
    """Sums of weights of every frequency group's channels, float64
    [nplane, npol, n_fg] (lr_sumwt on each group's channels)."""
    g = cf.grid
    n_fg = cf.spec.n_fg
    dev = vis.uvw.device
    chan_fg = np.zeros(vis.nchan, np.int32) if vis.chan_fg is None else vis.chan_fg
    out = torch.zeros((g.nplane, g.npol, n_fg), dtype=torch.float64, device=dev)
    for k in range(n_fg):
        cp = np.where(chan_fg == k, vis.chan_plane, -1).astype(np.int32)
        if not (cp >= 0).any():
            continue
        s = torch.zeros((g.nplane, g.npol), dtype=torch.float64, device=dev)
        lr.lr_sumwt(cf, vis.with_(chan_plane=cp, plan=None), precision, s)
        out[:, :, k] = s
    return out


def aw_normalisation(cf, vis, precision):
    """(taper_x, taper_y, weight image) of an A-projection table for these
    data: the PS taper at the image pixels and lr_pb_image of the groups'
    sums of weights."""
    g = cf.grid
    dev = vis.uvw.device
    tx = lr.lr_ps_taper(cf, g.nx, device=dev)
    ty = lr.lr_ps_taper(cf, g.ny, device=dev)
    return tx, ty, lr.lr_pb_image(cf, fg_weight_sums(cf, vis, precision))


def dirty_image_aw(cf, vis, precision, pb_min=0.1, norm=None, work=None):
    """Image of vis through A-projection kernels: Re F^dagger G(W V) /
    (taper_x taper_y sumwt pb) where pb >= pb_min, else 0; returns (image,
    sumwt).  norm: aw_normalisation() of the same data, to reuse."""
    g = cf.grid
    cdt = torch.complex128 if precision == lr.LR_F64 else torch.complex64
    dev = vis.uvw.device
    tx, ty, pb = aw_normalisation(cf, vis, precision) if norm is None else norm
    grid = torch.empty((g.nplane, g.npol, g.ny, g.nx), dtype=cdt, device=dev)
    sumwt = torch.empty((g.nplane, g.npol), dtype=torch.float64, device=dev)
    lr.lr_grid_overwrite(cf, vis, precision, grid, sumwt=sumwt, work=work)
    img = centred_ifft2(grid).contiguous()
    return lr.lr_image_normalize_pb(cf, precision, img, tx, ty, sumwt, pb, pb_min), sumwt


def residual_image_aw(cf, vis, precision, model, pb_min=0.1, norm=None, op=None):
    """Image of V - D F (Gamma I) through A-projection kernels, Gamma = 1 /
    (taper_x taper_y): the model image I is the sky (D applies the beam);
    returns (image, sumwt)."""
    tx, ty, pb = aw_normalisation(cf, vis, precision) if norm is None else norm
    pred = predict(cf, vis, precision, model, gcf=(tx, ty), op=op)
    return dirty_image_aw(cf, vis.with_(vis=(vis.vis - pred).contiguous()), precision,
                          pb_min=pb_min, norm=(tx, ty, pb))
