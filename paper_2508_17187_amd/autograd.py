"""Differentiable degridding.

Eq. ME-MOD-GRIDDED predicts model visibilities as V = D F I (degridding D
of the Fourier transform F of the image); Eq. ImChisq is the weighted chi^2
of V against the data and Eq. ResIm states that its gradient is the
residual image F^dagger G W (V - V_model).  Here D is the forward pass
(lr_degrid) and its hand-written adjoint, unit-weight gridding G_1
(lr_grid with weights 1 on unflagged samples), is the backward pass: for
the complex-linear map y = D x, PyTorch's vector-Jacobian product is
D^H grad_y = G_1 grad_y.

F (centred, unnormalised, image -> grid with exp(-2 pi i (ul + vm))) and
the grid-correction division lie outside the gridding hot path and use
torch.fft.
"""

import torch

from . import lr


class DegridOp:
    """Everything a differentiable degrid needs besides the grid: the CF,
    the visibility descriptor (uvw, channels, flags), precision and the
    workspaces, kept resident between calls."""

    def __init__(self, cf, vis, precision, plan=True):
        self.cf = cf
        self.p = precision
        cdt = torch.complex128 if precision == lr.LR_F64 else torch.complex64
        rdt = torch.float64 if precision == lr.LR_F64 else torch.float32
        self.cdt, self.rdt = cdt, rdt
        dev = vis.uvw.device
        shape = (vis.nrow, vis.nchan, vis.npol)
        # flags come from the weights; the operator itself carries no weights
        self.mask = (vis.weight != 0).to(rdt) if vis.weight is not None else \
            torch.ones(shape, dtype=rdt, device=dev)
        base = vis.with_(vis=None, weight=self.mask, plan=None)
        self.plan = lr.Plan(cf, base) if plan else None
        self.vis = base.with_(plan=self.plan)
        self.shape = shape
        g = cf.grid
        self.grid_shape = (g.nplane, g.npol, g.ny, g.nx)
        self.work_d = lr._work(lr.LR_OP_DEGRID, cf, self.vis, precision, None)
        self.work_g = lr._work(lr.LR_OP_GRID, cf, self.vis, precision, None)

    def degrid(self, grid):
        out = torch.empty(self.shape, dtype=self.cdt, device=grid.device)
        lr.lr_degrid(self.cf, self.vis.with_(vis=out), self.p, grid.contiguous(),
                     work=self.work_d)
        return out

    def grid_adjoint(self, v):
        g = torch.empty(self.grid_shape, dtype=self.cdt, device=v.device)
        lr.lr_grid_overwrite(self.cf, self.vis.with_(vis=v.contiguous()), self.p, g,
                             work=self.work_g)
        return g


class Degrid(torch.autograd.Function):
    """V = D(grid); backward: grad_grid = G_1(grad_V)."""

    @staticmethod
    def forward(ctx, grid, op):
        ctx.op = op
        return op.degrid(grid.to(op.cdt))

    @staticmethod
    def backward(ctx, grad_v):
        return ctx.op.grid_adjoint(grad_v.to(ctx.op.cdt)), None


_CHECKER = {}


def _checker(ny, nx, dtype, device):
    """(-1)^(y + x) over an ny x nx plane, and the same times (-1)^((ny + nx)/2)."""
    key = (ny, nx, dtype, str(device))
    if key not in _CHECKER:
        y = torch.arange(ny, device=device).view(ny, 1)
        x = torch.arange(nx, device=device).view(1, nx)
        c = (1 - 2 * ((y + x) % 2)).to(dtype)
        _CHECKER[key] = (c, c * (1 - 2 * (((ny + nx) // 2) % 2)))
    return _CHECKER[key]


def _real_dtype(t):
    return t.real.dtype if t.is_complex() else t.dtype


def centred_fft2(img):
    """F: grid[v][u] = sum_pix img[m][l] exp(-2 pi i (u l + v m)), pixel n/2 at 0.
    For even sizes the centring shifts are a (-1)^(y + x) factor on either
    side of the plain transform (with the sign i^(ny + nx)): two elementwise
    passes instead of four rolls and a copy."""
    ny, nx = img.shape[-2:]
    if ny % 2 or nx % 2:
        return torch.fft.fftshift(torch.fft.fft2(torch.fft.ifftshift(img, dim=(-2, -1))),
                                  dim=(-2, -1))
    c, cs = _checker(ny, nx, _real_dtype(img), img.device)
    return torch.fft.fft2(img * c) * cs


def centred_ifft2(grid):
    """F^dagger, unnormalised (the same centring factors, and no 1/n)."""
    ny, nx = grid.shape[-2:]
    if ny % 2 or nx % 2:
        return torch.fft.fftshift(torch.fft.ifft2(torch.fft.ifftshift(grid, dim=(-2, -1))),
                                  dim=(-2, -1)) * (nx * ny)
    c, cs = _checker(ny, nx, _real_dtype(grid), grid.device)
    return torch.fft.ifft2(grid * c, norm="forward") * cs


def predict(image, op, gamma=None):
    """Model visibilities D F (gamma * image) for a real image
    [nplane, npol, ny, nx]; gamma is the grid-correction weight (1/gcf) or
    None."""
    x = image if gamma is None else image * gamma
    grid = centred_fft2(x.to(op.cdt))
    return Degrid.apply(grid, op)


class WeightedResidual(torch.autograd.Function):
    """sum W |V_obs - V|^2 in three passes (the residual, its weighting and
    one dot product) with a one-pass backward: for a real loss of complex V
    PyTorch's gradient is 2 dL/d conj(V) = -2 W (V_obs - V)."""

    @staticmethod
    def forward(ctx, v, vis_obs, weight):
        r = vis_obs - v
        wr = r * weight
        ctx.save_for_backward(r, wr)
        return torch.vdot(r.reshape(-1), wr.reshape(-1)).real

    @staticmethod
    def backward(ctx, g):
        r, wr = ctx.saved_tensors
        gv = -2.0 * g * wr if ctx.needs_input_grad[0] else None
        go = 2.0 * g * wr if ctx.needs_input_grad[1] else None
        gw = g * (r.real ** 2 + r.imag ** 2) if ctx.needs_input_grad[2] else None
        return gv, go, gw


def chi2(image, op, vis_obs, weight, gamma=None):
    """Eq. ImChisq: sum W |V_obs - D F gamma I|^2."""
    return WeightedResidual.apply(predict(image, op, gamma), vis_obs, weight)
