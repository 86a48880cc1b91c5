"""Mosaic imaging: the mosaic rows of the imaging-mode table (Eq. CIJ).

Each row belongs to a field (pointing) P whose phase centre s(P) lies at
(l_P, m_P) from the joint image centre s0.  Gridding moves the field's
visibilities to s0 (lr_rephase) and shifts its kernels by s(P) - s0 plus the
antennas' mean pointing offset: the pointing phasor of lr_grid / lr_degrid
on virtual antennas f * nant + a whose offsets are ant_dlm[a] +
field_dlm[f] (the loss factor depends on ds_i - ds_j only, so it is
unchanged).  Degridding applies the same kernels and moves the predicted
visibilities back to each field's phase centre.  Without antenna offsets
this is the "no PO correction" row, with them the "with PO correction" row.
"""

import torch

from . import lr


def virtual_antennas(ant1, ant2, nant, field, field_dlm, ant_dlm=None):
    """Device tensors (ant1', ant2' int32 [nrow], ant_dlm' float64
    [nfield * nant, 2])."""
    f = field.to(torch.int64)
    a1 = (f * nant + ant1.to(torch.int64)).to(torch.int32).contiguous()
    a2 = (f * nant + ant2.to(torch.int64)).to(torch.int32).contiguous()
    base = torch.zeros((nant, 2), dtype=torch.float64, device=field.device) if ant_dlm is None \
        else ant_dlm.to(torch.float64)
    dlm = (field_dlm.to(torch.float64)[:, None, :] + base[None, :, :]).reshape(-1, 2).contiguous()
    return a1, a2, dlm


class Mosaic:
    """The fields of one data set: row field ids (int32 [nrow]), field phase
    centres (float64 [nfield, 2]) and, optionally, antenna pointing
    offsets (float64 [nant, 2]); builds the virtual-antenna view of a Vis."""

    def __init__(self, field, field_dlm, ant1, ant2, nant, ant_dlm=None):
        self.field = field.to(torch.int32).contiguous()
        self.field_dlm = field_dlm.to(torch.float64).contiguous()
        self.ant1, self.ant2, self.dlm = virtual_antennas(ant1, ant2, nant, self.field,
                                                          self.field_dlm, ant_dlm)

    def vis(self, vis, values=None, plan=None):
        """A Vis of the same samples with the virtual antennas (and other
        visibility values, e.g. a rephased copy)."""
        return lr.Vis(vis.uvw, vis.freq, vis.chan_plane, vis.chan_fg,
                      vis=vis.vis if values is None else values, weight=vis.weight,
                      npol=vis.npol, ant1=self.ant1, ant2=self.ant2, ant_dlm=self.dlm, plan=plan)

    def to_image_centre(self, vis, values):
        """A copy of values [nrow, nchan, npol] moved to the image centre."""
        out = values.clone().contiguous()
        return lr.lr_rephase(out, vis.uvw, vis.freq, self.field, self.field_dlm, True)

    def to_field_centres(self, vis, values):
        """values moved (in place) from the image centre back to each field's
        phase centre."""
        return lr.lr_rephase(values, vis.uvw, vis.freq, self.field, self.field_dlm, False)

    def grid(self, cf, vis, precision, grid, plan=None, overwrite=True, **kw):
        """G of the mosaic: grid (= or +=) the fields' visibilities at s0."""
        v = self.vis(vis, self.to_image_centre(vis, vis.vis), plan=plan)
        f = lr.lr_grid_overwrite if overwrite else lr.lr_grid
        f(cf, v, precision, grid, **kw)
        return grid

    def degrid(self, cf, vis, precision, grid, plan=None, **kw):
        """D of the mosaic: model visibilities of grid at each field's phase
        centre, [nrow, nchan, npol]."""
        out = torch.empty((vis.nrow, vis.nchan, vis.npol),
                          dtype=torch.complex128 if precision == lr.LR_F64 else torch.complex64,
                          device=grid.device)
        lr.lr_degrid(cf, self.vis(vis, out, plan=plan), precision, grid, **kw)
        return self.to_field_centres(vis, out)
