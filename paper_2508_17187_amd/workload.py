"""Move a synthetic workload (any object with the fields of synth.Workload)
onto the device as the binding's descriptors.  Pure marshalling."""

import numpy as np
import torch

from . import lr


def grid_spec(g, nplane=None):
    return lr.GridSpec(g.nx, g.ny, g.npol, g.nplane if nplane is None else nplane,
                       g.cell_l, g.cell_m)


def cf_spec(c, storage):
    return dict(terms=int(c.terms), oversample=int(c.oversample), ps_support=int(c.ps_support),
                n_w=int(c.n_w), w_max=float(c.w_max), h_min=int(c.h_min), h_max=int(c.h_max),
                n_fg=int(len(c.fg_hz)), fg_hz=np.asarray(c.fg_hz, np.float64),
                dish_m=float(c.dish_m), screen_m=int(c.screen_m), storage=int(storage),
                pol_beam=int(getattr(c, "pol_beam", 0)),
                beam_ellipticity=float(getattr(c, "beam_ellipticity", 0.0)),
                beam_leakage=float(getattr(c, "beam_leakage", 0.0)))


def build_cf(wl, precision, device="cuda", stream=None):
    return lr.lr_cf_build(grid_spec(wl.grid), cf_spec(wl.cf, precision), device=device,
                          stream=stream)


def device_vis(wl, precision, device="cuda", pointing=None, with_vis=True, rows=None):
    """lr.Vis over device copies of the workload's arrays.  `rows` selects a
    slice of rows; pointing=None follows the workload, False turns it off."""
    cdt, rdt = (torch.complex128, torch.float64) if precision == lr.LR_F64 else \
        (torch.complex64, torch.float32)
    sl = slice(None) if rows is None else rows
    uvw = torch.as_tensor(np.ascontiguousarray(wl.obs.uvw[sl]), device=device)
    vis = torch.as_tensor(np.ascontiguousarray(wl.vis[sl]), device=device).to(cdt) \
        if with_vis else None
    wt = torch.as_tensor(np.ascontiguousarray(wl.weight[sl]), device=device).to(rdt)
    po = (wl.ant_dlm is not None) if pointing is None else bool(pointing)
    a1 = a2 = dlm = None
    if po:
        a1 = torch.as_tensor(np.ascontiguousarray(wl.obs.ant1[sl]), device=device)
        a2 = torch.as_tensor(np.ascontiguousarray(wl.obs.ant2[sl]), device=device)
        dlm = torch.as_tensor(np.ascontiguousarray(wl.ant_dlm), device=device)
    return lr.Vis(uvw, wl.obs.freq_hz, wl.chan_plane, wl.chan_fg, vis=vis, weight=wt,
                  npol=wl.grid.npol, ant1=a1, ant2=a2, ant_dlm=dlm)


def empty_grid(wl, precision, device="cuda", nplane=None):
    cdt = torch.complex128 if precision == lr.LR_F64 else torch.complex64
    g = wl.grid
    return torch.zeros((g.nplane if nplane is None else nplane, g.npol, g.ny, g.nx),
                       dtype=cdt, device=device)
