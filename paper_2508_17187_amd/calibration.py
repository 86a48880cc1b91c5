"""Diagonal G-Jones calibration (the calibration section, the solver of the
calibration figure): model prediction by the library's degridder, then the
ratio averages, update direction, damped update and exit test on the GPU.

    PreCompute    V^Mod = D F (Gamma I^Mod)           imaging.predict
    PreSolvePrep  X_ij, w_ij per interval (Eq. VAvg)    lr_cal_vavg
    UpdateDir / ModelUpdate / ExitCriteria
                  (Eqs. CalUpdateDir, CalUpdateModel) lr_cal_solve

V^c is the observed data itself: no earlier calibration term is applied.
"""

from dataclasses import dataclass

import torch

from . import lr
from .imaging import predict


@dataclass
class GainSolution:
    g: torch.Tensor            # complex128 [n_tsol, n_fsol, npar, nant]
    iterations: torch.Tensor   # int32 [n_tsol, n_fsol, npar]
    change: torch.Tensor       # float64 [n_tsol, n_fsol, npar], last max |change|
    X: torch.Tensor            # complex128 [n_tsol, n_fsol, npar, nant, nant]
    w: torch.Tensor            # float64, same shape


def solve_gains(vis_obs, vis_model, weight, ant1, ant2, nant, row_sol, n_tsol, chan_sol,
                n_fsol, rows_per_step=1, alpha=0.5, delta=1e-10, max_iter=500, g0=None,
                stream=None):
    """Antenna gains per solution interval and parallel hand from observed
    and model visibilities [nrow, nchan, npol] (device)."""
    X, w = lr.lr_cal_vavg(vis_obs, vis_model, weight, ant1, ant2, nant, row_sol, n_tsol,
                          chan_sol, n_fsol, rows_per_step=rows_per_step, stream=stream)
    g, it, ch = lr.lr_cal_solve(X, w, g0=g0, alpha=alpha, delta=delta, max_iter=max_iter,
                                stream=stream)
    return GainSolution(g, it, ch, X, w)


def calibrate(cf, vis, precision, model, ant1, ant2, nant, row_sol, n_tsol, chan_sol, n_fsol,
              rows_per_step=1, alpha=0.5, delta=1e-10, max_iter=500, gcf=None, op=None):
    """The whole solver: predict the model visibilities of `model` (a real
    image [nplane, npol, ny, nx]) for the samples of `vis` with the
    degridder, then solve for the gains that map them onto vis.vis."""
    vmod = predict(cf, vis, precision, model, gcf=gcf, op=op)
    sol = solve_gains(vis.vis, vmod, vis.weight, ant1, ant2, nant, row_sol, n_tsol, chan_sol,
                      n_fsol, rows_per_step=rows_per_step, alpha=alpha, delta=delta,
                      max_iter=max_iter)
    return sol, vmod
