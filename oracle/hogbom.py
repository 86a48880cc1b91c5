"""Hogbom minor cycle (the ModelUpdate step of the imaging section, with a
loop gain and a threshold exit) -- test infrastructure only.

One plane, FP64, in the plainest form: find the pixel of largest |residual|
(the first in row-major order on ties); stop if it is below the threshold or
the iteration budget is spent; otherwise add gain x peak to the model there
and subtract gain x peak x PSF, the PSF's centre (ny/2, nx/2) placed on the
peak, from the overlapping part of the residual.
"""

import numpy as np


def hogbom(residual, psf, gain, threshold, niter):
    """Returns (model, residual, iterations done)."""
    res = np.array(residual, np.float64, copy=True)
    psf = np.asarray(psf, np.float64)
    ny, nx = res.shape
    cy, cx = ny // 2, nx // 2
    model = np.zeros_like(res)
    it = 0
    while True:
        idx = int(np.argmax(np.abs(res)))
        peak = res.flat[idx]
        if abs(peak) < threshold or it >= niter:
            break
        c = gain * peak
        py, px = divmod(idx, nx)
        model[py, px] += c
        # residual pixel (y, x) takes PSF pixel (y - py + cy, x - px + cx)
        y0, y1 = max(0, py - cy), min(ny, py - cy + ny)
        x0, x1 = max(0, px - cx), min(nx, px - cx + nx)
        res[y0:y1, x0:x1] -= c * psf[y0 - py + cy:y1 - py + cy, x0 - px + cx:x1 - px + cx]
        it += 1
    return model, res, it
