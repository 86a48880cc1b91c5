"""Pins of the oracle's Hogbom minor cycle (CPU only)."""

import numpy as np

from oracle.hogbom import hogbom


def delta(ny, nx):
    p = np.zeros((ny, nx))
    p[ny // 2, nx // 2] = 1.0
    return p


def test_delta_psf_converges_geometrically():
    """With a delta PSF one source of flux F leaves (1 - g)^n F after n
    iterations and the model holds the rest, exactly as the loop computes
    it."""
    res = np.zeros((16, 20))
    res[5, 7] = 2.0
    model, r, it = hogbom(res, delta(16, 20), 0.25, 0.0, 10)
    assert it == 10
    left = 2.0
    for _ in range(10):
        left = left - 0.25 * left
    assert r[5, 7] == left and np.count_nonzero(r) == 1
    assert abs(model[5, 7] - (2.0 - left)) < 1e-15 and np.count_nonzero(model) == 1


def test_threshold_exit_and_order_of_components():
    """Two deltas: the larger is cleaned first, and the loop stops once the
    largest residual is below the threshold."""
    res = np.zeros((16, 16))
    res[3, 3] = 1.0
    res[10, 12] = -0.6
    model, r, it = hogbom(res, delta(16, 16), 0.5, 0.2, 100)
    assert np.max(np.abs(r)) < 0.2
    # 1 -> 0.5 -> 0.25 (x), -0.6 -> -0.3 (y), then 0.25 and -0.3 < 0.2? no:
    # order of peaks: 1.0, -0.6, 0.5, -0.3, 0.25, then max 0.15 stops
    assert it == 5
    assert model[3, 3] == 0.5 + 0.25 + 0.125 and model[10, 12] == -0.3 - 0.15


def test_first_index_wins_ties_and_psf_is_centred():
    res = np.zeros((8, 8))
    res[2, 5] = 1.0
    res[6, 1] = -1.0                   # equal |value|, later in row-major order
    psf = np.zeros((8, 8))
    psf[4, 4] = 1.0
    psf[4, 5] = 0.5                    # one pixel right of the centre
    model, r, it = hogbom(res, psf, 1.0, 0.0, 1)
    assert it == 1 and model[2, 5] == 1.0 and model[6, 1] == 0.0
    assert r[2, 5] == 0.0 and r[2, 6] == -0.5 and r[6, 1] == -1.0


def test_flux_is_conserved_with_a_unit_peak_psf():
    """Every iteration moves gain x peak x PSF(centre) = gain x peak from the
    residual peak into the model, so residual + model at the peak pixels is
    the original value when the PSF is a delta; with a wider PSF the sum of
    model components equals the sum of subtracted peaks."""
    rng = np.random.default_rng(3)
    ny, nx = 24, 24
    y, x = np.mgrid[0:ny, 0:nx]
    psf = np.exp(-((y - ny // 2) ** 2 + (x - nx // 2) ** 2) / 3.0)
    res = np.zeros((ny, nx))
    for _ in range(4):
        py, px = rng.integers(4, 20, 2)
        res += rng.uniform(0.5, 1.0) * np.roll(np.roll(psf, py - ny // 2, 0), px - nx // 2, 1)
    model, r, it = hogbom(res, psf, 0.1, 1e-3, 500)
    assert it > 10 and np.max(np.abs(r)) < np.max(np.abs(res))
    # reconvolving the model with the PSF and adding the residual gives the input
    recon = np.zeros_like(res)
    for (py, px) in zip(*np.nonzero(model)):
        recon += model[py, px] * np.roll(np.roll(psf, py - ny // 2, 0), px - nx // 2, 1)
    # the rolls wrap around; inside the inner region they equal the clipped shifts
    inner = (slice(6, 18), slice(6, 18))
    assert np.max(np.abs((recon + r - res)[inner])) < 1e-3
