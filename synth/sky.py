"""Point-source skies and their visibilities by a direct Fourier sum.

V(u, v, w) = sum_s S_s exp(-2 pi i (u l_s + v m_s + w (n_s - 1))), with
(u, v, w) in wavelengths and n = sqrt(1 - l^2 - m^2): the measurement
equation (Eq. ME) with identity Mueller matrices and the image-to-visibility
sign convention used throughout this repository.  Parallel-hand
correlations carry V, cross-hands carry 0.
"""

from dataclasses import dataclass

import numpy as np

from .observation import C_LIGHT, DEG


@dataclass
class PointSky:
    l: np.ndarray      # direction cosines
    m: np.ndarray
    flux: np.ndarray   # Jy

    @property
    def n(self):
        return self.l.shape[0]


def random_point_sky(n_src, seed, half_width_deg=0.5, flux_lo=0.1, flux_hi=1.0,
                     log_flux=False):
    """(l, m) uniform in [-hw, hw]^2 degrees; flux uniform (or log-uniform)."""
    rng = np.random.default_rng(seed)
    l = np.sin(rng.uniform(-half_width_deg, half_width_deg, n_src) * DEG)
    m = np.sin(rng.uniform(-half_width_deg, half_width_deg, n_src) * DEG)
    if log_flux:
        flux = 10.0 ** rng.uniform(np.log10(flux_lo), np.log10(flux_hi), n_src)
    else:
        flux = rng.uniform(flux_lo, flux_hi, n_src)
    return PointSky(l=l, m=m, flux=flux)


def _pol_layout(npol):
    """Which correlations are parallel hands (carry V)."""
    if npol == 1:
        return [True]
    if npol == 2:
        return [True, True]
    if npol == 4:
        return [True, False, False, True]   # XX XY YX YY
    raise ValueError("npol must be 1, 2 or 4")


def dft_visibilities(uvw_m, freq_hz, sky, npol, row_block=32768, device="cpu"):
    """Direct sum over sources for every (row, channel); returns
    complex128 [nrow, nchan, npol] as a numpy array.  The sum runs in
    float64 with torch on `device` (the CPU by default)."""
    import torch
    nrow = uvw_m.shape[0]
    nchan = freq_hz.shape[0]
    out = np.zeros((nrow, nchan, npol), dtype=np.complex128)
    par = _pol_layout(npol)
    dev = torch.device(device)
    l = torch.as_tensor(sky.l, dtype=torch.float64, device=dev)
    m = torch.as_tensor(sky.m, dtype=torch.float64, device=dev)
    nm1 = torch.sqrt(1.0 - l * l - m * m) - 1.0
    flux = torch.as_tensor(sky.flux, dtype=torch.float64, device=dev)
    scale = torch.as_tensor(-2.0 * np.pi * freq_hz / C_LIGHT, dtype=torch.float64,
                            device=dev)
    for r0 in range(0, nrow, row_block):
        r1 = min(nrow, r0 + row_block)
        uvw = torch.as_tensor(uvw_m[r0:r1], dtype=torch.float64, device=dev)
        # geometric delay in metres for every (row, source)
        ph = (torch.outer(uvw[:, 0], l) + torch.outer(uvw[:, 1], m)
              + torch.outer(uvw[:, 2], nm1))
        arg = ph[:, None, :] * scale[None, :, None]        # [rows, nchan, nsrc]
        vr = torch.cos(arg) @ flux
        vi = torch.sin(arg) @ flux
        val = (vr + 1j * vi).cpu().numpy()
        for p in range(npol):
            if par[p]:
                out[r0:r1, :, p] = val
    return out


def add_noise(vis, sigma, seed):
    """Complex Gaussian noise, sigma per real and imaginary part; returns
    (noisy vis, natural weights 1/sigma^2)."""
    rng = np.random.default_rng(seed)
    n = rng.standard_normal(vis.shape) + 1j * rng.standard_normal(vis.shape)
    wt = np.full(vis.shape, 1.0 / (sigma * sigma))
    return vis + sigma * n, wt
