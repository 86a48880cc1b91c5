"""Image-plane helpers for the oracle's pins (test infrastructure only).

F (image -> visibility plane) uses exp(-2 pi i (u l + v m)), F^dagger uses
exp(+2 pi i (u l + v m)); both unnormalised and centred (pixel nx/2 is the
origin), matching the index convention of the oracle's gridder.  Eq. ResIm
gives the residual image as F^dagger G W (V - V_model); Eq. ImChisq gives
the imaging chi^2 whose gradient it is proportional to.
"""

import numpy as np

from .cfbuild import airy_power
from .conventions import C_LIGHT
from .pswf import pswf_nystrom


def centred_fft(img):
    """F: grid[v][u] = sum_pix img[m][l] exp(-2 pi i (u l + v m))."""
    return np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(img, axes=(-2, -1)),
                                       axes=(-2, -1)), axes=(-2, -1))


def centred_ifft(grid):
    """F^dagger, unnormalised: img[m][l] = sum_cells grid exp(+2 pi i (u l + v m))."""
    n = grid.shape[-1] * grid.shape[-2]
    return np.fft.fftshift(np.fft.ifft2(np.fft.ifftshift(grid, axes=(-2, -1)),
                                        axes=(-2, -1)), axes=(-2, -1)) * n


def response_1d(c1_o, O, o, n):
    """Image-plane response of one sample at offset o through the 1-D kernel
    c1_o (taps t = -h..h): sum_t c1[t] exp(2 pi i (t - o/O) xi), xi =
    (ix - n/2)/n."""
    h = (len(c1_o) - 1) // 2
    t = np.arange(-h, h + 1)
    xi = (np.arange(n) - n // 2) / n
    return np.exp(2j * np.pi * np.outer(xi, t - o / O)) @ c1_o


def gcf_1d(c1, O, n):
    """Grid correction: mean over o in [-O/2, O/2) of response_1d; c1 is the
    separable 1-D table [O+1][S] for offsets -O/2..O/2."""
    acc = np.zeros(n, np.complex128)
    for i, o in enumerate(range(-(O // 2), O // 2)):
        acc += response_1d(c1[i], O, o, n)
    return acc / O


def separable_1d(ocf, k=0, fg=0):
    """Recover the 1-D kernel of a separable (PS-only) table:
    C[ov][ou][tv][tu] = c1[ov][tv] c1[ou][tu]; with c1[o][t] taken from the
    o_v = 0, t_v = 0 slice divided by its centre value."""
    pl = ocf.plane(fg, k)
    O = ocf.O
    h = (pl.shape[-1] - 1) // 2
    mid = O // 2
    c00 = pl[mid, mid, h, h]
    s = np.sqrt(c00)
    c1 = pl[mid, :, h, :] / s          # [ou][tu] = c1[0][h] c1[ou][tu] / s
    return c1


def dft_image(uvw_m, freq_hz, vis, weight, nx, ny, cell_l, cell_m, pol=0):
    """Direct Fourier image sum W V exp(+2 pi i (u l + v m)) / sum W over
    every (row, chan) sample of one polarisation (w ignored)."""
    ix = (np.arange(nx) - nx // 2) * cell_l
    iy = (np.arange(ny) - ny // 2) * cell_m
    img = np.zeros((ny, nx), np.complex128)
    sw = 0.0
    for c, nu in enumerate(freq_hz):
        u = uvw_m[:, 0] * nu / C_LIGHT
        v = uvw_m[:, 1] * nu / C_LIGHT
        a = weight[:, c, pol] * vis[:, c, pol]
        ex = np.exp(2j * np.pi * np.outer(u, ix))      # [rows][l]
        ey = np.exp(2j * np.pi * np.outer(v, iy))      # [rows][m]
        img += (ey * a[:, None]).T @ ex
        sw += weight[:, c, pol].sum()
    return img / sw


def chi2(vis_obs, weight, vis_model):
    r = vis_obs - vis_model
    return float(np.sum(weight * (r.real ** 2 + r.imag ** 2)))


def ps_taper(n, ps_support):
    """The PS term's image-plane taper at n pixels: psi_0(c, 2 (i - n/2) / n),
    c = pi S_ps / 2 (Table AWP-CFSETUP, PS; the screen's own sampling of it,
    evaluated at the image pixels): the grid correction of tables whose
    planes are not separable."""
    psi = pswf_nystrom(np.pi * ps_support / 2.0)[0]
    return psi(2.0 * (np.arange(n) - n // 2) / n)


def pb_image(nx, ny, cell_l, cell_m, fg_hz, dish_m, fg_weight):
    """Weight image of A-projection (the primary-beam normalisation of
    Eq. ResIm's image when G carries the A term, Table AWP-CFSETUP): the
    data hold the beam B_fg once and the kernel of G applies it again, so a
    source at (l, m) images with sum_fg w_fg B_fg(rho)^2 / sum_fg w_fg,
    B_fg(rho) = [2 J1(x)/x]^2 at x = pi D nu_fg rho / c, rho = sqrt(l^2 +
    m^2), (l, m) = ((ix - nx/2) dl, (iy - ny/2) dm).  fg_weight: [..., n_fg]
    sums of weights per frequency group; returns [..., ny, nx] (0 where the
    weights sum to 0)."""
    w = np.asarray(fg_weight, np.float64)
    l = (np.arange(nx) - nx // 2) * cell_l
    m = (np.arange(ny) - ny // 2) * cell_m
    rho = np.sqrt(l[None, :] ** 2 + m[:, None] ** 2)
    b2 = np.stack([airy_power(np.pi * dish_m * nu * rho / C_LIGHT) ** 2 for nu in fg_hz])
    tot = w.sum(-1)
    num = np.tensordot(w, b2, axes=([-1], [0]))
    out = np.zeros(num.shape)
    ok = tot > 0
    out[ok] = num[ok] / tot[ok][..., None, None]
    return out


def normalise_aw(img, taper_x, taper_y, sumwt, pb, pb_min):
    """Re(img) / (taper_x taper_y sumwt pb) where pb >= pb_min, 0 elsewhere;
    img [..., ny, nx] with sumwt [...] and pb [..., ny, nx]."""
    d = taper_y[:, None] * taper_x[None, :] * np.asarray(sumwt)[..., None, None] * pb
    out = np.zeros(np.shape(pb))
    ok = pb >= pb_min
    out[ok] = np.real(img)[ok] / d[ok]
    return out
