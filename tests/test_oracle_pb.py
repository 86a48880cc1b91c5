"""Oracle pins of the A-projection weight image and the PS taper (the image
normalisation of Eq. ResIm when the kernels of G carry the A term, Table
AWP-CFSETUP A-Projection rows).

* The PS taper at the image pixels is the screen's own taper: psi_0(c, 0)
  = 1 at the centre, even, and equal to the Nystrom prolate at 2 xi.
* The weight image is 1 at the phase centre (B(0) = 1), the square of the
  Airy power pattern for one frequency group, radially symmetric, between
  its groups' values for several, and 0 at the pattern's first null.
* End to end: a point source half-way down the beam, with visibilities
  attenuated by the beam (the measurement equation), gridded by the
  oracle through PS * A kernels and transformed, comes back at its flux
  when the image is divided by taper x taper x sumwt x weight image;
  dividing by the beam once instead of its square leaves it at about half.
"""

import numpy as np
import pytest
from scipy import special

import oracle
import synth
from oracle.cfbuild import TERM_A, TERM_PS, airy_power
from oracle.conventions import C_LIGHT
from oracle.imaging import centred_ifft, normalise_aw, pb_image, ps_taper
from oracle.native import Problem
from oracle.pswf import pswf_nystrom


def test_ps_taper_is_the_prolate_at_the_pixels():
    n = 96
    t = ps_taper(n, 7)
    assert t[n // 2] == pytest.approx(1.0, abs=1e-15)
    assert np.allclose(t[1:], t[1:][::-1], atol=1e-15)          # even about pixel n/2
    psi = pswf_nystrom(np.pi * 7 / 2.0, n_nodes=96)[0]
    x = 2.0 * (np.arange(n) - n // 2) / n
    assert np.max(np.abs(t - psi(x))) < 1e-12


def test_weight_image_closed_forms():
    nx, ny, cell = 64, 48, 30.0 * np.pi / 180 / 3600
    fg = np.array([2.5e9, 3.5e9])
    pb1 = pb_image(nx, ny, cell, cell, fg[:1], 25.0, [1.0])
    assert pb1[ny // 2, nx // 2] == 1.0
    l = (np.arange(nx) - nx // 2) * cell
    m = (np.arange(ny) - ny // 2) * cell
    rho = np.sqrt(l[None, :] ** 2 + m[:, None] ** 2)
    x = np.pi * 25.0 * fg[0] * rho / C_LIGHT
    b = np.where(x == 0, 1.0, (2 * special.j1(np.where(x == 0, 1, x)) / np.where(x == 0, 1, x)) ** 2)
    assert np.max(np.abs(pb1 - b * b)) < 1e-15
    # radial symmetry: (l, m) -> (m, l) on a square patch
    sq = pb_image(64, 64, cell, cell, fg, 25.0, [0.3, 0.7])
    assert np.allclose(sq, sq.T, atol=1e-15)
    # two groups: a weighted mean of the groups' squares, between them
    pb2 = pb_image(nx, ny, cell, cell, fg, 25.0, [1.0, 3.0])
    g0 = pb_image(nx, ny, cell, cell, fg[:1], 25.0, [1.0])
    g1 = pb_image(nx, ny, cell, cell, fg[1:], 25.0, [1.0])
    assert np.max(np.abs(pb2 - (g0 + 3 * g1) / 4)) < 1e-15
    assert np.all(pb2 <= np.maximum(g0, g1) + 1e-15) and np.all(pb2 >= np.minimum(g0, g1) - 1e-15)
    # weights per plane / pol: leading axes carried through; no weight -> 0
    many = pb_image(nx, ny, cell, cell, fg, 25.0, [[1.0, 0.0], [0.0, 0.0]])
    assert many.shape == (2, ny, nx) and np.array_equal(many[1], np.zeros((ny, nx)))
    assert np.max(np.abs(many[0] - g0)) < 1e-15
    # the first null of the Airy pattern, x = 3.8317...
    r0 = special.jn_zeros(1, 1)[0] * C_LIGHT / (np.pi * 25.0 * fg[0])
    assert airy_power(np.pi * 25.0 * fg[0] * r0 / C_LIGHT) ** 2 < 1e-30


def beam_source_workload(l0, m0, flux):
    """A-projection workload (PS * A, one frequency group) with the
    visibilities of one point source at (l0, m0) as the measurement equation
    gives them: flux x the group's beam B(l0, m0) x exp(-2 pi i (u l0 + v
    m0)), unit weights, one polarisation."""
    wl = synth.tiny_workload(n_ant=14, diameter_m=400.0, n_time=48, dt_s=300.0, nchan=2,
                             npol=1, nx=128, ny=128, cell_arcsec=20.0, oversample=8,
                             terms=TERM_PS | TERM_A, h_min=8, h_max=8, f_lo=2.9e9, f_hi=3.1e9,
                             n_src=1, sigma=0.0, cfg_id=251)
    nu_fg = float(wl.cf.fg_hz[0])
    b = airy_power(np.pi * wl.cf.dish_m * nu_fg * np.hypot(l0, m0) / C_LIGHT)
    f = wl.obs.freq_hz
    u = wl.obs.uvw[:, 0:1] * f[None, :] / C_LIGHT
    v = wl.obs.uvw[:, 1:2] * f[None, :] / C_LIGHT
    wl.vis = (flux * b * np.exp(-2j * np.pi * (u * l0 + v * m0)))[..., None]
    wl.weight = np.ones(wl.vis.shape)
    return wl, float(b)


def test_point_source_comes_back_at_its_flux_through_the_weight_image():
    cell = 20.0 * np.pi / 180 / 3600
    ix, iy = 21, -6                       # about half-way down the beam at 3 GHz
    l0, m0 = ix * cell, iy * cell
    wl, b = beam_source_workload(l0, m0, 2.0)
    assert 0.35 < b < 0.65
    ocf = oracle.build_cf(wl.grid, wl.cf)
    pr = Problem.from_workload(wl, ocf)
    counts = pr.sumwt(wl.weight)[1]
    assert counts[2] == 0                 # nothing dropped
    grid = pr.grid(wl.vis, wl.weight)
    sumwt = pr.sumwt(wl.weight)[0][0, 0]
    g = wl.grid
    img = centred_ifft(grid[0, 0])
    tx, ty = ps_taper(g.nx, 7), ps_taper(g.ny, 7)
    pb = pb_image(g.nx, g.ny, g.cell_l, g.cell_m, wl.cf.fg_hz, wl.cf.dish_m, [sumwt])
    out = normalise_aw(img, tx, ty, sumwt, pb, 0.05)
    px, py = g.nx // 2 + ix, g.ny // 2 + iy
    assert out[py, px] == pytest.approx(2.0, rel=0.005)
    # the beam divided out once instead of twice leaves the flux times B
    once = normalise_aw(img, tx, ty, sumwt, np.sqrt(pb), 0.05)
    assert once[py, px] == pytest.approx(2.0 * b, rel=0.005)
    assert abs(once[py, px] - 2.0) > 0.5
    # outside the cut the image is 0
    assert np.all(out[pb < 0.05] == 0.0)
