"""Pins of the oracle's index map, gridder, degridder, PSF and sum of
weights against closed forms, brute force and invariants (CPU only)."""

from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import build_cf, channel_constants
from oracle.cfbuild import TERM_A, TERM_PS, TERM_W, kernel_fft, crop_plane, screen
from oracle.imaging import (centred_fft, centred_ifft, gcf_1d, response_1d,
                            separable_1d)
from oracle.native import Problem

C = synth.C_LIGHT


def rel(a, b):
    return np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel())


def make_problem(uvw, freq, nx=64, ny=64, npol=1, cell=4.0, O=100, n_w=1, h=(3, 3),
                 terms=TERM_PS, w_max=0.0, chan_plane=None, nplane=1, ant=None,
                 ant_dlm=None, psf=False, fg_hz=None):
    g = synth.GridSetup(nx, ny, npol, nplane, cell * synth.ARCSEC, cell * synth.ARCSEC)
    cf = synth.CFSetup(terms=terms, oversample=O, ps_support=7, n_w=n_w, w_max=w_max,
                       h_min=h[0], h_max=h[1],
                       fg_hz=np.array([3e9]) if fg_hz is None else fg_hz)
    ocf = build_cf(g, cf)
    nchan = len(freq)
    cp = np.zeros(nchan, np.int32) if chan_plane is None else chan_plane
    a1, a2 = (None, None) if ant is None else ant
    pr = Problem(uvw, freq, cp, np.zeros(nchan, np.int32), nx, ny, npol, nplane,
                 g.cell_l, g.cell_m, ocf, ant1=a1, ant2=a2, ant_dlm=ant_dlm, psf=psf)
    return pr, ocf, g


# --- index map ---------------------------------------------------------------

def test_map_floor_agrees_with_exact_rationals():
    rng = np.random.default_rng(3)
    nx, O = 256, 20
    cell = 1.0 * synth.ARCSEC
    freq = np.array([2.7e9])
    kx, _, _, ox, _ = channel_constants(freq, nx, nx, cell, cell, O, 1, 0.0)
    du_m = C / freq[0] / (nx * cell)
    u = rng.uniform(-100 * du_m, 100 * du_m, 3000)
    # add samples placed on exact 1/O boundaries (ties) and near them
    ties = (np.arange(-50, 50) / O) * du_m
    u = np.concatenate([u, ties, np.nextafter(ties, 1), np.nextafter(ties, -1)])
    uvw = np.stack([u, np.zeros_like(u), np.zeros_like(u)], 1)
    pr, _, _ = make_problem(uvw, freq, nx=nx, ny=nx, cell=1.0, O=O)
    m = pr.map()[:, 0]
    checked = 0
    for i, ui in enumerate(u):
        X = Fraction(ui) * Fraction(kx[0]) + Fraction(ox)
        q = X.numerator // X.denominator
        frac_dist = min(X - q, q + 1 - X)
        if frac_dist * 2 ** 52 < X:          # within ~1 ulp of an integer
            continue
        half = O // 2
        p = (q + half) // O
        o = q - p * O
        assert (m[i, 0], m[i, 2]) == (p, o), (i, ui)
        checked += 1
    assert checked > 3000


def test_map_mirror_property_and_w_plane():
    rng = np.random.default_rng(4)
    freq = np.array([3.1e9])
    du_m = C / freq[0] / (64 * 4.0 * synth.ARCSEC)
    u = rng.uniform(-20 * du_m, 20 * du_m, 2000)
    v = rng.uniform(-20 * du_m, 20 * du_m, 2000)
    w = rng.uniform(-900, 900, 2000)
    uvw = np.stack([u, v, w], 1)
    w_max = float(np.max(np.abs(w)) * freq[0] / C)
    pr, _, _ = make_problem(uvw, freq, O=20, n_w=8, h=(3, 6), terms=TERM_PS | TERM_W,
                            w_max=w_max)
    pm, _, _ = make_problem(-uvw, freq, O=20, n_w=8, h=(3, 6), terms=TERM_PS | TERM_W,
                            w_max=w_max)
    a, b = pr.map()[:, 0], pm.map()[:, 0]
    ok = (a[:, 2] != -10) & (a[:, 3] != -10)
    assert ok.sum() > 1500
    assert np.array_equal(b[ok, 0], 64 - a[ok, 0]) and np.array_equal(b[ok, 2], -a[ok, 2])
    assert np.array_equal(b[ok, 1], 64 - a[ok, 1]) and np.array_equal(b[ok, 3], -a[ok, 3])
    # w-plane: k = round-half-up of |w| (n_w - 1) / w_max, conj iff w < 0
    kref = np.floor(np.abs(w) * freq[0] / C * 7 / w_max + 0.5)
    close = np.abs(np.abs(w) * freq[0] / C * 7 / w_max + 0.5 - np.round(kref)) > 1e-9
    assert np.array_equal(a[close, 4], kref[close].astype(int))
    assert np.array_equal(a[:, 5], (w < 0).astype(int))
    assert np.array_equal(a[:, 4], b[:, 4])


def test_drop_rule_at_the_grid_edge():
    nx, O, h = 64, 10, 3
    freq = np.array([3e9])
    du_m = C / freq[0] / (nx * 4.0 * synth.ARCSEC)
    # cells relative to the centre: p = 32 + c; footprint [p - 3, p + 3]
    cells = np.array([-29, -30, 28, 29, -28, -31])
    uvw = np.stack([cells * du_m, np.zeros(6), np.zeros(6)], 1)
    pr, _, _ = make_problem(uvw, freq, nx=nx, ny=nx, O=O)
    keep = pr.map()[:, 0, 6]
    # p - 3 >= 0 and p + 3 <= 63
    assert list(keep) == [1, 0, 1, 0, 1, 0]
    pp = pr.with_psf(True)
    keep_psf = pp.map()[:, 0, 6]
    # PSF footprint must stay in [1, 63]
    assert list(keep_psf) == [0, 0, 1, 0, 1, 0]


# --- gridding ------------------------------------------------------------------

def test_single_sample_places_the_table_subkernel():
    freq = np.array([3e9])
    du_m = C / freq[0] / (64 * 4.0 * synth.ARCSEC)
    uvw = np.array([[5.37 * du_m, -7.61 * du_m, 0.0]])
    pr, ocf, _ = make_problem(uvw, freq, O=20)
    m = pr.map()[0, 0]
    vis = np.array([[[0.3 - 1.7j]]])
    wt = np.array([[[2.5]]])
    g = pr.grid(vis, wt)[0, 0]
    sub = ocf.sub(0, 0, m[3], m[2])
    ref = np.zeros_like(g)
    ar, ai = 2.5 * 0.3, 2.5 * -1.7
    ref[m[1] - 3:m[1] + 4, m[0] - 3:m[0] + 4] = (sub.real * ar - sub.imag * ai) + \
        1j * (sub.real * ai + sub.imag * ar)
    assert np.array_equal(g, ref)
    assert (m[0], m[1]) == (32 + 5, 32 - 8) and (m[2], m[3]) == (7, 8)


def _lattice_problem(nsamp=48, seed=5):
    rng = np.random.default_rng(seed)
    freq = np.array([3e9])
    nx = 64
    du_m = C / freq[0] / (nx * 4.0 * synth.ARCSEC)
    a = rng.integers(-20, 21, nsamp)
    b = rng.integers(-20, 21, nsamp)
    uvw = np.stack([a * du_m, b * du_m, np.zeros(nsamp)], 1)
    vis = (rng.standard_normal(nsamp) + 1j * rng.standard_normal(nsamp))[:, None, None]
    wt = rng.uniform(0.5, 2.0, nsamp)[:, None, None]
    return uvw, freq, vis, wt, a, b


def test_direct_dft_on_lattice_aligned_samples():
    uvw, freq, vis, wt, a, b = _lattice_problem()
    pr, ocf, g = make_problem(uvw, freq, O=100)
    m = pr.map()[:, 0]
    assert np.all(m[:, 2] == 0) and np.all(m[:, 3] == 0)
    img = centred_ifft(pr.grid(vis, wt)[0, 0])
    c1 = separable_1d(ocf)
    g0 = response_1d(c1[ocf.O // 2], ocf.O, 0, 64).real
    xi = (np.arange(64) - 32) / 64
    ref = np.einsum("s,sy,sx->yx", (wt * vis)[:, 0, 0], np.exp(2j * np.pi * np.outer(b, xi)),
                    np.exp(2j * np.pi * np.outer(a, xi)))
    ref = ref * np.outer(g0, g0)
    assert rel(img, ref) < 1e-13


def test_dirty_image_of_random_samples_within_the_computed_bound():
    rng = np.random.default_rng(6)
    freq = np.array([3e9])
    nx, O = 64, 100
    du_m = C / freq[0] / (nx * 4.0 * synth.ARCSEC)
    ns = 64
    x = rng.uniform(-20, 20, ns)
    y = rng.uniform(-20, 20, ns)
    uvw = np.stack([x * du_m, y * du_m, np.zeros(ns)], 1)
    vis = (rng.standard_normal(ns) + 1j * rng.standard_normal(ns))[:, None, None]
    wt = rng.uniform(0.5, 2.0, ns)[:, None, None]
    pr, ocf, g = make_problem(uvw, freq, O=O)
    img = centred_ifft(pr.grid(vis, wt)[0, 0])
    c1 = separable_1d(ocf)
    gc = gcf_1d(c1, O, nx).real
    xi = (np.arange(nx) - nx // 2) / nx
    dft = np.einsum("s,sy,sx->yx", (wt * vis)[:, 0, 0], np.exp(2j * np.pi * np.outer(y, xi)),
                    np.exp(2j * np.pi * np.outer(x, xi)))
    est = img / np.outer(gc, gc)
    # per-axis scalloping of every offset's response relative to the gcf
    sc = np.max([np.abs(response_1d(c1[i], O, o, nx) / gc - 1)
                 for i, o in enumerate(range(-O // 2, O // 2))], axis=0)
    q = 2 * np.pi * np.abs(xi) / (2 * O)
    bx = (1 + sc) * (1 + q)
    bound = np.outer(bx, bx) - 1
    inner = slice(nx // 4, 3 * nx // 4)
    err = np.abs(est - dft)[inner, inner]
    lim = (bound * np.sum(np.abs(wt * vis)))[inner, inner]
    assert np.all(err <= lim * 1.000001 + 1e-12)
    assert np.max(err) > 0


def test_unit_point_source_at_phase_centre():
    wl = synth.tiny_workload(npol=1, nchan=2, n_src=1, sigma=0.0)
    wl.vis[:] = 1.0                      # a 1 Jy point source at l = m = 0
    ocf = build_cf(wl.grid, wl.cf)
    pr = Problem.from_workload(wl, ocf)
    g = pr.grid(wl.vis, wl.weight)
    s, cnt = pr.sumwt(wl.weight)
    m = pr.map()
    taps = [ocf.sub(0, 0, mm[3], mm[2]).sum() for mm in m.reshape(-1, 8) if mm[6]]
    wts = wl.weight[..., 0].ravel()[m.reshape(-1, 8)[:, 6] == 1]
    centre = g.sum() / s.sum()           # image value at l = m = 0
    assert abs(centre - np.sum(wts * np.array(taps)) / s.sum()) < 1e-13
    scallop = max(abs(t - 1) for t in taps)
    assert abs(centre - 1) <= scallop + 1e-14 and scallop < 1e-2


def test_adjoint_identity_with_wproj_flags_and_pointing():
    wl = synth.tiny_workload(n_w=5, h_min=3, h_max=5, oversample=8,
                             terms=TERM_PS | TERM_W | TERM_A, nchan=3, n_time=8,
                             pointing_sigma=2e-5, diameter_m=1500.0, cell_arcsec=8.0)
    assert np.any(wl.obs.uvw[:, 2] < 0) and np.any(wl.obs.uvw[:, 2] > 0)
    rng = np.random.default_rng(7)
    wl.weight[rng.random(wl.weight.shape) < 0.1] = 0.0
    ocf = build_cf(wl.grid, wl.cf)
    pr = Problem.from_workload(wl, ocf)
    assert pr.po
    shape = pr.grid_shape()
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    y = rng.standard_normal(wl.vis.shape) + 1j * rng.standard_normal(wl.vis.shape)
    dx = pr.degrid(x, wl.weight)
    gy = pr.grid(y, (wl.weight != 0).astype(float))
    lhs = np.vdot(dx, y)
    rhs = np.vdot(x, gy)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
    assert np.count_nonzero(dx) > 0


def test_degrid_of_a_constant_grid_returns_conjugate_tap_sums():
    wl = synth.tiny_workload(n_w=3, h_min=3, h_max=4, oversample=6,
                             terms=TERM_PS | TERM_W, nchan=2)
    ocf = build_cf(wl.grid, wl.cf)
    pr = Problem.from_workload(wl, ocf)
    v = pr.degrid(np.ones(pr.grid_shape(), np.complex128))
    m = pr.map()
    for r in range(0, wl.obs.nrow, 7):
        for c in range(wl.obs.nchan):
            mm = m[r, c]
            if not mm[6]:
                assert np.all(v[r, c] == 0)
                continue
            ts = ocf.sub(0, mm[4], mm[3], mm[2]).sum()
            if mm[5]:
                ts = np.conj(ts)
            assert np.allclose(v[r, c], np.conj(ts), rtol=0, atol=1e-14)


def test_partition_additivity_and_channel_accumulate_vs_gather():
    wl = synth.tiny_workload(nchan=4, n_time=10)
    ocf = build_cf(wl.grid, wl.cf)
    pr = Problem.from_workload(wl, ocf)
    full = pr.grid(wl.vis, wl.weight)
    half = wl.obs.nrow // 2
    pa = Problem(wl.obs.uvw[:half], wl.obs.freq_hz, wl.chan_plane, wl.chan_fg,
                 wl.grid.nx, wl.grid.ny, wl.grid.npol, 1, wl.grid.cell_l, wl.grid.cell_m, ocf)
    pb = Problem(wl.obs.uvw[half:], wl.obs.freq_hz, wl.chan_plane, wl.chan_fg,
                 wl.grid.nx, wl.grid.ny, wl.grid.npol, 1, wl.grid.cell_l, wl.grid.cell_m, ocf)
    parts = pa.grid(wl.vis[:half], wl.weight[:half]) + pb.grid(wl.vis[half:], wl.weight[half:])
    assert rel(parts, full) < 1e-14
    cube = Problem(wl.obs.uvw, wl.obs.freq_hz, np.arange(4, dtype=np.int32), wl.chan_fg,
                   wl.grid.nx, wl.grid.ny, wl.grid.npol, 4, wl.grid.cell_l,
                   wl.grid.cell_m, ocf).grid(wl.vis, wl.weight)
    assert rel(cube.sum(axis=0, keepdims=True), full) < 1e-14
    # serial and threaded oracle are the same computation per cell
    assert np.array_equal(pr.grid(wl.vis, wl.weight, nthreads=1), full)


def test_counters_and_sumwt():
    wl = synth.tiny_workload(nchan=3, n_time=10, diameter_m=20000.0, nx=64, ny=64)
    rng = np.random.default_rng(8)
    wl.weight[:] = rng.integers(1, 5, wl.weight.shape).astype(float)
    wl.weight[rng.random(wl.weight.shape) < 0.2] = 0.0
    wl.chan_plane[:] = [0, -1, 0]
    ocf = build_cf(wl.grid, wl.cf)
    pr = Problem.from_workload(wl, ocf)
    s, cnt = pr.sumwt(wl.weight)
    keep = pr.map()[..., 6].astype(bool)
    flagged = (wl.weight == 0) | (wl.chan_plane < 0)[None, :, None]
    kept = ~flagged & keep[..., None]
    dropped = ~flagged & ~keep[..., None]
    assert cnt[0] == kept.sum() and cnt[1] == flagged.sum() and cnt[2] == dropped.sum()
    assert dropped.sum() > 0 and kept.sum() > 0
    assert cnt.sum() == wl.weight.size
    ref = (wl.weight * kept).sum(axis=(0, 1))
    assert np.array_equal(s[0], ref)


# --- PSF -----------------------------------------------------------------------

def test_psf_is_hermitian_and_equals_mirror_scatter():
    wl = synth.tiny_workload(n_w=3, h_min=3, h_max=4, oversample=6,
                             terms=TERM_PS | TERM_W, nchan=2)
    ocf = build_cf(wl.grid, wl.cf)
    pr = Problem.from_workload(wl, ocf)
    psf, s, cnt = pr.psf(wl.weight)
    ny, nx = wl.grid.ny, wl.grid.nx
    a = psf[0, 0]
    mir = np.conj(a[::-1, ::-1])          # [ny-1-i][nx-1-j]
    # psf[ny - i][nx - j] == conj psf[i][j] bitwise, for i, j >= 1
    assert np.array_equal(a[1:, 1:], np.conj(a[1:, 1:][::-1, ::-1]))
    assert np.all(a[0, :] == 0) and np.all(a[:, 0] == 0)
    m2 = pr.psf_mirror(wl.weight)
    assert rel(m2, psf) < 1e-14
    img = centred_ifft(psf[0, 0]) / s[0, 0]
    assert np.max(np.abs(img.imag)) < 1e-13 * np.max(np.abs(img.real))
    c = img[ny // 2, nx // 2].real
    assert abs(c - 1) < 2e-3


# --- pointing phasor -------------------------------------------------------------

def test_zero_pointing_offsets_reproduce_the_plain_result_bitwise():
    wl = synth.tiny_workload(n_w=3, h_min=3, h_max=4, oversample=6,
                             terms=TERM_PS | TERM_W, nchan=2, pointing_sigma=1e-5)
    ocf = build_cf(wl.grid, wl.cf)
    wl.ant_dlm[:] = 0.0
    po = Problem.from_workload(wl, ocf)
    plain = Problem.from_workload(wl, ocf, pointing=False)
    assert po.po and not plain.po
    assert np.array_equal(po.grid(wl.vis, wl.weight), plain.grid(wl.vis, wl.weight))
    g = np.random.default_rng(1).standard_normal(po.grid_shape()) + 0j
    assert np.array_equal(po.degrid(g), plain.degrid(g))


def test_pointing_phasor_matches_a_shifted_screen():
    nx, O, cell = 128, 20, 4.0
    freq = np.array([3e9])
    du_m = C / freq[0] / (nx * cell * synth.ARCSEC)
    uvw = np.array([[3.43 * du_m, -5.77 * du_m, 0.0]])
    d1 = np.array([6.0, -4.0]) * synth.ARCSEC
    d2 = np.array([2.0, 3.0]) * synth.ARCSEC
    ant_dlm = np.stack([d1, d2])
    pr, ocf, g = make_problem(uvw, freq, nx=nx, ny=nx, cell=cell, O=O, h=(6, 6),
                              ant=(np.array([0]), np.array([1])), ant_dlm=ant_dlm)
    vis = np.ones((1, 1, 1), np.complex128)
    wt = np.ones((1, 1, 1))
    g_po = pr.grid(vis, wt)[0, 0]
    # table from the whole screen shifted by the mean offset, times f
    shift = 0.5 * (d1 + d2)
    M = ocf.M
    scr = screen(M, nx, nx, g.cell_l, g.cell_m, TERM_PS, 7, 0.0, 3e9, 25.0, shift=shift)
    K = kernel_fft(scr, O)
    psi0 = 1.0
    sub_shift = crop_plane(K, M, O, 6, psi0)
    from oracle.cfbuild import airy_power
    dd = np.linalg.norm(d1 - d2)
    f = airy_power(np.array([np.pi * 25.0 * 3e9 * dd / 2 / C]))[0]
    assert 0 < f < 1
    m = pr.map()[0, 0]
    ref = np.zeros_like(g_po)
    ref[m[1] - 6:m[1] + 7, m[0] - 6:m[0] + 7] = f * sub_shift[m[3] + O // 2, m[2] + O // 2]
    assert rel(g_po, ref) < 1e-4
    plain = make_problem(uvw, freq, nx=nx, ny=nx, cell=cell, O=O, h=(6, 6))[0]
    assert rel(plain.grid(vis, wt)[0, 0], ref) > 1e-2    # the phasor matters


# --- chi^2 gradient (Eq. ImChisq / ResIm) ----------------------------------------

def test_chi2_gradient_equals_central_differences():
    wl = synth.tiny_workload(npol=1, nchan=2, n_time=8, nx=32, ny=32, cell_arcsec=8.0,
                             oversample=10)
    ocf = build_cf(wl.grid, wl.cf)
    pr = Problem.from_workload(wl, ocf)
    c1 = separable_1d(ocf)
    gc = gcf_1d(c1, ocf.O, 32).real
    gam = 1.0 / np.outer(gc, gc)
    rng = np.random.default_rng(9)
    img = rng.standard_normal((32, 32)) * 0.01

    def model(I):
        return pr.degrid(centred_fft(gam * I)[None, None], wl.weight)

    def chi2(I):
        r = wl.vis - model(I)
        return np.sum(wl.weight * np.abs(r) ** 2)

    r = wl.vis - model(img)
    grad = -2 * np.real(gam * centred_ifft(pr.grid(wl.weight * r,
                                                   (wl.weight != 0).astype(float))[0, 0]))
    eps = 0.01
    for _ in range(6):
        j = tuple(rng.integers(8, 24, 2))
        e = np.zeros_like(img)
        e[j] = eps
        fd = (chi2(img + e) - chi2(img - e)) / (2 * eps)
        assert abs(fd - grad[j]) <= 1e-7 * max(abs(fd), 1e-3 * np.abs(grad).max())
    # noise-free model visibilities make the gradient vanish
    wl.vis = model(img)
    r0 = wl.vis - model(img)
    assert np.max(np.abs(r0)) == 0
