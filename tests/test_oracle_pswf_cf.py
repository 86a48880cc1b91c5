"""Pins of the oracle's prolate spheroidal taper and convolution-function
table against things other than the oracle itself (CPU only)."""

import numpy as np
import pytest
from scipy import special

import synth
from oracle import build_cf, half_widths, pswf_nystrom, screen_size
from oracle.cfbuild import (TERM_A, TERM_PS, TERM_W, airy_power, crop_plane, kernel_fft,
                            plane_scale_exponents, quantised_table, round_bf16, screen)

C7 = np.pi * 7 / 2


def test_pswf_matches_library_spheroidal_function():
    # scipy's angular spheroidal function S_00(c, x) is proportional to psi_0
    psi = pswf_nystrom(C7)[0]
    x = np.linspace(-0.999, 0.999, 201)
    s, _ = special.pro_ang1(0, 0, C7, x)
    s0, _ = special.pro_ang1(0, 0, C7, 0.0)
    assert np.max(np.abs(s / s0 - psi(x))) < 1e-11


def test_pswf_eigen_residual_with_finer_quadrature():
    psi, mu, _, _ = pswf_nystrom(C7)
    t, w = np.polynomial.legendre.leggauss(256)
    x = np.random.default_rng(0).uniform(-1, 1, 1000)
    lhs = np.cos(C7 * np.outer(x, t)) @ (w * psi(t))
    assert np.max(np.abs(lhs - mu * psi(x))) < 1e-12


def test_pswf_even_positive_normalised_and_node_converged():
    psi64 = pswf_nystrom(C7, 64)[0]
    psi128 = pswf_nystrom(C7, 128)[0]
    x = np.linspace(-1, 1, 1001)
    assert abs(psi64(0.0)[0] - 1.0) < 1e-15
    assert np.max(np.abs(psi64(x) - psi64(-x))) < 1e-14
    assert np.all(psi64(x) > 0)
    assert np.max(np.abs(psi64(x) - psi128(x))) < 1e-12


def test_airy_power_pattern_landmarks():
    assert airy_power(np.array([0.0]))[0] == 1.0
    assert abs(airy_power(np.array([3.8317059702]))[0]) < 1e-18
    assert abs(airy_power(np.array([1.6163399]))[0] - 0.5) < 1e-6
    x = np.linspace(1e-6, 3.8, 500)
    assert np.all(np.diff(airy_power(x)) < 0)


def _small_grid(nx=64, cell=4.0):
    return synth.GridSetup(nx, nx, 1, 1, cell * synth.ARCSEC, cell * synth.ARCSEC)


def test_kernel_fft_equals_brute_force_dft():
    g = _small_grid()
    M, O = 14, 6
    scr = screen(M, g.nx, g.ny, g.cell_l, g.cell_m, TERM_PS | TERM_W, 7, 3.0e6, 3e9, 25.0)
    K = kernel_fft(scr, O)
    N = O * M
    rng = np.random.default_rng(1)
    j = np.arange(-(M // 2), M // 2 + 1)
    for _ in range(200):
        nu, nv = rng.integers(-N // 2, N // 2, 2)
        ph = np.exp(-2j * np.pi * (nu * j[None, :] + nv * j[:, None]) / N)
        ref = np.sum(scr * ph)
        assert abs(K[nv % N, nu % N] - ref) < 1e-12 * np.abs(K).max()


def test_uncropped_tap_sum_is_one_for_every_offset():
    g = _small_grid()
    M, O = 14, 8
    scr = screen(M, g.nx, g.ny, g.cell_l, g.cell_m, TERM_PS | TERM_W | TERM_A, 7, 2e6,
                 3e9, 25.0)
    K = kernel_fft(scr, O)
    N = O * M
    t = np.arange(M)
    for o in range(-O // 2, O // 2 + 1):
        n = (o - O * t) % N
        tot = K[np.ix_(n, n)].sum()
        # screen centre value T(0)^2 B(0) W(0) = 1
        assert abs(tot / (M * M) - scr[M // 2, M // 2]) < 1e-13 and abs(scr[M // 2, M // 2] - 1) < 1e-15
    # the screen is even, so with real even terms the kernel is real
    ps = screen(M, g.nx, g.ny, g.cell_l, g.cell_m, TERM_PS | TERM_A, 7, 0.0, 3e9, 25.0)
    assert np.max(np.abs(kernel_fft(ps, O).imag)) < 1e-13


def test_ps_table_is_separable_and_kernel_follows_pswf():
    wl = synth.tiny_workload(n_w=1, h_min=3, h_max=3, oversample=10)
    ocf = build_cf(wl.grid, wl.cf)
    pl = ocf.plane(0, 0)
    O = ocf.O
    mid, h = O // 2, 3
    c1 = pl[mid, :, h, :] / np.sqrt(pl[mid, mid, h, h])
    outer = np.einsum("at,bu->abtu", c1, c1)
    assert np.max(np.abs(pl - outer)) < 1e-14
    assert np.max(np.abs(pl.imag)) < 1e-15
    # with a finely sampled screen the uv kernel approaches psi_0(c, 2 tau / S_ps)
    g = _small_grid(nx=64)
    M = 512
    scr = screen(M, g.nx, g.ny, g.cell_l, g.cell_m, TERM_PS, 7, 0.0, 3e9, 25.0)
    K = kernel_fft(scr, 4)[0, :].real           # n_v = 0 row, n_u along
    psi = pswf_nystrom(C7)[0]
    tau = np.arange(-12, 13) / 4.0              # cells, |tau| <= 3
    ker = K[(np.arange(-12, 13)) % (4 * M)] / K[0]
    assert np.max(np.abs(ker - psi(2 * tau / 7.0))) < 2e-3


def test_term_reductions():
    wl = synth.tiny_workload(n_w=4, h_min=3, h_max=6, oversample=6,
                             terms=TERM_PS | TERM_W)
    wl.cf.w_max = 4.0e5
    aw = build_cf(wl.grid, wl.cf)
    # plane k = 0 has w = 0: W-projection reduces to the Standard kernel
    std = synth.tiny_workload(n_w=1, h_min=3, h_max=3, oversample=6)
    std.cf.screen_m = aw.M
    s0 = build_cf(std.grid, std.cf)
    assert np.array_equal(aw.plane(0, 0), s0.plane(0, 0))
    # A with a vanishing dish is flat (B = 1): A*W == W
    wl2 = synth.tiny_workload(n_w=4, h_min=3, h_max=6, oversample=6,
                              terms=TERM_PS | TERM_W | TERM_A)
    wl2.cf.w_max = 4.0e5
    wl2.cf.dish_m = 1e-9
    a = build_cf(wl2.grid, wl2.cf)
    assert np.max(np.abs(a.table - aw.table)) < 1e-14
    # conjugate symmetry of the W-term: K_{-w} = conj K_w
    g = wl.grid
    sp = screen(14, g.nx, g.ny, g.cell_l, g.cell_m, TERM_PS | TERM_W, 7, 3e5, 3e9, 25.)
    sm = screen(14, g.nx, g.ny, g.cell_l, g.cell_m, TERM_PS | TERM_W, 7, -3e5, 3e9, 25.)
    assert np.max(np.abs(kernel_fft(sm, 4) - np.conj(kernel_fft(sp, 4)))) < 1e-12


def test_support_rule_and_screen_size():
    assert list(half_widths(1, 3, 3)) == [3]
    h = half_widths(32, 8, 32)
    assert h[0] == 8 and h[-1] == 32 and np.all(np.diff(h) >= 0)
    assert np.all(np.diff(h) <= 1)
    h5 = half_widths(128, 8, 64)
    assert h5[0] == 8 and h5[-1] == 64
    assert screen_size(half_widths(32, 8, 32)) == 130
    assert screen_size(np.array([3])) == 14


def test_storage_forms_round_to_nearest_even():
    wl = synth.tiny_workload(n_w=3, h_min=3, h_max=5, oversample=4,
                             terms=TERM_PS | TERM_W)
    wl.cf.w_max = 5e5
    ocf = build_cf(wl.grid, wl.cf)
    ex = plane_scale_exponents(ocf)
    for g in range(ocf.n_fg):
        for k in range(ocf.n_w):
            p = ocf.plane(g, k)
            mx = max(np.abs(p.real).max(), np.abs(p.imag).max()) * 2.0 ** ex[k]
            assert 0.5 <= mx < 1.0
    t = ocf.table
    mag = np.maximum(np.abs(t.real), np.abs(t.imag))
    for form, ulp in (("f32", 2.0 ** -24), ("f16", 2.0 ** -11), ("bf16", 2.0 ** -8)):
        q = quantised_table(ocf, form)
        big = mag > 1e-3 * mag.max()          # normal range for every form
        rel = np.abs(q.real - t.real)[big] / np.abs(t.real)[big].clip(1e-300)
        relr = rel[np.abs(t.real)[big] > 1e-3 * mag.max()]
        assert relr.size and relr.max() <= ulp * 1.0000001
    # bf16 rounding: ties go to even
    assert round_bf16(np.array([1.0 + 2.0 ** -8]))[0] == 1.0
    assert round_bf16(np.array([1.0 + 3 * 2.0 ** -8]))[0] == 1.0 + 2.0 ** -6


def test_compact_table_holds_the_same_planes_and_guards_the_rest():
    """A table restricted to some planes (compact storage) holds exactly the
    full table's values for them; the oracle refuses to grid a sample whose
    plane is missing instead of reading past the table."""
    from oracle.native import Problem
    wl = synth.tiny_workload(n_w=4, h_min=3, h_max=6, oversample=6, terms=TERM_PS | TERM_W,
                             n_time=6, nchan=2)
    full = build_cf(wl.grid, wl.cf)
    part = build_cf(wl.grid, wl.cf, planes={(0, 1), (0, 3)}, compact=True)
    for k in (1, 3):
        assert np.array_equal(part.plane(0, k), full.plane(0, k))
    assert part.table.size == full.plane(0, 1).size + full.plane(0, 3).size
    assert part.plane_off[0] == -1 and part.plane_off[2] == -1
    pr = Problem.from_workload(wl, part)
    m = pr.map().reshape(-1, 8)
    if np.any((m[:, 6] == 1) & ~np.isin(m[:, 4], [1, 3])):
        with pytest.raises(ValueError):
            pr.grid(wl.vis, wl.weight)
    pr_full = Problem.from_workload(wl, build_cf(wl.grid, wl.cf, planes={(0, 0), (0, 1),
                                                                           (0, 2), (0, 3)},
                                                 compact=True))
    assert np.array_equal(pr_full.grid(wl.vis, wl.weight),
                          Problem.from_workload(wl, full).grid(wl.vis, wl.weight))


# --- sign of the W term ---------------------------------------------------------
#
# Eq. ME (with the F sign of the conventions) gives a sample of a unit point
# source at (l0, m0) the phase exp(-2 pi i (u l0 + v m0 + w (n0 - 1))),
# n = sqrt(1 - l^2 - m^2).  Degridding D predicts a sample from F of the
# model image, and gridding G = D^H; for W-projection to remove the w-phase,
# the image-plane response of a gridded sample on w-plane k must carry
# exp(+2 pi i w_k (n - 1)) relative to the w = 0 plane, and degridding must
# reproduce the direct sum above for either sign of w.  Both checks below
# fail by O(1) when the screen's W sign is flipped (planted in the oracle by
# swapping its screen for one evaluated at -w_k).

def _wproj_setup(O=20, n_w=3, w_max=6000.0):
    nx = 64
    cell = 120.0 * synth.ARCSEC
    g = synth.GridSetup(nx, nx, 1, 1, cell, cell)
    cf = synth.CFSetup(terms=TERM_PS | TERM_W, oversample=O, ps_support=7, n_w=n_w,
                       w_max=w_max, h_min=4, h_max=10, fg_hz=np.array([3e9]))
    return g, cf


def _flipped_w_screen(monkeypatch):
    import oracle.cfbuild as cfb
    orig = cfb.screen

    def flipped(M, nx, ny, cell_l, cell_m, terms, ps_support, w_k, *a, **kw):
        return orig(M, nx, ny, cell_l, cell_m, terms, ps_support, -w_k, *a, **kw)

    monkeypatch.setattr(cfb, "screen", flipped)


def _plane_response(g, cf, ocf, k, p=(34, 29), nu=3e9):
    """F^dagger of the grid of one unit sample at the lattice point p (offset
    0) with w exactly on plane k."""
    from oracle.imaging import centred_ifft
    from oracle.native import Problem
    du = 1.0 / (g.nx * g.cell_l)
    lam = synth.C_LIGHT / nu
    w = k * cf.w_max / (cf.n_w - 1)
    uvw = np.array([[(p[0] - g.nx // 2) * du * lam, (p[1] - g.ny // 2) * du * lam, w * lam]])
    pr = Problem(uvw, np.array([nu]), np.zeros(1, np.int32), np.zeros(1, np.int32), g.nx, g.ny,
                 1, 1, g.cell_l, g.cell_m, ocf)
    m = pr.map()[0, 0]
    assert m[6] == 1 and m[2] == 0 and m[3] == 0 and m[4] == k
    return centred_ifft(pr.grid(np.ones((1, 1, 1), complex), np.ones((1, 1, 1)))[0, 0])


def _w_phase_deviation(g, cf, ocf):
    ix = np.arange(g.nx) - g.nx // 2
    ll, mm = np.meshgrid(ix * g.cell_l, ix * g.cell_m)
    n1 = np.sqrt(1.0 - ll * ll - mm * mm) - 1.0
    inner = (np.abs(ix)[None, :] < g.nx // 4) & (np.abs(ix)[:, None] < g.nx // 4)
    r0 = _plane_response(g, cf, ocf, 0)
    out = []
    for k in range(1, cf.n_w):
        wk = k * cf.w_max / (cf.n_w - 1)
        want = np.exp(2j * np.pi * wk * n1)
        out.append((np.abs(wk * n1[inner]).max(),
                    np.abs(_plane_response(g, cf, ocf, k) / r0 - want)[inner].max()))
    return out


def test_w_term_sign_image_plane_response():
    g, cf = _wproj_setup()
    dev = _w_phase_deviation(g, cf, build_cf(g, cf))
    # the w-phase reaches a quarter turn and more over the inner half
    assert dev[-1][0] > 0.4
    for _, d in dev:
        assert d < 2e-3


def test_w_term_sign_flipped_screen_fails_image_plane_pin(monkeypatch):
    g, cf = _wproj_setup()
    _flipped_w_screen(monkeypatch)
    dev = _w_phase_deviation(g, cf, build_cf(g, cf))
    assert max(d for _, d in dev) > 1.0


def _predict_point_source(g, cf, ocf, nsamp=400, seed=3):
    """Degrid the centred FFT of a unit point source (divided by the PS grid
    correction of plane 0) at random (u, v) with w on planes of either sign;
    return (prediction, direct sum of Eq. ME, pixel offsets of the source)."""
    from oracle.imaging import centred_fft, gcf_1d, separable_1d
    from oracle.native import Problem
    nx, O = g.nx, cf.oversample
    gc = gcf_1d(separable_1d(ocf, k=0), O, nx).real
    dx, dy = 12, -10
    l0, m0 = dx * g.cell_l, dy * g.cell_m
    n0 = np.sqrt(1.0 - l0 * l0 - m0 * m0) - 1.0
    img = np.zeros((nx, nx))
    img[nx // 2 + dy, nx // 2 + dx] = 1.0
    grid = centred_fft(img / np.outer(gc, gc))[None, None]
    rng = np.random.default_rng(seed)
    nu = 3e9
    lam = synth.C_LIGHT / nu
    du = 1.0 / (nx * g.cell_l)
    u = rng.uniform(-18, 18, nsamp) * du
    v = rng.uniform(-18, 18, nsamp) * du
    w = np.where(rng.random(nsamp) < 0.5, -1.0, 1.0) * rng.integers(0, cf.n_w, nsamp) * (
        cf.w_max / (cf.n_w - 1))
    pr = Problem(np.stack([u, v, w], 1) * lam, np.array([nu]), np.zeros(1, np.int32),
                 np.zeros(1, np.int32), nx, nx, 1, 1, g.cell_l, g.cell_m, ocf)
    assert pr.map()[..., 6].all()
    got = pr.degrid(grid)[:, 0, 0]
    want = np.exp(-2j * np.pi * (u * l0 + v * m0 + w * n0))
    return got, want, (dx, dy), np.abs(w * n0).max()


def test_w_projection_predicts_the_direct_sum_for_both_signs_of_w():
    g, cf = _wproj_setup(O=40, n_w=5)
    got, want, (dx, dy), wn = _predict_point_source(g, cf, build_cf(g, cf))
    assert wn > 0.2
    # offsets quantise u, v to 1/O of a cell: phase error <= pi (|dx| + |dy|)
    # / (nx O); the kernel truncation adds ~1e-3
    bound = np.pi * (abs(dx) + abs(dy)) / (g.nx * cf.oversample) + 5e-3
    assert np.abs(got - want).max() < bound
    assert np.sqrt(np.mean(np.abs(got - want) ** 2)) < 0.5 * bound


def test_w_projection_prediction_fails_with_flipped_screen(monkeypatch):
    g, cf = _wproj_setup(O=40, n_w=5)
    _flipped_w_screen(monkeypatch)
    got, want, _, _ = _predict_point_source(g, cf, build_cf(g, cf))
    assert np.sqrt(np.mean(np.abs(got - want) ** 2)) > 0.5
