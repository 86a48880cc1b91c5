"""Oracle pins of the sparse Mueller matrix of CFs (the F M^DD of the AWP
framework's VisResampler, physical-architecture section; Eq. ME with
M^DD = J (x) J for identical antennas).

Reading of the polarised beam (the paper gives none): linear feeds, one
real symmetric Jones matrix J = [[E_X, d], [d, E_Y]] with elliptical Airy
voltage patterns (ellipticity eta) and a four-lobed cross-polar leakage
d = kappa (s l)(s m) a(s rho).

* Kind map: M[q][p] = J[q1][p1] J[q2][p2] evaluated through the kinds
  equals the Kronecker product np.kron(J, J) at random directions; the
  orders kept by pol_beam 1 / 2 / 3 are 4 / 12 / 16 elements.
* Closed forms of the beam: 1 and 0 at the centre, no leakage on the axes,
  the ellipticity along l and m, E_X(l, m) = E_Y(m, l), evenness.
* eta = kappa = 0 reduces every diagonal kind to the scalar A-term table
  and the off-diagonal kinds to zero, so gridding and degridding equal the
  scalar path.
* Degridding a model of polarised point sources through the Mueller
  kernels reproduces the measurement equation V_q = sum_p M_qp(s) I_p(s)
  e^{-2 pi i u.s} evaluated by direct sum with np.kron(J, J) (leakage and
  ellipticity large enough that a wrong element would show by far).
* Gridding is the adjoint of degridding: <D x, y> = <x, G y>.
"""

import copy

import numpy as np
import pytest

import oracle
import synth
from oracle.cfbuild import (TERM_A, TERM_PS, airy_voltage, jones_linear, kind_beam,
                            mueller_kinds)
from oracle.conventions import C_LIGHT
from oracle.imaging import centred_fft, ps_taper
from oracle.native import Problem


def test_kind_map_is_the_kronecker_product_and_keeps_orders():
    rng = np.random.default_rng(0)
    nu, dish, eta, kappa = 3e9, 25.0, 0.15, 0.3
    for _ in range(20):
        l, m = rng.uniform(-0.01, 0.01, 2)
        ex, ey, d = jones_linear(l, m, nu, dish, eta, kappa)
        J = np.array([[ex, d], [d, ey]])
        K = np.kron(J, J)                    # rows (q1 q2), columns (p1 p2)
        km = mueller_kinds(3)
        got = np.array([[kind_beam(km[q, p], l, m, nu, dish, eta, kappa)
                         for p in range(4)] for q in range(4)])
        assert np.allclose(got, K, rtol=1e-14, atol=1e-300)
    counts = {b: int((mueller_kinds(b) >= 0).sum()) for b in (1, 2, 3)}
    assert counts == {1: 4, 2: 12, 3: 16}
    assert list(np.diag(mueller_kinds(1))) == [0, 2, 2, 1]
    assert np.all(mueller_kinds(1)[~np.eye(4, dtype=bool)] == -1)
    assert set(mueller_kinds(2).ravel()) == {-1, 0, 1, 2, 3, 4}
    assert set(mueller_kinds(3).ravel()) == {0, 1, 2, 3, 4, 5}
    for b in (1, 2, 3):
        assert np.array_equal(mueller_kinds(b), mueller_kinds(b).T)


def test_beam_closed_forms():
    nu, dish, eta, kappa = 3e9, 25.0, 0.1, 0.25
    s = np.pi * dish * nu / C_LIGHT
    ex, ey, d = jones_linear(0.0, 0.0, nu, dish, eta, kappa)
    assert (ex, ey, d) == (1.0, 1.0, 0.0)
    l = np.linspace(-0.004, 0.004, 9)
    ex, ey, d = jones_linear(l, 0.0 * l, nu, dish, eta, kappa)
    assert np.all(d == 0.0)
    assert np.allclose(ex, airy_voltage(s * np.abs(l) / (1 + eta)), rtol=1e-15)
    assert np.allclose(ey, airy_voltage(s * np.abs(l) / (1 - eta)), rtol=1e-15)
    ex2, ey2, _ = jones_linear(0.0 * l, l, nu, dish, eta, kappa)
    assert np.allclose(ex2, ey, rtol=1e-15) and np.allclose(ey2, ex, rtol=1e-15)
    _, _, dd = jones_linear(l, l, nu, dish, eta, kappa)
    assert np.allclose(dd, kappa * (s * l) ** 2 * airy_voltage(s * np.sqrt(2) * np.abs(l)),
                       rtol=1e-14)
    # first null of E_X along l at s l / (1 + eta) = j_{1,1}
    from scipy import special
    l0 = special.jn_zeros(1, 1)[0] * (1 + eta) / s
    assert abs(jones_linear(l0, 0.0, nu, dish, eta, kappa)[0]) < 1e-15
    rng = np.random.default_rng(1)
    lm = rng.uniform(-0.005, 0.005, (2, 50))
    for kind in range(6):
        a = kind_beam(kind, lm[0], lm[1], nu, dish, eta, kappa)
        b = kind_beam(kind, -lm[0], -lm[1], nu, dish, eta, kappa)
        assert np.array_equal(a, b)


def beam_workload(pol_beam, eta, kappa, n_w=1, seed=301):
    wl = synth.tiny_workload(n_ant=12, diameter_m=400.0, n_time=30, dt_s=300.0, nchan=2,
                             npol=4, nx=128, ny=128, cell_arcsec=20.0, oversample=8,
                             terms=TERM_PS | TERM_A, h_min=8, h_max=8, n_w=n_w,
                             f_lo=2.9e9, f_hi=3.1e9, n_src=3, cfg_id=seed)
    wl.cf.pol_beam, wl.cf.beam_ellipticity, wl.cf.beam_leakage = pol_beam, eta, kappa
    return wl


def lattice_problem(wl, ocf, n=400, seed=9):
    """One channel, n samples whose (u, v) fall exactly on grid cells (offset
    0): the gridding error is then the kernel's aliasing alone, with no
    oversampling quantisation."""
    g = wl.grid
    rng = np.random.default_rng(seed)
    nu = wl.obs.freq_hz[:1]
    iu = rng.integers(-g.nx // 2 + 12, g.nx // 2 - 12, n)
    iv = rng.integers(-g.ny // 2 + 12, g.ny // 2 - 12, n)
    uvw = np.zeros((n, 3))
    uvw[:, 0] = iu / (g.nx * g.cell_l) * C_LIGHT / nu[0]
    uvw[:, 1] = iv / (g.ny * g.cell_m) * C_LIGHT / nu[0]
    return Problem(uvw, nu, np.zeros(1, np.int32), np.zeros(1, np.int32), g.nx, g.ny, 4, 1,
                   g.cell_l, g.cell_m, ocf)


def test_no_ellipticity_or_leakage_is_the_scalar_beam():
    wl = beam_workload(3, 0.0, 0.0)
    ocf = oracle.build_cf(wl.grid, wl.cf)
    sc = copy.copy(wl.cf)
    sc.pol_beam = 0
    ocs = oracle.build_cf(wl.grid, sc)
    n = ocs.table.size
    assert ocf.n_kind == 6 and ocf.kind_elems == n
    for kind in (0, 1, 2):
        assert np.allclose(ocf.table[kind * n:(kind + 1) * n], ocs.table, rtol=0,
                           atol=1e-15 * np.max(np.abs(ocs.table)))
    assert np.all(ocf.table[3 * n:] == 0)
    pm = Problem.from_workload(wl, ocf)
    ps = Problem.from_workload(wl, ocs)
    gm, gs = pm.grid(wl.vis, wl.weight), ps.grid(wl.vis, wl.weight)
    assert np.linalg.norm(gm - gs) <= 1e-14 * np.linalg.norm(gs)
    rng = np.random.default_rng(3)
    x = rng.standard_normal(gs.shape) + 1j * rng.standard_normal(gs.shape)
    vm, vs = pm.degrid(x, wl.weight), ps.degrid(x, wl.weight)
    assert np.linalg.norm(vm - vs) <= 1e-14 * np.linalg.norm(vs)


def test_degridding_through_mueller_kernels_is_the_measurement_equation():
    eta, kappa = 0.12, 0.35
    wl = beam_workload(3, eta, kappa)
    g = wl.grid
    ocf = oracle.build_cf(g, wl.cf)
    pr = lattice_problem(wl, ocf)
    rng = np.random.default_rng(7)
    # polarised point sources on pixel centres inside the main lobe, off the axes
    pix = [(14, 9), (-11, 17), (6, -15), (-18, -7)]
    model = np.zeros((1, 4, g.ny, g.nx), np.complex128)
    srcs = []
    for ix, iy in pix:
        I, Q, U, V = rng.uniform(0.5, 1.0), *rng.uniform(-0.3, 0.3, 3)
        corr = np.array([I + Q, U + 1j * V, U - 1j * V, I - Q])   # XX, XY, YX, YY
        model[0, :, g.ny // 2 + iy, g.nx // 2 + ix] = corr
        srcs.append((ix * g.cell_l, iy * g.cell_m, corr))
    tx, ty = ps_taper(g.nx, 7), ps_taper(g.ny, 7)
    mg = centred_fft(model / (ty[:, None] * tx[None, :]))
    ones = np.ones((pr.nrow, 1, 4))
    m = pr.map()
    assert np.all(m[..., 2] == 0) and np.all(m[..., 3] == 0) and np.all(m[..., 6] == 1)
    pred = pr.degrid(mg, ones)[:, 0]

    def direct(eta, kappa):
        # the measurement equation by direct sum, M = kron(J, J) per source
        u = pr.uvw[:, 0] * pr.freq[0] / C_LIGHT
        v = pr.uvw[:, 1] * pr.freq[0] / C_LIGHT
        out = np.zeros((pr.nrow, 4), np.complex128)
        for l, m_, corr in srcs:
            ex, ey, d = jones_linear(l, m_, float(wl.cf.fg_hz[0]), wl.cf.dish_m, eta, kappa)
            J = np.array([[ex, d], [d, ey]])
            out += np.exp(-2j * np.pi * (u * l + v * m_))[:, None] * (np.kron(J, J) @ corr)
        return out

    ref = direct(eta, kappa)
    err = np.linalg.norm(pred - ref) / np.linalg.norm(ref)
    print("Mueller degrid vs measurement equation (lattice samples), rel-RMS", err)
    assert err < 5e-6
    # a beam without leakage or ellipticity misses the polarised sky by far
    assert np.linalg.norm(pred - direct(0.0, 0.0)) / np.linalg.norm(ref) > 0.1
    # and so does every single element of the kind map moved to a wrong kind
    km = ocf.mueller.copy()
    for q, p in [(0, 0), (1, 2), (0, 3), (3, 1)]:
        bad = copy.copy(ocf)
        bad.mueller = km.copy()
        bad.mueller[q, p] = (km[q, p] + 1) % 6
        pb = lattice_problem(wl, bad)
        e = np.linalg.norm(pb.degrid(mg, ones)[:, 0] - ref) / np.linalg.norm(ref)
        assert e > 1e3 * err, (q, p, e)


def test_off_lattice_error_is_that_of_the_scalar_beam():
    # on ordinary samples the oversampling error of the Mueller path is the
    # scalar beam's: the extra kinds add no error of their own
    errs = {}
    for name, (pb, eta, kappa) in {"scalar": (0, 0.0, 0.0), "mueller": (3, 0.12, 0.35)}.items():
        wl = beam_workload(pb, eta, kappa)
        g = wl.grid
        ocf = oracle.build_cf(g, wl.cf)
        model = np.zeros((1, 4, g.ny, g.nx), np.complex128)
        model[0, :, g.ny // 2 + 9, g.nx // 2 + 14] = [1.2, 0.2 + 0.1j, 0.2 - 0.1j, 0.8]
        tx, ty = ps_taper(g.nx, 7), ps_taper(g.ny, 7)
        pred = Problem.from_workload(wl, ocf).degrid(
            centred_fft(model / (ty[:, None] * tx[None, :])), wl.weight)
        l, m_ = 14 * g.cell_l, 9 * g.cell_m
        f = wl.obs.freq_hz
        u = wl.obs.uvw[:, 0:1] * f[None, :] / C_LIGHT
        v = wl.obs.uvw[:, 1:2] * f[None, :] / C_LIGHT
        ex, ey, d = jones_linear(l, m_, float(wl.cf.fg_hz[0]), wl.cf.dish_m, eta, kappa)
        J = np.array([[ex, d], [d, ey]])
        vq = np.kron(J, J) @ model[0, :, g.ny // 2 + 9, g.nx // 2 + 14]
        ref = np.exp(-2j * np.pi * (u * l + v * m_))[..., None] * vq
        errs[name] = np.linalg.norm(pred - ref) / np.linalg.norm(ref)
    print("off-lattice rel-RMS", errs)
    assert errs["mueller"] < 1.2 * errs["scalar"]


@pytest.mark.parametrize("pol_beam", [1, 2, 3])
def test_gridding_is_the_adjoint_of_degridding(pol_beam):
    wl = beam_workload(pol_beam, 0.1, 0.3, n_w=1, seed=311)
    g = wl.grid
    ocf = oracle.build_cf(g, wl.cf)
    pr = Problem.from_workload(wl, ocf)
    rng = np.random.default_rng(5)
    x = rng.standard_normal((1, 4, g.ny, g.nx)) + 1j * rng.standard_normal((1, 4, g.ny, g.nx))
    y = rng.standard_normal(wl.vis.shape) + 1j * rng.standard_normal(wl.vis.shape)
    ones = np.ones(wl.weight.shape)
    dx = pr.degrid(x, ones)
    gy = pr.grid(y, ones)
    a = np.vdot(dx, y)
    b = np.vdot(x, gy)
    assert abs(a - b) <= 1e-12 * abs(a)
