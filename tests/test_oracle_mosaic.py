"""Pins of the oracle's mosaic rows (imaging-mode table; Eq. CIJ), CPU only.

The change of phase centre is pinned against direct-sum visibilities: a sky
observed with phase centre s(P) and moved to s0 must equal the same sky
observed with phase centre s0 (w = 0, where the flat-sky shift is exact).
Zero offsets change nothing, the two directions are inverse, and the
virtual antennas reproduce the single-pointing phasor (zero field offsets)
and a common pointing offset (one field)."""

import copy

import numpy as np

import synth
import oracle
from oracle import mosaic
from oracle.cfbuild import TERM_A, TERM_PS
from oracle.native import Problem
from synth.sky import PointSky, dft_visibilities


def observation(seed=180):
    wl = synth.tiny_workload(n_ant=7, n_time=10, nchan=3, cfg_id=seed)
    return wl


def test_change_of_phase_centre_matches_direct_sums():
    wl = observation()
    uvw = wl.obs.uvw.copy()
    uvw[:, 2] = 0.0
    rng = np.random.default_rng(1)
    sky = PointSky(l=rng.uniform(-3e-4, 3e-4, 5), m=rng.uniform(-3e-4, 3e-4, 5),
                   flux=rng.uniform(0.1, 1.0, 5))
    lp, mp = 2.0e-4, -1.5e-4
    # the same sky seen from phase centre s(P): positions relative to s(P)
    sky_p = PointSky(l=sky.l - lp, m=sky.m - mp, flux=sky.flux)
    v0 = dft_visibilities(uvw, wl.obs.freq_hz, sky, 4)
    vp = dft_visibilities(uvw, wl.obs.freq_hz, sky_p, 4)
    field = np.zeros(len(uvw), np.int32)
    got = mosaic.rephase(vp, uvw, wl.obs.freq_hz, field, [[lp, mp]])
    assert np.max(np.abs(got - v0)) < 1e-12 * np.max(np.abs(v0))
    back = mosaic.rephase(v0, uvw, wl.obs.freq_hz, field, [[lp, mp]], to_image_centre=False)
    assert np.max(np.abs(back - vp)) < 1e-12 * np.max(np.abs(vp))


def test_zero_offsets_and_rows_outside_every_field():
    wl = observation(181)
    v = wl.vis
    field = np.zeros(wl.obs.nrow, np.int32)
    assert np.array_equal(mosaic.rephase(v, wl.obs.uvw, wl.obs.freq_hz, field, [[0.0, 0.0]]), v)
    field[::3] = 5                                   # no such field
    out = mosaic.rephase(v, wl.obs.uvw, wl.obs.freq_hz, field, [[1e-4, 2e-4]])
    assert np.array_equal(out[::3], v[::3])
    assert not np.allclose(out[1::3], v[1::3])


def _grid(wl, ant1, ant2, dlm):
    w2 = copy.deepcopy(wl)
    w2.obs.ant1, w2.obs.ant2, w2.ant_dlm = ant1, ant2, dlm
    ocf = oracle.build_cf(w2.grid, w2.cf)
    return Problem.from_workload(w2, ocf, pointing=True).grid(w2.vis, w2.weight)


def test_virtual_antennas_reproduce_the_pointing_phasor():
    wl = synth.tiny_workload(n_ant=6, n_time=6, nchan=2, nx=64, ny=64, oversample=8,
                             terms=TERM_PS | TERM_A, h_min=3, h_max=3, cfg_id=182,
                             pointing_sigma=2e-5)
    nant = wl.ant_dlm.shape[0]
    ref = _grid(wl, wl.obs.ant1, wl.obs.ant2, wl.ant_dlm)
    # two fields with zero offsets: exactly the single-pointing result
    field = (np.arange(wl.obs.nrow) % 2).astype(np.int32)
    a1, a2, dlm = mosaic.virtual_antennas(wl.obs.ant1, wl.obs.ant2, nant, field,
                                          np.zeros((2, 2)), wl.ant_dlm)
    assert np.array_equal(_grid(wl, a1, a2, dlm), ref)
    # one field offset by d, antennas without offsets: a common offset d
    d = np.array([[3e-5, -2e-5]])
    field0 = np.zeros(wl.obs.nrow, np.int32)
    a1, a2, dlm = mosaic.virtual_antennas(wl.obs.ant1, wl.obs.ant2, nant, field0, d)
    common = np.tile(d, (nant, 1))
    assert np.array_equal(_grid(wl, a1, a2, dlm), _grid(wl, wl.obs.ant1, wl.obs.ant2, common))
