"""Array layouts and (u, v, w) tracks for synthetic observations.

The (u, v, w) coordinates follow the textbook Earth-rotation synthesis
relations (Thompson, Moran & Swenson, ch. 4): local east/north/up antenna
positions are rotated to the equatorial (X, Y, Z) frame at the array
latitude, and baseline vectors are projected with hour angle H and
declination delta.  The paper's experiment uses the VLA (its data section),
whose site latitude is used here.
"""

from dataclasses import dataclass, field

import numpy as np

C_LIGHT = 299792458.0            # m/s
VLA_LATITUDE_DEG = 34.0784       # deg
SIDEREAL_DAY_S = 86164.0905      # s
ARCSEC = np.pi / (180.0 * 3600.0)
DEG = np.pi / 180.0


@dataclass
class Observation:
    """Rows are time-major: row = itime * nbl + ibl."""
    uvw: np.ndarray          # [nrow, 3] float64, metres
    freq_hz: np.ndarray      # [nchan] float64
    ant1: np.ndarray         # [nrow] int32
    ant2: np.ndarray         # [nrow] int32
    n_ant: int
    n_time: int
    ant_enu: np.ndarray = field(repr=False, default=None)

    @property
    def nrow(self):
        return self.uvw.shape[0]

    @property
    def nchan(self):
        return self.freq_hz.shape[0]


def antenna_layout(n_ant, diameter_m, seed):
    """Antennas uniform in a disc of the given diameter: r = (D/2) sqrt(U1),
    theta = 2 pi U2, height 0.  Returns [n_ant, 3] (east, north, up) metres."""
    rng = np.random.default_rng(seed)
    u1 = rng.random(n_ant)
    u2 = rng.random(n_ant)
    r = 0.5 * diameter_m * np.sqrt(u1)
    th = 2.0 * np.pi * u2
    return np.stack([r * np.cos(th), r * np.sin(th), np.zeros(n_ant)], axis=1)


def baselines(n_ant):
    """All pairs i < j in lexicographic order, as (ant1, ant2) int32 arrays."""
    i, j = np.triu_indices(n_ant, k=1)
    return i.astype(np.int32), j.astype(np.int32)


def enu_to_xyz(enu, lat_rad):
    e, n, u = enu[..., 0], enu[..., 1], enu[..., 2]
    sl, cl = np.sin(lat_rad), np.cos(lat_rad)
    x = -sl * n + cl * u
    y = e
    z = cl * n + sl * u
    return np.stack([x, y, z], axis=-1)


def uvw_tracks(ant_enu, n_time, dt_s, dec_deg, lat_deg=VLA_LATITUDE_DEG):
    """(u, v, w) in metres for every (time, baseline), time-major, with the
    hour angle centred on transit: H_k = omega * ((k + 1/2) dt - T/2)."""
    a1, a2 = baselines(ant_enu.shape[0])
    xyz = enu_to_xyz(ant_enu, lat_deg * DEG)
    b = xyz[a2] - xyz[a1]                                  # [nbl, 3]
    omega = 2.0 * np.pi / SIDEREAL_DAY_S
    t = (np.arange(n_time) + 0.5) * dt_s - 0.5 * n_time * dt_s
    h = omega * t                                          # [ntime]
    d = dec_deg * DEG
    sh, ch = np.sin(h)[:, None], np.cos(h)[:, None]
    sd, cd = np.sin(d), np.cos(d)
    bx, by, bz = b[None, :, 0], b[None, :, 1], b[None, :, 2]
    u = sh * bx + ch * by
    v = -sd * ch * bx + sd * sh * by + cd * bz
    w = cd * ch * bx - cd * sh * by + sd * bz
    uvw = np.stack([u, v, w], axis=-1).reshape(-1, 3)
    nbl = a1.shape[0]
    return (np.ascontiguousarray(uvw), np.tile(a1, n_time), np.tile(a2, n_time),
            nbl)


def channel_freqs(nchan, f_lo=2.0e9, f_hi=4.0e9, single_hz=None):
    """Channel centres nu_c = f_lo + (c + 1/2)(f_hi - f_lo)/nchan; or one
    channel at `single_hz`."""
    if single_hz is not None:
        return np.full(1, float(single_hz))
    return f_lo + (np.arange(nchan) + 0.5) * (f_hi - f_lo) / nchan


def make_observation(n_ant, diameter_m, n_time, dt_s, dec_deg, freq_hz, seed):
    enu = antenna_layout(n_ant, diameter_m, seed)
    uvw, a1, a2, _ = uvw_tracks(enu, n_time, dt_s, dec_deg)
    return Observation(uvw=uvw, freq_hz=np.asarray(freq_hz, dtype=np.float64),
                       ant1=a1.astype(np.int32), ant2=a2.astype(np.int32),
                       n_ant=n_ant, n_time=n_time, ant_enu=enu)
