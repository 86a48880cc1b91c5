"""Workload presets: the five configurations the gridding hot path is
measured and checked on, plus small variants for tests.

Sizes follow the configurations' own statements; where they are silent the
choice is recorded on the preset (cell size of the W-projection grid, disc
read as diameter, site latitude, seeds 1000+i / 2000+i / 3000+i for layout,
sky and noise of configuration i).
"""

from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np

from .observation import ARCSEC, C_LIGHT, channel_freqs, make_observation, Observation
from .sky import PointSky, add_noise, dft_visibilities, random_point_sky

TERM_PS, TERM_W, TERM_A = 1, 2, 4


@dataclass
class GridSetup:
    nx: int
    ny: int
    npol: int
    nplane: int
    cell_l: float        # radians
    cell_m: float


@dataclass
class CFSetup:
    terms: int           # bit set of TERM_PS | TERM_W | TERM_A
    oversample: int      # O, even
    ps_support: int      # S_ps of the prolate spheroidal taper
    n_w: int             # number of w planes
    w_max: float         # wavelengths, largest |w| mapped to plane n_w - 1
    h_min: int           # half-widths: support S_k = 2 h_k + 1
    h_max: int
    fg_hz: np.ndarray    # [n_fg] A-term frequency of each group
    dish_m: float = 25.0
    screen_m: int = 0    # 0 = smallest even >= 2 * max support
    pol_beam: int = 0    # 0: one power pattern for every pol; 1..3: polarised
                         # beam, Mueller terms up to order pol_beam - 1 in leakage
    beam_ellipticity: float = 0.0
    beam_leakage: float = 0.0

    @property
    def n_fg(self):
        return int(len(self.fg_hz))


@dataclass
class Workload:
    name: str
    obs: Observation
    vis: np.ndarray              # [nrow, nchan, npol] complex128
    weight: np.ndarray           # [nrow, nchan, npol] float64
    grid: GridSetup
    cf: CFSetup
    chan_plane: np.ndarray       # [nchan] int32, -1 = skip
    chan_fg: np.ndarray          # [nchan] int32
    sky: Optional[PointSky] = None
    sigma: float = 0.0
    ant_dlm: Optional[np.ndarray] = None   # [n_ant, 2] pointing offsets, rad
    extra: dict = field(default_factory=dict)

    @property
    def nsamples(self):
        return int(self.obs.nrow * self.obs.nchan * self.grid.npol)


def max_abs_w_lambda(obs):
    return float(np.max(np.abs(obs.uvw[:, 2])) * np.max(obs.freq_hz) / C_LIGHT)


def _build(name, *, n_ant, diameter_m, n_time, dt_s, dec_deg, freq_hz, npol,
           n_src, sigma, grid, cf, cfg_id, chan_plane=None, chan_fg=None,
           sky_half_width_deg=0.5, flux=(0.1, 1.0), log_flux=False,
           with_vis=True, pointing_sigma=0.0, dft_device="cpu", layout_only=False):
    obs = make_observation(n_ant, diameter_m, n_time, dt_s, dec_deg, freq_hz,
                           seed=1000 + cfg_id)
    sky = random_point_sky(n_src, seed=2000 + cfg_id,
                           half_width_deg=sky_half_width_deg,
                           flux_lo=flux[0], flux_hi=flux[1], log_flux=log_flux)
    nchan = obs.nchan
    if layout_only:
        v = wt = None
    elif with_vis:
        v = dft_visibilities(obs.uvw, obs.freq_hz, sky, npol, device=dft_device)
        if sigma > 0:
            v, wt = add_noise(v, sigma, seed=3000 + cfg_id)
        else:
            wt = np.ones(v.shape)
    else:
        v = np.zeros((obs.nrow, nchan, npol), np.complex128)
        wt = np.ones(v.shape)
    if chan_plane is None:
        chan_plane = np.zeros(nchan, np.int32)
    if chan_fg is None:
        chan_fg = np.zeros(nchan, np.int32)
    ant_dlm = None
    if pointing_sigma > 0:
        rng = np.random.default_rng(5000 + cfg_id)
        ant_dlm = rng.normal(0.0, pointing_sigma, size=(n_ant, 2))
    if cf.w_max <= 0 and cf.n_w > 1:
        cf = replace(cf, w_max=max_abs_w_lambda(obs))
    return Workload(name=name, obs=obs, vis=v, weight=wt, grid=grid, cf=cf,
                    chan_plane=np.asarray(chan_plane, np.int32),
                    chan_fg=np.asarray(chan_fg, np.int32), sky=sky, sigma=sigma,
                    ant_dlm=ant_dlm)


def config1_plain():
    """Plain FP64, no w-term: 27 antennas in a 1 km disc, 64 x 56.25 s over
    1 h at dec +30, one channel at 3 GHz, one polarisation (22,464 samples),
    5 point sources, sigma 0.01 Jy, PS kernel S=7 O=100, 256^2 at 2 arcsec."""
    grid = GridSetup(256, 256, 1, 1, 2 * ARCSEC, 2 * ARCSEC)
    cf = CFSetup(terms=TERM_PS, oversample=100, ps_support=7, n_w=1, w_max=0.0,
                 h_min=3, h_max=3, fg_hz=np.array([3.0e9]))
    return _build("config1_plain_fp64", n_ant=27, diameter_m=1000.0, n_time=64,
                  dt_s=3600.0 / 64, dec_deg=30.0,
                  freq_hz=channel_freqs(1, single_hz=3.0e9), npol=1, n_src=5,
                  sigma=0.01, grid=grid, cf=cf, cfg_id=1)


def config2_wproj(with_vis=True, n_time=600, nchan=16, dft_device="cpu"):
    """W-projection: 351 baselines of a 36 km disc, 600 dumps over 10 s,
    16 channels over 2-4 GHz, 4 correlations (13,478,400 samples), 200
    sources, sigma 0.01 Jy.  32 w-planes, supports 17..65, O=20, on a
    2048^2 x 4 grid at 0.2 arcsec (the cell is not stated; 0.2 arcsec keeps
    the longest baseline on the grid)."""
    grid = GridSetup(2048, 2048, 4, 1, 0.2 * ARCSEC, 0.2 * ARCSEC)
    cf = CFSetup(terms=TERM_PS | TERM_W, oversample=20, ps_support=7, n_w=32,
                 w_max=0.0, h_min=8, h_max=32, fg_hz=np.array([3.0e9]))
    return _build("config2_wproj", n_ant=27, diameter_m=36000.0, n_time=n_time,
                  dt_s=10.0 / 600, dec_deg=30.0, freq_hz=channel_freqs(nchan),
                  npol=4, n_src=200, sigma=0.01, grid=grid, cf=cf, cfg_id=2,
                  with_vis=with_vis, dft_device=dft_device)


def config2_ps(with_vis=True, n_time=600, nchan=16, dft_device="cpu"):
    """The W-projection data gridded with the Standard (PS only) kernel,
    S=7, O=100: the shape on which HBM bandwidth binds."""
    w = config2_wproj(with_vis=with_vis, n_time=n_time, nchan=nchan, dft_device=dft_device)
    w.name = "config2_ps"
    w.cf = CFSetup(terms=TERM_PS, oversample=100, ps_support=7, n_w=1, w_max=0.0,
                   h_min=3, h_max=3, fg_hz=np.array([3.0e9]))
    return w


def config3_awproj(with_vis=True, n_time=600, nchan=64, n_fg=8, dft_device="cpu"):
    """A+W projection: the W-projection layout over 64 channels and 4
    correlations with per-antenna Airy A-terms (25 m dishes) in 8 frequency
    groups and random pointing offsets of 1% of the 3 GHz FWHM per axis."""
    freq = channel_freqs(nchan)
    per = nchan // n_fg
    chan_fg = np.arange(nchan) // per
    fg_hz = np.array([freq[chan_fg == g].mean() for g in range(n_fg)])
    grid = GridSetup(4096, 4096, 4, 1, 0.2 * ARCSEC, 0.2 * ARCSEC)
    cf = CFSetup(terms=TERM_PS | TERM_W | TERM_A, oversample=20, ps_support=7,
                 n_w=32, w_max=0.0, h_min=8, h_max=32, fg_hz=fg_hz, dish_m=25.0)
    fwhm = 1.029 * (C_LIGHT / 3.0e9) / 25.0
    return _build("config3_awproj", n_ant=27, diameter_m=36000.0, n_time=n_time,
                  dt_s=10.0 / 600, dec_deg=30.0, freq_hz=freq, npol=4, n_src=200,
                  sigma=0.01, grid=grid, cf=cf, cfg_id=3, chan_fg=chan_fg,
                  with_vis=with_vis, pointing_sigma=0.01 * fwhm, dft_device=dft_device)


C5_CHUNK_ROWS = 390625      # 1e8 samples per chunk at 64 channels x 4 pols


def config5(n_time=14400, nchan=64, n_fg=8):
    """Large single image: 351 baselines of a 36 km disc, 8 h at 2 s
    (14,400 dumps), 64 channels over 2-4 GHz, 4 correlations
    (1,293,926,400 samples, streamed in chunks of C5_CHUNK_ROWS rows);
    128 w-planes with supports 17..129, O=20, Airy A-terms (25 m dishes) in
    8 frequency groups; 8192^2 x 4 at 0.3 arcsec.  Layout only: the sample
    values of a chunk come from chunk_values (their values do not change
    the work)."""
    freq = channel_freqs(nchan)
    per = nchan // n_fg
    chan_fg = np.arange(nchan) // per
    fg_hz = np.array([freq[chan_fg == g].mean() for g in range(n_fg)])
    grid = GridSetup(8192, 8192, 4, 1, 0.3 * ARCSEC, 0.3 * ARCSEC)
    cf = CFSetup(terms=TERM_PS | TERM_W | TERM_A, oversample=20, ps_support=7, n_w=128,
                 w_max=0.0, h_min=8, h_max=64, fg_hz=fg_hz, dish_m=25.0)
    return _build("config5", n_ant=27, diameter_m=36000.0, n_time=n_time, dt_s=2.0,
                  dec_deg=30.0, freq_hz=freq, npol=4, n_src=0, sigma=0.0, grid=grid, cf=cf,
                  cfg_id=5, chan_fg=chan_fg, layout_only=True)


def config5_ps(n_time=14400, nchan=64):
    """The large-image layout gridded with the Standard kernel (PS only,
    S=7, O=100, one plane): the shape on which HBM bandwidth binds."""
    w = config5(n_time=n_time, nchan=nchan)
    w.name = "config5_ps"
    w.chan_fg = np.zeros(nchan, np.int32)
    w.cf = CFSetup(terms=TERM_PS, oversample=100, ps_support=7, n_w=1, w_max=0.0,
                   h_min=3, h_max=3, fg_hz=np.array([3.0e9]))
    return w


def chunk_values(nrow, nchan, npol, seed):
    """Seeded sample values for a chunk of rows: complex Gaussian
    visibilities (unit variance per part) and weights uniform in [0.5, 1.5),
    as complex64 / float32."""
    rng = np.random.default_rng(seed)
    shape = (nrow, nchan, npol)
    v = np.empty(shape, np.complex64)
    v.real = rng.standard_normal(shape, np.float32)
    v.imag = rng.standard_normal(shape, np.float32)
    w = (rng.random(shape, np.float32) + np.float32(0.5)).astype(np.float32)
    return v, w


@dataclass
class JobSpec:
    job_id: int
    arrival_s: float
    op: str              # "grid" or "degrid"
    n_samples: int
    n_grid: int          # grid side
    n_w: int
    seed: int


def config4_jobs(n_jobs=256, rate_hz=20.0, seed=4004, vis_lo=1e4, vis_hi=2e7,
                 sizes=(512, 1024, 2048, 4096), max_w=64):
    """Serving stream: Poisson arrivals, log-uniform sample counts, grid side
    from `sizes`, w-plane count uniform in [1, max_w], op grid/degrid with
    probability 1/2 each."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, n_jobs)
    arr = np.cumsum(gaps) - gaps[0]
    nvis = np.floor(10.0 ** rng.uniform(np.log10(vis_lo), np.log10(vis_hi), n_jobs))
    ng = rng.choice(np.asarray(sizes), n_jobs)
    nw = rng.integers(1, max_w + 1, n_jobs)
    op = np.where(rng.random(n_jobs) < 0.5, "grid", "degrid")
    return [JobSpec(i, float(arr[i]), str(op[i]), int(nvis[i]), int(ng[i]),
                    int(nw[i]), int(seed * 1000 + i)) for i in range(n_jobs)]


def tiny_workload(*, n_ant=6, diameter_m=3000.0, n_time=12, dt_s=60.0, nchan=3,
                  npol=4, nx=96, ny=80, cell_arcsec=4.0, n_w=1, h_min=3, h_max=3,
                  oversample=8, terms=TERM_PS, n_src=3, sigma=0.01, nplane=1,
                  chan_plane=None, chan_fg=None, fg_hz=None, cfg_id=90,
                  pointing_sigma=0.0, dec_deg=30.0, f_lo=2.0e9, f_hi=4.0e9):
    """Small seeded workloads for tests: same generators, small sizes."""
    freq = channel_freqs(nchan, f_lo=f_lo, f_hi=f_hi)
    if fg_hz is None:
        fg_hz = np.array([freq.mean()])
    grid = GridSetup(nx, ny, npol, nplane, cell_arcsec * ARCSEC, cell_arcsec * ARCSEC)
    cf = CFSetup(terms=terms, oversample=oversample, ps_support=7, n_w=n_w,
                 w_max=0.0, h_min=h_min, h_max=h_max, fg_hz=np.asarray(fg_hz))
    return _build("tiny", n_ant=n_ant, diameter_m=diameter_m, n_time=n_time,
                  dt_s=dt_s, dec_deg=dec_deg, freq_hz=freq, npol=npol, n_src=n_src,
                  sigma=sigma, grid=grid, cf=cf, cfg_id=cfg_id,
                  chan_plane=chan_plane, chan_fg=chan_fg,
                  sky_half_width_deg=(nx * cell_arcsec / 3600.0) / 4.0,
                  pointing_sigma=pointing_sigma)
