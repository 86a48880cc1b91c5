"""Seeded synthetic observations for the gridding/degridding hot path.

This package produces inputs only: antenna layouts, (u, v, w) tracks from
Earth-rotation synthesis, channel frequencies, point-source skies evaluated
by a direct sum of the measurement equation (Eq. ME with unit Mueller
matrices), Gaussian noise and natural weights.  It contains none of the
gridding, degridding or convolution-function arithmetic, and it is the only
code that both the CPU oracle and the HIP path use.
"""

from .observation import (  # noqa: F401
    C_LIGHT, VLA_LATITUDE_DEG, ARCSEC, DEG,
    Observation, antenna_layout, baselines, uvw_tracks, channel_freqs,
    make_observation,
)
from .sky import PointSky, random_point_sky, dft_visibilities, add_noise  # noqa: F401
from .configs import (  # noqa: F401
    GridSetup, CFSetup, Workload,
    config1_plain, config2_wproj, config2_ps, config3_awproj, config4_jobs,
    config5, config5_ps, chunk_values, C5_CHUNK_ROWS, tiny_workload,
)
