"""Conventions the paper leaves open, as read for this oracle.

The paper states gridding G and degridding D (Eqs. ME-MOD-GRIDDED and
IMAGE-MOD) without an index convention, kernel family, support rule or
normalisation.  The readings below are the oracle's; the GPU library
implements the same readings in its own code.

* Pixel (iy, ix) <-> (m, l) = ((iy - ny/2) dm, (ix - nx/2) dl); u = 0 sits at
  pixel nx/2; the uv cell is du = 1 / (nx dl).
* Per channel (FP64, left to right, no contraction):
      s  = nu / c
      kx = ((s * nx) * dl) * O        ky = ((s * ny) * dm) * O
      kw = s * ((n_w - 1) / w_max)    (0 when n_w == 1)
      ox = (nx/2) * O + 0.5           oy = (ny/2) * O + 0.5
* Support of w-plane k: S_k = 2 h_k + 1 with h_k growing linearly in k from
  h_min to h_max, rounded half up.
"""

import numpy as np

C_LIGHT = 299792458.0


def half_widths(n_w, h_min, h_max):
    """h_k = h_min + floor((2 (h_max - h_min) k + n_w - 1) / (2 (n_w - 1)))."""
    if n_w == 1:
        return np.array([h_min], dtype=np.int32)
    k = np.arange(n_w, dtype=np.int64)
    return (h_min + (2 * (h_max - h_min) * k + n_w - 1) // (2 * (n_w - 1))).astype(np.int32)


def channel_constants(freq_hz, nx, ny, cell_l, cell_m, O, n_w, w_max):
    """Return kx, ky, kw (arrays over channels) and ox, oy (floats)."""
    kx = np.empty(len(freq_hz))
    ky = np.empty(len(freq_hz))
    kw = np.empty(len(freq_hz))
    for i, nu in enumerate(freq_hz):
        s = float(nu) / C_LIGHT
        kx[i] = ((s * nx) * cell_l) * O
        ky[i] = ((s * ny) * cell_m) * O
        kw[i] = s * ((n_w - 1) / w_max) if n_w > 1 else 0.0
    ox = (nx // 2) * O + 0.5
    oy = (ny // 2) * O + 0.5
    return kx, ky, kw, float(ox), float(oy)


def screen_size(h, screen_m=0):
    """M = smallest even number >= 2 * S_max (S_max = 2 max(h) + 1)."""
    if screen_m:
        return int(screen_m)
    smax = 2 * int(np.max(h)) + 1
    m = 2 * smax
    return m + (m % 2)


def plane_offsets(n_fg, h, O):
    """Offset, in complex elements, of plane (fg, k) in the table laid out as
    [fg][k][o_v + O/2][o_u + O/2][t_v + h_k][t_u + h_k]."""
    sizes = (O + 1) ** 2 * (2 * np.asarray(h, np.int64) + 1) ** 2
    off = np.zeros(n_fg * len(h), np.int64)
    acc = 0
    for g in range(n_fg):
        for k in range(len(h)):
            off[g * len(h) + k] = acc
            acc += int(sizes[k])
    return off, acc
