"""Mosaic imaging rows of the imaging-mode table (phase centre s(P) of each
pointing differs from the joint image centre s0; Eq. CIJ) -- test
infrastructure only.

Reading of Eq. CIJ for a pointing P with phase centre offset
(l_P, m_P) = s(P) - s0 (direction cosines) and antenna pointing offsets
ds_i:
  * the visibilities are moved from the phase centre s(P) to the joint image
    centre s0: V_0 = V_P exp(-2 pi i (u l_P + v m_P)), u and v in
    wavelengths (the flat-sky shift; the w-term of the change of phase
    centre is not applied);
  * the kernel is shifted by s(P) - s0 + (ds_i + ds_j) / 2, with the loss
    factor f(ds_i - ds_j) unchanged: exactly the pointing phasor of the
    single-pointing rows applied to "virtual antennas" (field, antenna)
    whose offsets are ds_a + s(P) - s0.
Degridding returns to the field's phase centre with the inverse factor.

FP64, plain loops over rows.  The phase argument a = (u_m nu / c) l_P +
(v_m nu / c) m_P is formed in FP64 and reduced modulo 1 before the sine
and cosine.
"""

import numpy as np

from .conventions import C_LIGHT


def rephase(vis, uvw_m, freq_hz, field, field_dlm, to_image_centre=True):
    """vis [nrow, nchan, npol] moved from each row's field phase centre to
    the image centre (to_image_centre=True) or back.  Rows whose field is
    outside [0, nfield) are left unchanged."""
    vis = np.array(vis, np.complex128, copy=True)
    uvw_m = np.asarray(uvw_m, np.float64)
    s = np.asarray(freq_hz, np.float64) / C_LIGHT
    field_dlm = np.asarray(field_dlm, np.float64).reshape(-1, 2)
    nf = field_dlm.shape[0]
    sign = -1.0 if to_image_centre else 1.0
    for r in range(vis.shape[0]):
        f = int(field[r])
        if f < 0 or f >= nf:
            continue
        lp, mp = field_dlm[f]
        for c in range(vis.shape[1]):
            u = uvw_m[r, 0] * s[c]
            v = uvw_m[r, 1] * s[c]
            a = u * lp + v * mp
            a = a - np.rint(a)
            ph = sign * 2.0 * np.pi * a
            vis[r, c, :] *= complex(np.cos(ph), np.sin(ph))
    return vis


def virtual_antennas(ant1, ant2, nant, field, field_dlm, ant_dlm=None):
    """(ant1', ant2', ant_dlm') with antenna a of field f renumbered
    f * nant + a and offset ant_dlm[a] + field_dlm[f]."""
    field = np.asarray(field, np.int64)
    field_dlm = np.asarray(field_dlm, np.float64).reshape(-1, 2)
    base = np.zeros((nant, 2)) if ant_dlm is None else np.asarray(ant_dlm, np.float64)
    nf = field_dlm.shape[0]
    dlm = np.zeros((nf * nant, 2))
    for f in range(nf):
        for a in range(nant):
            dlm[f * nant + a] = base[a] + field_dlm[f]
    a1 = (field * nant + np.asarray(ant1, np.int64)).astype(np.int32)
    a2 = (field * nant + np.asarray(ant2, np.int64)).astype(np.int32)
    return a1, a2, dlm
