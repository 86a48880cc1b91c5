"""Convolution-function table (the CFCache of the paper's AWP framework).

Paper: Table AWP-CFSETUP composes the kernel from the prolate spheroidal
taper (PS), the antenna aperture term (A) and the W-term (W); the ConvFunc
component computes c_ij and the CFCache holds the result (physical
architecture section).  The construction itself is not given; the reading
used here is:

  screen   S(l_j, m_i) = a_j a_i T(l_j) T(m_i) [B(rho)] [W_k(l, m)] on the
           (M+1) x (M+1) points l_j = j Lx / M, j = -M/2..M/2, Lx = nx dl
           (likewise m), a_j = 1/2 at j = +-M/2 and 1 elsewhere (trapezoid
           end weights: the screen stays even, so real even terms give a
           real kernel and K_{-w} = conj K_w holds), with
           T(l) = psi_0(c, 2 l / Lx), c = pi S_ps / 2            (PS term)
           B(rho) = [2 J1(x)/x]^2, x = pi D nu_fg rho / c_light   (A term,
                    power pattern of identical dishes, diagonal Mueller)
           W_k = exp(-2 pi i w_k (sqrt(1 - l^2 - m^2) - 1)), 0 outside the
                 unit circle, w_k = k w_max / (n_w - 1)            (W term)
  kernel   K(n_u, n_v) = sum_{j,i} S e^{-2 pi i (n_u j + n_v i) / (O M)},
           the length-O*M DFT of the zero-padded screen (library FFT here)
  table    C[fg][k][o_v + O/2][o_u + O/2][t_v + h][t_u + h]
             = conj K(o_u - O t_u, o_v - O t_v) / (M^2 T(0)^2)
           for o in [-O/2, O/2] (O + 1 offsets) and t in [-h_k, h_k].

The sparse Mueller matrix of CFs (the F M^DD of the AWP framework's
VisResampler; the paper gives no polarised beam model).  Reading: linear
feeds, correlations XX, XY, YX, YY indexed q = 2 q1 + q2 (X = 0, Y = 1),
one real symmetric Jones matrix shared by all antennas,

  J = [[E_X, d], [d, E_Y]],  a(x) = 2 J1(x) / x,  s = pi D nu_fg / c_light,
  E_X(l, m) = a(s sqrt((l / (1 + eta))^2 + (m / (1 - eta))^2))   (E_Y: eta -> -eta)
  d(l, m)   = kappa (s l) (s m) a(s rho)                           (cross-polar leakage)

so that M^DD = J (x) J (Eq. ME with identical antennas), M[q][p] =
J[q1][p1] J[q2][p2].  Every element is even in (l, m), so K_{-w} = conj K_w
still holds for each.  The distinct products ("kinds") are E_X^2, E_Y^2,
E_X E_Y (order 0 in d), E_X d, E_Y d (order 1) and d^2 (order 2); pol_beam
= n keeps the elements of order below n (1: the four diagonal terms, 2:
twelve, 3: all sixteen).  With eta = kappa = 0 every diagonal kind is the
power pattern a^2 of the scalar A term and the others vanish.  The table
holds the kinds one after the other, each laid out as the scalar table.

With this normalisation the un-cropped tap sum of every offset is exactly 1.
Storage forms: f64; f32 by round-to-nearest-even; f16 / bf16 as
RNE(C * 2^e_k) with e_k per plane chosen so that the largest component
magnitude times 2^e_k lies in [0.5, 1).
"""

from dataclasses import dataclass

import numpy as np
from scipy import fft as sfft
from scipy import special

from .conventions import C_LIGHT, half_widths, plane_offsets, screen_size
from .pswf import pswf_nystrom

TERM_PS, TERM_W, TERM_A = 1, 2, 4


@dataclass
class OracleCF:
    table: np.ndarray        # complex128, flat
    plane_off: np.ndarray    # int64 [n_fg * n_w]
    h: np.ndarray            # int32 [n_w]
    O: int
    n_w: int
    n_fg: int
    w_max: float
    M: int
    terms: int
    n_kind: int = 1          # Mueller kinds held (1: the scalar beam)
    kind_elems: int = 0      # complex elements per kind
    mueller: np.ndarray = None   # int32 [4][4] kind of M[q][p], -1 not kept (None: scalar)

    def sub(self, fg, k, ov, ou, kind=0):
        """S x S sub-kernel for offset (ov, ou) in [-O/2, O/2]."""
        S = 2 * int(self.h[k]) + 1
        no = self.O + 1
        base = kind * self.kind_elems + int(self.plane_off[fg * self.n_w + k]) + \
            ((ov + self.O // 2) * no + (ou + self.O // 2)) * S * S
        return self.table[base:base + S * S].reshape(S, S)

    def plane(self, fg, k, kind=0):
        S = 2 * int(self.h[k]) + 1
        no = self.O + 1
        base = kind * self.kind_elems + int(self.plane_off[fg * self.n_w + k])
        return self.table[base:base + no * no * S * S].reshape(no, no, S, S)


# --- polarised beam: Jones elements and Mueller kinds ------------------------

KINDS = (("ex", "ex"), ("ey", "ey"), ("ex", "ey"), ("ex", "d"), ("ey", "d"), ("d", "d"))
N_KIND = {0: 1, 1: 3, 2: 5, 3: 6}


def mueller_kinds(pol_beam):
    """[4][4] int32: kind index of M[q][p] = J[q1][p1] J[q2][p2], or -1 when
    its order in the leakage d is pol_beam or more."""
    sym = (("ex", "d"), ("d", "ey"))
    out = np.full((4, 4), -1, np.int32)
    for q in range(4):
        q1, q2 = divmod(q, 2)
        for p in range(4):
            p1, p2 = divmod(p, 2)
            pair = (sym[q1][p1], sym[q2][p2])
            order = pair.count("d")
            if order < pol_beam:
                key = tuple(sorted(pair, key=["ex", "ey", "d"].index))
                out[q, p] = KINDS.index(key)
    return out


def airy_voltage(x):
    x = np.asarray(x, dtype=np.float64)
    out = np.ones_like(x)
    nz = x != 0
    out[nz] = 2.0 * special.j1(x[nz]) / x[nz]
    return out


def jones_linear(l, m, nu, dish_m, eta, kappa):
    """(E_X, E_Y, d) at direction cosines (l, m) for frequency nu."""
    s = np.pi * dish_m * nu / C_LIGHT
    l = np.asarray(l, np.float64)
    m = np.asarray(m, np.float64)
    ex = airy_voltage(s * np.sqrt((l / (1.0 + eta)) ** 2 + (m / (1.0 - eta)) ** 2))
    ey = airy_voltage(s * np.sqrt((l / (1.0 - eta)) ** 2 + (m / (1.0 + eta)) ** 2))
    d = kappa * (s * l) * (s * m) * airy_voltage(s * np.sqrt(l * l + m * m))
    return ex, ey, d


def kind_beam(kind, l, m, nu, dish_m, eta, kappa):
    ex, ey, d = jones_linear(l, m, nu, dish_m, eta, kappa)
    f = {"ex": ex, "ey": ey, "d": d}
    a, b = KINDS[kind]
    return f[a] * f[b]


def airy_power(x):
    x = np.asarray(x, dtype=np.float64)
    out = np.ones_like(x)
    nz = x != 0
    b = 2.0 * special.j1(x[nz]) / x[nz]
    out[nz] = b * b
    return out


def screen(M, nx, ny, cell_l, cell_m, terms, ps_support, w_k, nu_fg, dish_m, psi=None,
           shift=(0.0, 0.0), pol_beam=0, kind=0, eta=0.0, kappa=0.0):
    """(M+1) x (M+1) complex128 screen, rows = m (v axis), columns = l (u
    axis), sample j at l = j Lx / M for j = -M/2..M/2, edge samples halved.
    `shift` evaluates every term at (l - dl, m - dm) (used only by a test of
    the pointing phasor).  With pol_beam > 0 the A term is the Mueller kind
    `kind` of the polarised beam instead of the power pattern."""
    Lx, Ly = nx * cell_l, ny * cell_m
    j = np.arange(-(M // 2), M // 2 + 1)
    l = j * Lx / M - shift[0]
    m = j * Ly / M - shift[1]
    a = np.ones(M + 1)
    a[0] = a[-1] = 0.5
    ll, mm = np.meshgrid(l, m)          # [i][j] = (m_i, l_j)
    s = np.outer(a, a).astype(np.complex128)
    if terms & TERM_PS:
        if psi is None:
            psi = pswf_nystrom(np.pi * ps_support / 2.0)[0]
        s *= np.outer(psi(2.0 * m / Ly), psi(2.0 * l / Lx))
    if terms & TERM_A:
        if pol_beam:
            s *= kind_beam(kind, ll, mm, nu_fg, dish_m, eta, kappa)
        else:
            rho = np.sqrt(ll * ll + mm * mm)
            s *= airy_power(np.pi * dish_m * nu_fg * rho / C_LIGHT)
    if terms & TERM_W:
        r2 = ll * ll + mm * mm
        inside = r2 < 1.0
        n1 = np.zeros_like(r2)
        # sqrt(1 - r^2) - 1 written without cancellation
        n1[inside] = -r2[inside] / (1.0 + np.sqrt(1.0 - r2[inside]))
        wt = np.exp(-2j * np.pi * w_k * n1)
        wt[~inside] = 0.0
        s *= wt
    return s


def kernel_fft(scr, O):
    """K[n_v mod OM, n_u mod OM] = sum_{i,j} S[i][j] e^{-2 pi i (n_u j + n_v i)/(OM)},
    j, i = -M/2..M/2."""
    M = scr.shape[0] - 1
    N = O * M
    pad = np.zeros((N, N), np.complex128)
    idx = np.arange(-(M // 2), M // 2 + 1) % N
    if O == 1:
        # +M/2 and -M/2 coincide modulo M: their halves add
        pad[np.ix_(idx[:-1], idx[:-1])] += scr[:-1, :-1]
        pad[np.ix_(idx[:-1], [idx[-1]])] += scr[:-1, -1:]
        pad[np.ix_([idx[-1]], idx)] += scr[-1:, :]
    else:
        pad[np.ix_(idx, idx)] = scr
    return sfft.fft2(pad, workers=-1)


def crop_plane(K, M, O, h, t0_sq):
    """[O+1][O+1][S][S] = conj K(o_u - O t_u, o_v - O t_v) / (M^2 T(0)^2)."""
    N = O * M
    o = np.arange(-(O // 2), O // 2 + 1)
    t = np.arange(-h, h + 1)
    n = (o[:, None] - O * t[None, :]) % N          # [o][t]
    # K indexed [n_v][n_u]; output [ov][ou][tv][tu]
    out = K[n[:, None, :, None], n[None, :, None, :]]
    return np.conj(out) / (M * M * t0_sq)


def build_cf(grid, cf, n_nodes=64, planes=None, compact=False):
    """Build the FP64 table for a synth GridSetup / CFSetup pair.  `planes`
    (a set of (fg, k)) restricts the work to those planes; the others stay 0,
    or with compact=True are not stored at all (offset -1), which keeps the
    table of a large configuration small when only a few planes are needed."""
    h = half_widths(cf.n_w, cf.h_min, cf.h_max)
    M = screen_size(h, cf.screen_m)
    O = cf.oversample
    n_fg = cf.n_fg
    off, total = plane_offsets(n_fg, h, O)
    if compact:
        if planes is None:
            raise ValueError("compact needs the list of planes")
        off = np.full(n_fg * cf.n_w, -1, np.int64)
        total = 0
        for g, k in sorted(planes):
            off[g * cf.n_w + k] = total
            total += (O + 1) ** 2 * (2 * int(h[k]) + 1) ** 2
    pol_beam = int(getattr(cf, "pol_beam", 0))
    if pol_beam and not cf.terms & TERM_A:
        raise ValueError("a polarised beam needs the A term")
    eta = float(getattr(cf, "beam_ellipticity", 0.0))
    kappa = float(getattr(cf, "beam_leakage", 0.0))
    n_kind = N_KIND[pol_beam]
    table = np.zeros(n_kind * total, np.complex128)
    psi = None
    t0 = 1.0
    if cf.terms & TERM_PS:
        psi = pswf_nystrom(np.pi * cf.ps_support / 2.0, n_nodes)[0]
        t0 = float(psi(0.0)[0])
    for kind in range(n_kind):
        for g in range(n_fg):
            for k in range(cf.n_w):
                if planes is not None and (g, k) not in planes:
                    continue
                w_k = k * cf.w_max / (cf.n_w - 1) if cf.n_w > 1 else 0.0
                scr = screen(M, grid.nx, grid.ny, grid.cell_l, grid.cell_m, cf.terms,
                             cf.ps_support, w_k, float(cf.fg_hz[g]), cf.dish_m, psi,
                             pol_beam=pol_beam, kind=kind, eta=eta, kappa=kappa)
                K = kernel_fft(scr, O)
                pl = crop_plane(K, M, O, int(h[k]), t0 * t0)
                base = kind * total + int(off[g * cf.n_w + k])
                table[base:base + pl.size] = pl.ravel()
    return OracleCF(table=table, plane_off=off, h=h, O=O, n_w=cf.n_w, n_fg=n_fg,
                    w_max=cf.w_max, M=M, terms=cf.terms, n_kind=n_kind, kind_elems=total,
                    mueller=mueller_kinds(pol_beam) if pol_beam else None)


# --- storage forms ---------------------------------------------------------

def plane_scale_exponents(ocf):
    """e per (kind, fg, k), flat in that order: largest component magnitude
    times 2^e in [0.5, 1)."""
    npl = ocf.n_fg * ocf.n_w
    out = np.zeros(ocf.n_kind * npl, np.int32)
    for kind in range(ocf.n_kind):
        for g in range(ocf.n_fg):
            for k in range(ocf.n_w):
                p = ocf.plane(g, k, kind)
                mx = max(np.max(np.abs(p.real)), np.max(np.abs(p.imag)))
                if mx == 0:
                    continue
                _, e = np.frexp(mx)
                out[kind * npl + g * ocf.n_w + k] = -int(e)
    return out


def round_bf16(x):
    """Round-to-nearest-even of float64 values to 8 significant bits
    (bfloat16 within its normal range), returned as float64."""
    x = np.asarray(x, np.float64)
    mant, ex = np.frexp(x)                 # x = mant * 2^ex, |mant| in [0.5, 1)
    return np.ldexp(np.rint(mant * 256.0), ex - 8)


def quantised_table(ocf, storage):
    """The table as the given storage form decodes it, in float64/complex128:
    'f64', 'f32', 'f16', 'bf16'."""
    t = ocf.table
    if storage == "f64":
        return t.copy()
    if storage == "f32":
        return t.astype(np.complex64).astype(np.complex128)
    ex = plane_scale_exponents(ocf)
    out = np.empty_like(t)
    npl = ocf.n_fg * ocf.n_w
    for kind in range(ocf.n_kind):
        for g in range(ocf.n_fg):
            for k in range(ocf.n_w):
                S = 2 * int(ocf.h[k]) + 1
                base = kind * ocf.kind_elems + int(ocf.plane_off[g * ocf.n_w + k])
                n = (ocf.O + 1) ** 2 * S * S
                e = int(ex[kind * npl + g * ocf.n_w + k])
                v = np.ldexp(t[base:base + n].real, e), np.ldexp(t[base:base + n].imag, e)
                if storage == "f16":
                    q = [a.astype(np.float16).astype(np.float64) for a in v]
                elif storage == "bf16":
                    q = [round_bf16(a) for a in v]
                else:
                    raise ValueError(storage)
                out[base:base + n] = np.ldexp(q[0], -e) + 1j * np.ldexp(q[1], -e)
    return out
