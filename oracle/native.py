"""ctypes binding of the oracle's C loops (gridding.c).

TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
benchmark's CPU-baseline leg.  `build()` compiles gridding.c with gcc
(-O2 -ffp-contract=off -fopenmp); nothing here touches a GPU.
"""

import ctypes as C
import os
import subprocess

import numpy as np

from .conventions import C_LIGHT, channel_constants

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gridding.c")
_LIB = os.path.join(_HERE, "liboracle_gridding.so")
_lib = None


def build(force=True):
    """Compile the oracle's C loops.  Always recompiles when force is set."""
    if not force and os.path.exists(_LIB):
        return _LIB
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
           "-shared", "-std=c11", "-D_DEFAULT_SOURCE", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


class OCtx(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("npol", C.c_int32), ("nplane", C.c_int32),
        ("O", C.c_int32), ("n_w", C.c_int32), ("n_fg", C.c_int32), ("psf", C.c_int32),
        ("h", C.c_void_p), ("plane_off", C.c_void_p), ("cf", C.c_void_p),
        ("nrow", C.c_int64), ("nchan", C.c_int32),
        ("uvw", C.c_void_p), ("kx", C.c_void_p), ("ky", C.c_void_p), ("kw", C.c_void_p),
        ("ox", C.c_double), ("oy", C.c_double),
        ("chan_plane", C.c_void_p), ("chan_fg", C.c_void_p),
        ("ant1", C.c_void_p), ("ant2", C.c_void_p), ("ant_dlm", C.c_void_p),
        ("f_scale", C.c_void_p), ("du_dl", C.c_double), ("dv_dm", C.c_double),
        ("mueller", C.c_void_p), ("kind_stride", C.c_int64),
    ]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        l = C.CDLL(_LIB)
        for name in ("oracle_map", "oracle_sumwt", "oracle_grid", "oracle_degrid",
                     "oracle_hermitian_sym", "oracle_psf_mirror"):
            getattr(l, name).restype = None
        _lib = l
    return _lib


def _p(a):
    return a.ctypes.data if a is not None else None


class Problem:
    """Everything the C loops need, kept alive for the duration of calls.

    uvw [nrow,3] f64 metres; freq [nchan]; chan_plane/chan_fg [nchan];
    grid geometry (nx, ny, npol, nplane, cell_l, cell_m); table from
    oracle.cfbuild; optional pointing offsets (ant1, ant2, ant_dlm, dish_m).
    """

    def __init__(self, uvw, freq_hz, chan_plane, chan_fg, nx, ny, npol, nplane,
                 cell_l, cell_m, ocf, table=None, ant1=None, ant2=None, ant_dlm=None,
                 dish_m=25.0, psf=False):
        self.uvw = np.ascontiguousarray(uvw, np.float64)
        self.freq = np.ascontiguousarray(freq_hz, np.float64)
        self.chan_plane = np.ascontiguousarray(chan_plane, np.int32)
        self.chan_fg = np.ascontiguousarray(chan_fg, np.int32)
        self.nx, self.ny, self.npol, self.nplane = nx, ny, npol, nplane
        self.ocf = ocf
        tab = ocf.table if table is None else table
        self.table = np.ascontiguousarray(tab, np.complex128)
        self.h = np.ascontiguousarray(ocf.h, np.int32)
        self.plane_off = np.ascontiguousarray(ocf.plane_off, np.int64)
        kx, ky, kw, ox, oy = channel_constants(self.freq, nx, ny, cell_l, cell_m,
                                               ocf.O, ocf.n_w, ocf.w_max)
        self.kx, self.ky, self.kw = kx, ky, kw
        self.po = ant1 is not None and ant_dlm is not None
        if self.po:
            self.ant1 = np.ascontiguousarray(ant1, np.int32)
            self.ant2 = np.ascontiguousarray(ant2, np.int32)
            self.ant_dlm = np.ascontiguousarray(ant_dlm, np.float64)
            self.f_scale = np.ascontiguousarray(np.pi * dish_m * self.freq / C_LIGHT)
        else:
            self.ant1 = self.ant2 = self.ant_dlm = self.f_scale = None
        c = OCtx()
        c.nx, c.ny, c.npol, c.nplane = nx, ny, npol, nplane
        c.O, c.n_w, c.n_fg, c.psf = ocf.O, ocf.n_w, ocf.n_fg, int(psf)
        c.h, c.plane_off, c.cf = _p(self.h), _p(self.plane_off), _p(self.table)
        c.nrow, c.nchan = self.uvw.shape[0], self.freq.shape[0]
        c.uvw, c.kx, c.ky, c.kw = _p(self.uvw), _p(kx), _p(ky), _p(kw)
        c.ox, c.oy = ox, oy
        c.chan_plane, c.chan_fg = _p(self.chan_plane), _p(self.chan_fg)
        c.ant1, c.ant2, c.ant_dlm = _p(self.ant1), _p(self.ant2), _p(self.ant_dlm)
        c.f_scale = _p(self.f_scale)
        c.du_dl = 1.0 / (nx * cell_l)
        c.dv_dm = 1.0 / (ny * cell_m)
        self.mueller = None
        if getattr(ocf, "mueller", None) is not None:
            if npol != 4:
                raise ValueError("a Mueller table needs the four correlations")
            self.mueller = np.ascontiguousarray(ocf.mueller, np.int32).ravel()
        c.mueller = _p(self.mueller)
        c.kind_stride = int(getattr(ocf, "kind_elems", 0))
        self.ctx = c
        self.cell_l, self.cell_m = cell_l, cell_m
        self.nrow, self.nchan = c.nrow, c.nchan
        self.partial_table = bool(np.any(self.plane_off < 0))

    def _check_planes(self):
        """With a table that holds only some planes, every kept sample must
        use one of them (checked with this oracle's own index map)."""
        if not self.partial_table:
            return
        m = self.map().reshape(-1, 8)
        cp = np.tile(self.chan_plane, self.nrow)
        kept = (m[:, 6] == 1) & (cp >= 0)
        idx = m[kept, 7].astype(np.int64) * self.ocf.n_w + m[kept, 4]
        if np.any(self.plane_off[idx] < 0):
            raise ValueError("a kept sample needs a CF plane the table does not hold")

    @classmethod
    def from_workload(cls, wl, ocf, table=None, psf=False, pointing=None):
        """pointing: None = as the workload has it; False = off."""
        po = wl.ant_dlm is not None if pointing is None else bool(pointing)
        g = wl.grid
        return cls(wl.obs.uvw, wl.obs.freq_hz, wl.chan_plane, wl.chan_fg, g.nx, g.ny,
                   g.npol, g.nplane, g.cell_l, g.cell_m, ocf, table=table,
                   ant1=wl.obs.ant1 if po else None, ant2=wl.obs.ant2 if po else None,
                   ant_dlm=wl.ant_dlm if po else None, dish_m=wl.cf.dish_m, psf=psf)

    def with_psf(self, flag=True):
        import copy
        q = copy.copy(self)
        q.ctx = OCtx.from_buffer_copy(self.ctx)
        q.ctx.psf = int(flag)
        return q

    # -- calls ---------------------------------------------------------------
    def map(self):
        out = np.zeros((self.nrow, self.nchan, 8), np.int32)
        lib().oracle_map(C.byref(self.ctx), C.c_void_p(_p(out)))
        return out

    def grid_shape(self):
        return (self.nplane, self.npol, self.ny, self.nx)

    def sumwt(self, weight):
        w = np.ascontiguousarray(weight, np.float64)
        s = np.zeros((self.nplane, self.npol), np.float64)
        cnt = np.zeros(3, np.int64)
        lib().oracle_sumwt(C.byref(self.ctx), C.c_void_p(_p(w)), C.c_void_p(_p(s)),
                           C.c_void_p(_p(cnt)))
        return s, cnt

    def grid(self, vis, weight, nthreads=0, unit_vis=False, out=None):
        self._check_planes()
        v = np.ascontiguousarray(vis, np.complex128)
        w = np.ascontiguousarray(weight, np.float64)
        g = np.zeros(self.grid_shape(), np.complex128) if out is None else out
        lib().oracle_grid(C.byref(self.ctx), C.c_void_p(_p(v)), C.c_void_p(_p(w)),
                          C.c_void_p(_p(g)), C.c_int(int(unit_vis)), C.c_int(nthreads))
        return g

    def degrid(self, grid, weight=None, nthreads=0):
        self._check_planes()
        g = np.ascontiguousarray(grid, np.complex128)
        w = None if weight is None else np.ascontiguousarray(weight, np.float64)
        v = np.zeros((self.nrow, self.nchan, self.npol), np.complex128)
        lib().oracle_degrid(C.byref(self.ctx), C.c_void_p(_p(g)),
                            C.c_void_p(_p(w)) if w is not None else None,
                            C.c_void_p(_p(v)), C.c_int(nthreads))
        return v

    def psf(self, weight, nthreads=0):
        """PSF grid by symmetrisation of the unit-visibility weight grid
        (footprints restricted to [1, N-1]); returns (psf, sumwt, counters)."""
        q = self.with_psf(True)
        gw = q.grid(np.zeros(1, np.complex128), weight,
                    nthreads=nthreads, unit_vis=True)
        out = np.zeros_like(gw)
        lib().oracle_hermitian_sym(C.byref(q.ctx), C.c_void_p(_p(gw)), C.c_void_p(_p(out)))
        s, cnt = q.sumwt(weight)
        return out, s, cnt

    def psf_mirror(self, weight):
        q = self.with_psf(True)
        w = np.ascontiguousarray(weight, np.float64)
        g = np.zeros(self.grid_shape(), np.complex128)
        lib().oracle_psf_mirror(C.byref(q.ctx), C.c_void_p(_p(w)), C.c_void_p(_p(g)))
        return g
