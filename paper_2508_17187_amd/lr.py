"""ctypes binding of liblr.so (argument marshalling only).

The functions keep the C names (lr_cf_build, lr_grid, lr_degrid,
lr_make_psf, lr_sumwt, lr_debug_map, lr_plan_build, ...).  Device memory
and streams come from PyTorch; every step of the computation runs in the
library's HIP kernels.  There is no CPU fallback: importing this module
without the built library raises.
"""

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblr.so")

LR_OK, LR_E_ARG, LR_E_DTYPE, LR_E_WORKSPACE, LR_E_CF, LR_E_DEVICE, LR_E_RANGE = 0, -1, -2, -3, -4, -5, -6
LR_F64, LR_F32, LR_F32_CF16, LR_F32_CFBF16 = 0, 1, 2, 3
LR_TERM_PS, LR_TERM_W, LR_TERM_A = 1, 2, 4
LR_OP_CF_BUILD, LR_OP_GRID, LR_OP_DEGRID, LR_OP_PSF, LR_OP_SUMWT = 0, 1, 2, 3, 4

PRECISIONS = {"f64": LR_F64, "f32": LR_F32, "f16cf": LR_F32_CF16, "bf16cf": LR_F32_CFBF16}


class LRError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (_status_name(status), msg))
        self.status = status


def _status_name(s):
    return {0: "LR_OK", -1: "LR_E_ARG", -2: "LR_E_DTYPE", -3: "LR_E_WORKSPACE", -4: "LR_E_CF",
            -5: "LR_E_DEVICE", -6: "LR_E_RANGE"}.get(s, "LR_E_%d" % s)


class GridSpec(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("npol", C.c_int32),
                ("nplane", C.c_int32), ("cell_l", C.c_double), ("cell_m", C.c_double)]


class CFSpec(C.Structure):
    _fields_ = [("terms", C.c_uint32), ("oversample", C.c_int32), ("ps_support", C.c_int32),
                ("n_w", C.c_int32), ("w_max", C.c_double), ("h_min", C.c_int32),
                ("h_max", C.c_int32), ("n_fg", C.c_int32), ("fg_hz", C.c_void_p),
                ("dish_m", C.c_double), ("screen_m", C.c_int32), ("storage", C.c_int32),
                ("pol_beam", C.c_int32), ("beam_ellipticity", C.c_double),
                ("beam_leakage", C.c_double)]


class VisDesc(C.Structure):
    _fields_ = [("nrow", C.c_int64), ("nchan", C.c_int32), ("npol", C.c_int32),
                ("nant", C.c_int32), ("uvw", C.c_void_p), ("freq_hz", C.c_void_p),
                ("chan_plane", C.c_void_p), ("chan_fg", C.c_void_p), ("vis", C.c_void_p),
                ("weight", C.c_void_p), ("ant1", C.c_void_p), ("ant2", C.c_void_p),
                ("ant_dlm", C.c_void_p), ("plan", C.c_void_p)]


EXPORTS = {
    "lr_cf_bytes": (C.c_size_t, [C.c_void_p, C.c_void_p]),
    "lr_workspace_bytes": (C.c_size_t, [C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]),
    "lr_cf_build": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p,
                              C.c_size_t, C.c_void_p, C.c_void_p]),
    "lr_cf_attach": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "lr_cf_free": (None, [C.c_void_p]),
    "lr_cf_scale_exponents": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "lr_cf_layout": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "lr_cf_kinds": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "lr_plan_bytes": (C.c_size_t, [C.c_void_p, C.c_void_p, C.c_int]),
    "lr_plan_build": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_size_t,
                                C.c_void_p, C.c_void_p]),
    "lr_plan_free": (None, [C.c_void_p]),
    "lr_plan_packed_bytes": (C.c_size_t, [C.c_void_p]),
    "lr_plan_pack": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p]),
    "lr_plan_info": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "lr_set_profile_events": (C.c_int, [C.c_void_p, C.c_void_p]),
    "lr_set_deterministic": (C.c_int, [C.c_int32]),
    "lr_deterministic": (C.c_int32, []),
    "lr_grid": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                          C.c_void_p, C.c_size_t, C.c_void_p]),
    "lr_grid_overwrite": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p,
                                    C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "lr_grid_static": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p,
                                 C.c_void_p, C.c_void_p]),
    "lr_degrid": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p,
                            C.c_void_p, C.c_size_t, C.c_void_p]),
    "lr_make_psf": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p,
                              C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "lr_sumwt": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                           C.c_size_t, C.c_void_p]),
    "lr_debug_map": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]),
    "lr_gcf": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p]),
    "lr_rephase": (C.c_int, [C.c_int64, C.c_int32, C.c_int32, C.c_int, C.c_void_p, C.c_void_p,
                             C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                             C.c_void_p]),
    "lr_cal_vavg": (C.c_int, [C.c_int64, C.c_int32, C.c_int32, C.c_int, C.c_void_p, C.c_void_p,
                              C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                              C.c_int32, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p,
                              C.c_void_p, C.c_void_p]),
    "lr_cal_solve": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int64, C.c_double,
                               C.c_double, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                               C.c_void_p]),
    "lr_hogbom_work_bytes": (C.c_size_t, [C.c_int32, C.c_int32]),
    "lr_hogbom": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int,
                            C.c_double, C.c_double, C.c_int32, C.c_void_p, C.c_void_p,
                            C.c_size_t, C.c_void_p]),
    "lr_image_normalize": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_void_p, C.c_void_p]),
    "lr_ps_taper": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "lr_pb_image": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "lr_image_normalize_pb": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                                        C.c_void_p, C.c_void_p]),
    "lr_status_str": (C.c_char_p, [C.c_int]),
    "lr_last_error": (C.c_char_p, []),
}

_lib = None


def lib():
    """Load liblr.so; raises when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("liblr.so is not built (run python -m paper_2508_17187_amd.build); "
                              "there is no fallback path")
        l = C.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            f = getattr(l, name)
            f.restype = res
            f.argtypes = args
        _lib = l
    return _lib


def _check(status):
    if status != LR_OK:
        raise LRError(status, lib().lr_last_error().decode())


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _on_stream(t, stream):
    """Tell torch's caching allocator that `t` is used by work on `stream`
    (when it is not the current stream), so that its block is not handed to
    other work before that stream's kernels are done with it."""
    if t is not None and stream is not None and stream != torch.cuda.current_stream():
        t.record_stream(stream)
    return t


def _vis_dtype(precision):
    return (torch.complex128, torch.float64) if precision == LR_F64 else (torch.complex64,
                                                                          torch.float32)


# ---------------------------------------------------------------------------
class CF:
    """A CF table built on the GPU (lr_cf_build) and its host handle."""

    def __init__(self, grid, spec, device="cuda", stream=None, blob=None):
        self.grid = grid if isinstance(grid, GridSpec) else GridSpec(*grid)
        self.fg = np.ascontiguousarray(spec.pop("fg_hz"), np.float64)
        self.spec = CFSpec(fg_hz=self.fg.ctypes.data, **spec)
        self.precision = self.spec.storage
        L = lib()
        nbytes = L.lr_cf_bytes(C.byref(self.spec), C.byref(self.grid))
        if nbytes == 0:
            raise LRError(LR_E_ARG, L.lr_last_error().decode())
        self.nbytes = nbytes
        self.handle = C.c_void_p()
        if blob is None:
            self.blob = torch.empty(nbytes, dtype=torch.uint8, device=device)
            wb = L.lr_workspace_bytes(LR_OP_CF_BUILD, C.byref(self.spec), C.byref(self.grid),
                                      None, self.precision)
            work = torch.empty(max(wb, 1), dtype=torch.uint8, device=device)
            _on_stream(self.blob, stream)
            _on_stream(work, stream)
            _check(L.lr_cf_build(C.byref(self.spec), C.byref(self.grid), _ptr(self.blob),
                                 nbytes, _ptr(work), wb, _stream(stream),
                                 C.byref(self.handle)))
            self._work = work      # kept until the CF build has run on the stream
        else:
            self.blob = blob
            _check(L.lr_cf_attach(C.byref(self.spec), C.byref(self.grid), _ptr(blob),
                                  blob.numel(), C.byref(self.handle)))

    def layout(self):
        off, eb, ne = C.c_size_t(), C.c_size_t(), C.c_int64()
        po = np.zeros(self.spec.n_fg * self.spec.n_w, np.int64)
        _check(lib().lr_cf_layout(self.handle, C.byref(off), C.byref(eb), C.byref(ne),
                                  po.ctypes.data_as(C.c_void_p)))
        return off.value, eb.value, ne.value, po

    def kinds(self):
        """(n_kind, kind_of [4][4]): the Mueller kinds the table holds and the
        kind of each element M[q][p] (-1: not held)."""
        n = C.c_int32()
        km = np.zeros(16, np.int32)
        _check(lib().lr_cf_kinds(self.handle, C.byref(n), km.ctypes.data_as(C.c_void_p)))
        return n.value, km.reshape(4, 4)

    def plane_host(self, fg, k, kind=0):
        """One (fg, k) plane of Mueller kind `kind` of an FP64 or FP32 table as
        complex128 on the host, flat in table order (test hook for tables too
        big to copy whole)."""
        off, eb, ne, po = self.layout()
        if eb not in (8, 16):
            raise ValueError("plane_host reads FP64 / FP32 tables")
        ke = ne // self.kinds()[0]
        i = fg * self.spec.n_w + k
        end = int(po[i + 1]) if i + 1 < len(po) else ke
        b0 = off + eb * (kind * ke + int(po[i]))
        raw = self.blob[b0:b0 + eb * (end - int(po[i]))].cpu().numpy()
        return raw.view(np.complex128 if eb == 16 else np.complex64).astype(np.complex128)

    def table_host(self):
        """The stored table decoded to complex128 on the host (test hook):
        fp16 / bf16 entries are divided by their plane's 2^e.  Kinds follow
        one another."""
        off, eb, ne, po = self.layout()
        raw = self.blob[off:off + eb * ne].cpu().numpy()
        if eb == 16:
            return raw.view(np.complex128).copy()
        if eb == 8:
            return raw.view(np.complex64).astype(np.complex128)
        u = raw.view(np.uint32)
        if self.precision == LR_F32_CF16:
            re = (u & 0xFFFF).astype(np.uint16).view(np.float16).astype(np.float64)
            im = (u >> 16).astype(np.uint16).view(np.float16).astype(np.float64)
        else:
            re = ((u & 0xFFFF) << 16).astype(np.uint32).view(np.float32).astype(np.float64)
            im = (u & 0xFFFF0000).astype(np.uint32).view(np.float32).astype(np.float64)
        out = re + 1j * im
        ex = self.scale_exponents()
        nk = self.kinds()[0]
        ke = ne // nk
        bounds = list(po) + [ke]
        for kind in range(nk):
            for i in range(len(po)):
                a, b = kind * ke + bounds[i], kind * ke + bounds[i + 1]
                e = -int(ex[kind * len(po) + i])
                out[a:b] = np.ldexp(out[a:b].real, e) + 1j * np.ldexp(out[a:b].imag, e)
        return out

    def scale_exponents(self, stream=None):
        n = self.spec.n_fg * self.spec.n_w * self.kinds()[0]
        out = np.zeros(n, np.int32)
        _check(lib().lr_cf_scale_exponents(self.handle, out.ctypes.data_as(C.c_void_p),
                                           _stream(stream)))
        return out

    def __del__(self):
        try:
            if self.handle:
                lib().lr_cf_free(self.handle)
                self.handle = C.c_void_p()
        except Exception:
            pass


class Vis:
    """Visibility data on the device plus the host channel tables.

    uvw: [nrow, 3] float64 tensor; freq_hz, chan_plane, chan_fg: host arrays;
    vis / weight: [nrow, nchan, npol] tensors (complex128/float64 or
    complex64/float32); ant1, ant2 (int32 [nrow]) and ant_dlm (float64
    [nant, 2]) switch the pointing phasor on."""

    def __init__(self, uvw, freq_hz, chan_plane=None, chan_fg=None, vis=None, weight=None,
                 npol=None, ant1=None, ant2=None, ant_dlm=None, plan=None):
        self.uvw = uvw
        self.freq = np.ascontiguousarray(freq_hz, np.float64)
        nchan = self.freq.shape[0]
        self.chan_plane = np.ascontiguousarray(
            np.zeros(nchan) if chan_plane is None else chan_plane, np.int32)
        self.chan_fg = None if chan_fg is None else np.ascontiguousarray(chan_fg, np.int32)
        self.vis = vis
        self.weight = weight
        self.npol = npol if npol is not None else (vis.shape[-1] if vis is not None else
                                                   weight.shape[-1])
        self.ant1, self.ant2, self.ant_dlm = ant1, ant2, ant_dlm
        self.plan = plan

    @property
    def nrow(self):
        return int(self.uvw.shape[0])

    @property
    def nchan(self):
        return int(self.freq.shape[0])

    def desc(self):
        d = VisDesc()
        d.nrow = self.nrow
        d.nchan = self.nchan
        d.npol = self.npol
        d.nant = 0 if self.ant_dlm is None else int(self.ant_dlm.shape[0])
        d.uvw = self.uvw.data_ptr()
        d.freq_hz = self.freq.ctypes.data
        d.chan_plane = self.chan_plane.ctypes.data
        d.chan_fg = None if self.chan_fg is None else self.chan_fg.ctypes.data
        d.vis = None if self.vis is None else self.vis.data_ptr()
        d.weight = None if self.weight is None else self.weight.data_ptr()
        d.ant1 = None if self.ant1 is None else self.ant1.data_ptr()
        d.ant2 = None if self.ant2 is None else self.ant2.data_ptr()
        d.ant_dlm = None if self.ant_dlm is None else self.ant_dlm.data_ptr()
        d.plan = None if self.plan is None else self.plan.handle.value
        return d

    def with_(self, **kw):
        import copy
        v = copy.copy(self)
        for k, x in kw.items():
            setattr(v, k, x)
        return v


class Plan:
    """Binning plan (lr_plan_build) in a device buffer owned by this object."""

    def __init__(self, cf, vis, psf=False, stream=None, buf=None):
        """buf: a uint8 device tensor to build into (reused when large
        enough, e.g. by a streaming loop), else one is allocated."""
        L = lib()
        v = vis.with_(plan=None)
        d = v.desc()
        n = L.lr_plan_bytes(cf.handle, C.byref(d), int(psf))
        if n == 0:
            raise LRError(LR_E_ARG, L.lr_last_error().decode())
        if buf is not None and buf.numel() >= n:
            self.buf = buf
        else:
            self.buf = torch.empty(n, dtype=torch.uint8, device=vis.uvw.device)
        _on_stream(self.buf, stream)
        self.handle = C.c_void_p()
        self.cf = cf
        self.psf = bool(psf)
        _check(L.lr_plan_build(cf.handle, C.byref(d), int(psf), _ptr(self.buf), n,
                               _stream(stream), C.byref(self.handle)))

    def packed(self, stream=None):
        """A copy of this plan in a buffer of its actual size
        (lr_plan_pack); this plan's buffer may be dropped afterwards."""
        L = lib()
        n = L.lr_plan_packed_bytes(self.handle)
        if n == 0:
            raise LRError(LR_E_ARG, L.lr_last_error().decode())
        q = Plan.__new__(Plan)
        q.buf = torch.empty(n, dtype=torch.uint8, device=self.buf.device)
        _on_stream(q.buf, stream)
        _on_stream(self.buf, stream)
        q.handle = C.c_void_p()
        q.cf, q.psf = self.cf, self.psf
        _check(L.lr_plan_pack(self.handle, _ptr(q.buf), n, _stream(stream), C.byref(q.handle)))
        return q

    def info(self):
        a, b, c, d = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib().lr_plan_info(self.handle, C.byref(a), C.byref(b), C.byref(c), C.byref(d)))
        return {"n_groups": a.value, "n_kept": b.value, "n_pairs": c.value, "taps": d.value}

    def __del__(self):
        try:
            if self.handle:
                lib().lr_plan_free(self.handle)
                self.handle = C.c_void_p()
        except Exception:
            pass


def plan_bytes(cf, vis, psf=False):
    """Device bytes lr_plan_build needs for this vis shape."""
    d = vis.with_(plan=None).desc()
    n = lib().lr_plan_bytes(cf.handle, C.byref(d), int(psf))
    if n == 0:
        raise LRError(LR_E_ARG, lib().lr_last_error().decode())
    return n


def workspace_bytes(op, cf, vis, precision):
    d = vis.desc()
    return lib().lr_workspace_bytes(op, C.byref(cf.spec), C.byref(cf.grid), C.byref(d), precision)


def workspace_bytes_for(op, grid, spec, nrow, nchan, npol, precision):
    """lr_workspace_bytes from the specifications alone (no table built, no
    data on the device); for the visibility operations it includes a
    transient binning plan."""
    fg = np.ascontiguousarray(spec["fg_hz"], np.float64)
    cs = CFSpec(fg_hz=fg.ctypes.data, **{k: v for k, v in spec.items() if k != "fg_hz"})
    d = VisDesc()
    d.nrow, d.nchan, d.npol = int(nrow), int(nchan), int(npol)
    n = lib().lr_workspace_bytes(op, C.byref(cs), C.byref(grid), C.byref(d), precision)
    if n == 0:
        raise LRError(LR_E_ARG, lib().lr_last_error().decode())
    return n


def cf_bytes_for(grid, spec):
    """lr_cf_bytes from the specifications alone."""
    fg = np.ascontiguousarray(spec["fg_hz"], np.float64)
    cs = CFSpec(fg_hz=fg.ctypes.data, **{k: v for k, v in spec.items() if k != "fg_hz"})
    n = lib().lr_cf_bytes(C.byref(cs), C.byref(grid))
    if n == 0:
        raise LRError(LR_E_ARG, lib().lr_last_error().decode())
    return n


def _work(op, cf, vis, precision, work, stream=None):
    n = workspace_bytes(op, cf, vis, precision)
    if n == 0:
        raise LRError(LR_E_ARG, lib().lr_last_error().decode())
    if work is None or work.numel() < n:
        work = torch.empty(n, dtype=torch.uint8, device=vis.uvw.device)
    return _on_stream(work, stream)


def lr_grid(cf, vis, precision, grid, sumwt=None, counters=None, work=None, stream=None):
    work = _work(LR_OP_GRID, cf, vis, precision, work, stream)
    d = vis.desc()
    _check(lib().lr_grid(cf.handle, C.byref(d), precision, _ptr(grid), _ptr(sumwt),
                         _ptr(counters), _ptr(work), work.numel(), _stream(stream)))
    return work


def lr_grid_overwrite(cf, vis, precision, grid, sumwt=None, counters=None, work=None,
                      stream=None):
    work = _work(LR_OP_GRID, cf, vis, precision, work, stream)
    d = vis.desc()
    _check(lib().lr_grid_overwrite(cf.handle, C.byref(d), precision, _ptr(grid), _ptr(sumwt),
                                   _ptr(counters), _ptr(work), work.numel(), _stream(stream)))
    return work


def lr_grid_static(cf, vis, precision, grid, sumwt=None, counters=None, stream=None):
    """lr_grid without workspace (the library's fixed scratch); vis.plan
    must be set."""
    d = vis.desc()
    _check(lib().lr_grid_static(cf.handle, C.byref(d), precision, _ptr(grid), _ptr(sumwt),
                                _ptr(counters), _stream(stream)))


def lr_degrid(cf, vis, precision, grid, counters=None, work=None, stream=None):
    work = _work(LR_OP_DEGRID, cf, vis, precision, work, stream)
    d = vis.desc()
    _check(lib().lr_degrid(cf.handle, C.byref(d), precision, _ptr(grid), _ptr(counters),
                           _ptr(work), work.numel(), _stream(stream)))
    return work


def lr_make_psf(cf, vis, precision, psf_grid, sumwt=None, counters=None, work=None,
                stream=None):
    work = _work(LR_OP_PSF, cf, vis, precision, work, stream)
    d = vis.desc()
    _check(lib().lr_make_psf(cf.handle, C.byref(d), precision, _ptr(psf_grid), _ptr(sumwt),
                             _ptr(counters), _ptr(work), work.numel(), _stream(stream)))
    return work


def lr_sumwt(cf, vis, precision, sumwt, counters=None, work=None, stream=None):
    work = _work(LR_OP_SUMWT, cf, vis, precision, work, stream)
    d = vis.desc()
    _check(lib().lr_sumwt(cf.handle, C.byref(d), precision, _ptr(sumwt), _ptr(counters),
                          _ptr(work), work.numel(), _stream(stream)))
    return work


def lr_debug_map(cf, vis, psf=False, stream=None):
    out = torch.empty((vis.nrow, vis.nchan, 8), dtype=torch.int32, device=vis.uvw.device)
    d = vis.desc()
    _check(lib().lr_debug_map(cf.handle, C.byref(d), int(psf), _ptr(out), _stream(stream)))
    return out


def lr_set_profile_events(start, stop):
    """start / stop: hipEvent_t handles as ints (or None, None)."""
    _check(lib().lr_set_profile_events(start, stop))


def lr_cf_build(grid, spec, device="cuda", stream=None):
    return CF(grid, dict(spec), device=device, stream=stream)


def lr_plan_build(cf, vis, psf=False, stream=None):
    return Plan(cf, vis, psf=psf, stream=stream)


def lr_gcf(cf, n, fg=0, k=0, device="cuda", stream=None):
    """Grid correction of a separable plane: complex128 [n] on the device."""
    out = torch.empty(n, dtype=torch.complex128, device=device)
    _check(lib().lr_gcf(cf.handle, fg, k, n, _ptr(out), _stream(stream)))
    return out


def lr_image_normalize(cf, precision, img, gcf_x, gcf_y, sumwt, out=None, stream=None):
    """Re(img) / (gcf_x gcf_y sumwt) for img [nplane, npol, ny, nx]."""
    if out is None:
        out = torch.empty(img.shape, dtype=torch.float64 if precision == LR_F64
                          else torch.float32, device=img.device)
    _check(lib().lr_image_normalize(cf.handle, precision, _ptr(img), _ptr(gcf_x), _ptr(gcf_y),
                                    _ptr(sumwt), _ptr(out), _stream(stream)))
    return out


def lr_ps_taper(cf, n, device="cuda", stream=None):
    """The PS term's taper at n image pixels: float64 [n] on the device."""
    out = torch.empty(n, dtype=torch.float64, device=device)
    _check(lib().lr_ps_taper(cf.handle, n, _ptr(out), _stream(stream)))
    return out


def lr_pb_image(cf, fg_weight, stream=None):
    """Weight image of A-projection, float64 [nplane, npol, ny, nx], from the
    sums of weights per frequency group fg_weight (float64 device tensor
    [nplane, npol, n_fg])."""
    g = cf.grid
    if fg_weight.dtype != torch.float64 or tuple(fg_weight.shape) != (g.nplane, g.npol,
                                                                        cf.spec.n_fg):
        raise LRError(LR_E_ARG, "fg_weight must be float64 [nplane, npol, n_fg]")
    out = torch.empty((g.nplane, g.npol, g.ny, g.nx), dtype=torch.float64,
                      device=fg_weight.device)
    _check(lib().lr_pb_image(cf.handle, _ptr(fg_weight.contiguous()), _ptr(out),
                             _stream(stream)))
    return out


def lr_image_normalize_pb(cf, precision, img, gcf_x, gcf_y, sumwt, pb, pb_min, out=None,
                          stream=None):
    """Re(img) / (gcf_x gcf_y sumwt pb) where pb >= pb_min, else 0."""
    if out is None:
        out = torch.empty(img.shape, dtype=torch.float64 if precision == LR_F64
                          else torch.float32, device=img.device)
    _check(lib().lr_image_normalize_pb(cf.handle, precision, _ptr(img), _ptr(gcf_x),
                                       _ptr(gcf_y), _ptr(sumwt), _ptr(pb), pb_min, _ptr(out),
                                       _stream(stream)))
    return out


def lr_hogbom(psf, residual, model, gain, threshold, niter, work=None, stream=None):
    """Hogbom minor cycle on one plane (residual updated in place, model
    accumulated); returns the number of subtractions."""
    ny, nx = residual.shape[-2:]
    p = LR_F64 if residual.dtype == torch.float64 else LR_F32
    n = lib().lr_hogbom_work_bytes(nx, ny)
    if work is None or work.numel() < n:
        work = torch.empty(n, dtype=torch.uint8, device=residual.device)
    it = C.c_int32()
    _check(lib().lr_hogbom(_ptr(psf), _ptr(residual), _ptr(model), nx, ny, p, gain, threshold,
                           niter, C.byref(it), _ptr(work), work.numel(), _stream(stream)))
    return it.value


def lr_cal_vavg(vis_obs, vis_model, weight, ant1, ant2, nant, row_sol, n_tsol, chan_sol,
                n_fsol, rows_per_step=1, stream=None):
    """Ratio averages of Eq. VAvg: (X complex128, w float64), each
    [n_tsol, n_fsol, npar, nant, nant], from [nrow, nchan, npol] device
    tensors (complex128 / float64, or complex64 / float32) and int32 device
    antenna ids and interval indices."""
    nrow, nchan, npol = vis_obs.shape
    p = LR_F64 if vis_obs.dtype == torch.complex128 else LR_F32
    cdt, rdt = _vis_dtype(p)
    for t, dt in ((vis_obs, cdt), (vis_model, cdt), (weight, rdt), (ant1, torch.int32),
                  (ant2, torch.int32), (row_sol, torch.int32), (chan_sol, torch.int32)):
        if t is not None and (t.dtype != dt or not t.is_contiguous()):
            raise LRError(LR_E_DTYPE, "expected contiguous %s, got %s" % (dt, t.dtype))
    if vis_model.shape != vis_obs.shape or (weight is not None and weight.shape != vis_obs.shape):
        raise LRError(LR_E_ARG, "vis_obs, vis_model and weight differ in shape")
    npar = 1 if npol == 1 else 2
    dev = vis_obs.device
    X = torch.empty((n_tsol, n_fsol, npar, nant, nant), dtype=torch.complex128, device=dev)
    w = torch.empty((n_tsol, n_fsol, npar, nant, nant), dtype=torch.float64, device=dev)
    _check(lib().lr_cal_vavg(nrow, nchan, npol, p, _ptr(vis_obs), _ptr(vis_model), _ptr(weight),
                             _ptr(ant1), _ptr(ant2), nant, _ptr(row_sol), n_tsol,
                             _ptr(chan_sol), n_fsol, rows_per_step, _ptr(X), _ptr(w),
                             _stream(stream)))
    return X, w


def lr_cal_solve(X, w, g0=None, alpha=0.5, delta=1e-10, max_iter=500, stream=None):
    """Gains of every problem in X, w (lr_cal_vavg's outputs, any leading
    shape): returns (g complex128 [..., nant], iterations int32 [...],
    last max change float64 [...]).  g0: starting gains (default 1)."""
    nant = X.shape[-1]
    lead = X.shape[:-2]
    n = int(np.prod(lead)) if len(lead) else 1
    if g0 is None:
        g = torch.ones(lead + (nant,), dtype=torch.complex128, device=X.device)
    else:
        g = g0.to(torch.complex128).clone().contiguous()
    it = torch.empty(lead, dtype=torch.int32, device=X.device)
    ch = torch.empty(lead, dtype=torch.float64, device=X.device)
    _check(lib().lr_cal_solve(_ptr(X.contiguous()), _ptr(w.contiguous()), nant, n, alpha, delta,
                              max_iter, _ptr(g), _ptr(it), _ptr(ch), _stream(stream)))
    return g, it, ch


def lr_rephase(vis, uvw, freq_hz, field, field_dlm, to_image_centre=True, stream=None):
    """Move mosaic visibilities [nrow, nchan, npol] (device, in place) from
    each row's field phase centre to the joint image centre, or back."""
    nrow, nchan, npol = vis.shape
    p = LR_F64 if vis.dtype == torch.complex128 else LR_F32
    if not vis.is_contiguous() or field.dtype != torch.int32 or field_dlm.dtype != torch.float64:
        raise LRError(LR_E_DTYPE, "contiguous vis, int32 field ids and float64 offsets expected")
    freq = np.ascontiguousarray(freq_hz, np.float64)
    _check(lib().lr_rephase(nrow, nchan, npol, p, _ptr(vis), _ptr(uvw), freq.ctypes.data,
                            _ptr(field.contiguous()), _ptr(field_dlm.contiguous()),
                            int(field_dlm.shape[0]), -1 if to_image_centre else 1,
                            _stream(stream)))
    return vis


def set_deterministic(on=True):
    """Scheduling-independent sums in lr_grid / lr_grid_overwrite / lr_sumwt
    (lr_set_deterministic); returns the previous setting."""
    prev = bool(lib().lr_deterministic())
    _check(lib().lr_set_deterministic(1 if on else 0))
    return prev
