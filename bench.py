#!/usr/bin/env python3
"""Benchmark of the gridding / degridding hot path on one MI355X.

Headline workload: the large single image, every input resident in HBM:
351 baselines x 14,400 dumps x 64 channels x 4 correlations
(1,293,926,400 visibilities) in 13 chunks of 390,625 rows with one packed
binning plan each, A+W kernels (128 w-planes, supports up to 129, O = 20)
onto an 8192 x 8192 x 4 grid.  A step grids every chunk into a fresh grid
(lr_grid_overwrite for the first chunk, lr_grid for the rest) and then
degrids every chunk from that grid.  The CF table (PreCompute) and the
plans (PreSolvePrep) are built once before the timed region and reported
separately.  Further legs (W-projection in four precision forms, the
Standard kernel, imaging, calibration, mosaic, deterministic order, the
stream from host memory, serving) and the CPU oracle's rate follow.

Prints one JSON line; `value` is visibilities gridded + degridded per second
in the FP32 form.
"""

import argparse
import ctypes as C
import gc
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "visibilities gridded+degridded/sec, FP32/FP16-CF vs FP64; p50/p99 job latency"
PEAK = {"f64": 78.6e12, "f32": 157.3e12, "f16cf": 157.3e12, "bf16cf": 157.3e12}
HBM_PEAK = 8.0e12
N_CU, CLOCK_HZ = 256, 2.4e9


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class HipEvents:
    """hipEvent_t pairs through the HIP runtime (timing on the call's stream)."""

    def __init__(self):
        self.hip = C.CDLL("libamdhip64.so")
        self.hip.hipEventCreate.argtypes = [C.POINTER(C.c_void_p)]
        self.hip.hipEventElapsedTime.argtypes = [C.POINTER(C.c_float), C.c_void_p, C.c_void_p]
        self.hip.hipEventSynchronize.argtypes = [C.c_void_p]
        self.hip.hipEventDestroy.argtypes = [C.c_void_p]

    def pair(self):
        a, b = C.c_void_p(), C.c_void_p()
        assert self.hip.hipEventCreate(C.byref(a)) == 0
        assert self.hip.hipEventCreate(C.byref(b)) == 0
        return a.value, b.value

    def ms(self, a, b):
        self.hip.hipEventSynchronize(C.c_void_p(b))
        t = C.c_float()
        assert self.hip.hipEventElapsedTime(C.byref(t), C.c_void_p(a), C.c_void_p(b)) == 0
        return float(t.value)

    def free(self, a, b):
        self.hip.hipEventDestroy(C.c_void_p(a))
        self.hip.hipEventDestroy(C.c_void_p(b))


def run_form(wl, form, steps, warmup, ev):
    import torch
    from paper_2508_17187_amd import lr
    from paper_2508_17187_amd import workload as W
    p = lr.PRECISIONS[form]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cf = W.build_cf(wl, p)
    torch.cuda.synchronize()
    t_cf = time.perf_counter() - t0
    v = W.device_vis(wl, p)
    t0 = time.perf_counter()
    plan = lr.Plan(cf, v)
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    v.plan = plan
    vout = v.with_(vis=torch.empty_like(v.vis))
    g = W.empty_grid(wl, p)
    wg = lr._work(lr.LR_OP_GRID, cf, v, p, None)
    wd = lr._work(lr.LR_OP_DEGRID, cf, vout, p, None)
    info = plan.info()
    sample_taps = per_sample_taps(cf, v)
    kern = gridder_kernel(cf)

    def step(prof=None, marks=None):
        if marks:
            marks[0].record()
        if prof:
            lr.lr_set_profile_events(*prof[0])
        lr.lr_grid_overwrite(cf, v, p, g, work=wg)
        if marks:
            marks[1].record()
        if prof:
            lr.lr_set_profile_events(*prof[1])
        lr.lr_degrid(cf, vout, p, g, work=wd)
        if marks:
            marks[2].record()

    for _ in range(warmup):
        step()
    pairs = [(ev.pair(), ev.pair()) for _ in range(steps)]
    # whole calls, on the stream the library launches on (torch's current one)
    marks = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        step(pairs[i], marks[i])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kg = [ev.ms(*pr[0]) for pr in pairs]
    kd = [ev.ms(*pr[1]) for pr in pairs]
    og = [m[0].elapsed_time(m[1]) for m in marks]
    od = [m[1].elapsed_time(m[2]) for m in marks]
    for pr in pairs:
        ev.free(*pr[0])
        ev.free(*pr[1])
    # the same step captured once in a HIP graph and replayed: removes the
    # host-side launch overhead of the eager loop (no allocation, memset or
    # synchronisation happens inside the captured calls)
    dt_graph = None
    try:
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            step()
        torch.cuda.current_stream().wait_stream(side)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            step()
        for _ in range(warmup):
            graph.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            graph.replay()
        torch.cuda.synchronize()
        dt_graph = time.perf_counter() - t0
    except Exception as e:          # report eager numbers only
        log("  graph capture unavailable:", repr(e))
    n = wl.nsamples
    best = dt if dt_graph is None else min(dt, dt_graph)
    res = {
        "vis_per_s": n * steps / best,
        "ms_per_step": 1e3 * best / steps,
        "ms_per_step_eager": 1e3 * dt / steps,
        "ms_per_step_graph": None if dt_graph is None else 1e3 * dt_graph / steps,
        "grid_kernel_ms": sum(kg) / len(kg),
        "degrid_kernel_ms": sum(kd) / len(kd),
        "grid_call_ms": sum(og) / len(og),
        "degrid_call_ms": sum(od) / len(od),
        "cf_build_ms": 1e3 * t_cf,
        "cf_table_bytes": int(cf.nbytes),
        "plan_build_ms": 1e3 * t_plan,
        "n_groups": info["n_groups"],
        "n_kept_pairs": info["n_kept"],
        "taps": info["taps"],
        "sample_taps": sample_taps,
        "gridder_kernel": kern,
    }
    return res, g, vout.vis


def per_sample_taps(cf, v):
    """Kernel taps of the method as written, without merging: S_k^2 for
    every kept sample (row, channel, pol with nonzero weight), S_k the
    support of the sample's plane (from the index map and the table
    layout: a plane of support S holds (O + 1)^2 S^2 entries)."""
    import numpy as np
    import torch
    from paper_2508_17187_amd import lr
    m = lr.lr_debug_map(cf, v)
    _, _, ne, po = cf.layout()
    ends = np.append(po[1:], ne)
    s2 = torch.as_tensor((ends - po) // (cf.spec.oversample + 1) ** 2, device=m.device)
    plane = m[..., 7].long() * cf.spec.n_w + m[..., 4].long()
    keep = m[..., 6] != 0
    npol = v.npol
    live = (v.weight != 0).sum(-1) if v.weight is not None else torch.full_like(plane, npol)
    taps = torch.where(keep, s2[plane.clamp(0, len(po) - 1)] * live, 0)
    return int(taps.sum().item())


ELEM = {"f64": 16, "f32": 8, "f16cf": 4, "bf16cf": 4}
CSRC = os.path.join(ROOT, "paper_2508_17187_amd", "csrc")
# source file of each timed kernel (with the shared device helpers)
KERNEL_FILES = {"k_grid_tile": "k_grid.hip", "k_presum_col": "k_grid.hip",
                "k_expand": "k_grid.hip", "k_grid_sep": "k_sep.hip",
                "k_degrid": "k_degrid.hip", "k_degrid_small": "k_degrid.hip"}


def kernel_source_sha(kernel):
    """SHA-256 of the kernel's source file, the shared device helpers and
    the binning plan (which decides the kernel's work decomposition and
    launch order)."""
    import hashlib
    h = hashlib.sha256()
    for f in ("k_common.h", "k_plan.hip", KERNEL_FILES[kernel]):
        h.update(open(os.path.join(CSRC, f), "rb").read())
    return h.hexdigest()


def traffic_per_launch(workload, kernel, form):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    counter summary profiles/<workload>_traffic.json (FETCH_SIZE and
    WRITE_SIZE passes scaled by a plain device copy), or None when there is
    none for this form or the kernel's source has changed since."""
    try:
        tr = json.load(open(os.path.join(ROOT, "profiles", workload + "_traffic.json")))
        k = tr["kernels"][kernel]
        if tr.get("form") == form and k.get("source_sha256") == kernel_source_sha(kernel):
            return k["hbm_bytes_per_launch"]
    except (OSError, ValueError, KeyError):
        pass
    return None


def gridder_kernel(cf):
    """The gridder an ordinary gridding call launches with this table:
    k_grid_sep for a real table (no A term, one w-plane) with one frequency
    group and a support of at most 15, k_grid_tile otherwise."""
    sp = cf.spec
    real = not (sp.terms & 4) and (not (sp.terms & 2) or sp.n_w == 1)
    _, _, ne, po = cf.layout()
    s2 = ((po[1] if len(po) > 1 else ne) - po[0]) // (sp.oversample + 1) ** 2
    return "k_grid_sep" if real and sp.n_fg == 1 and s2 <= 15 * 15 else "k_grid_tile"


def cf_read_bytes(form, r):
    """Kernel bytes a gridding or degridding pass must read: every group's
    sub-kernel once, but no more than the whole table (a small table, such
    as the Standard kernel's, is read once and then served from cache)."""
    return min(r["taps"] * ELEM[form], r["cf_table_bytes"])


def gridder_roofline(wl, form, r, traffic_workload=None):
    """Roofline of the gridder kernel (one launch grids all groups).

    Algorithmic flops: 8 per complex multiply-add, npol per kernel tap of
    every group.  Algorithmic bytes: the presummed group values (npol
    complex), every group's S x S sub-kernel once, the grid written once.
    The binding roof is the one with the longer time at peak."""
    npol = wl.grid.npol
    kern = r.get("gridder_kernel", "k_grid_tile")
    cplx = 16 if form == "f64" else 8
    flops = 8.0 * npol * r["taps"]
    grid_bytes = wl.grid.nplane * npol * wl.grid.nx * wl.grid.ny * cplx
    bytes_ = r["n_groups"] * npol * cplx + cf_read_bytes(form, r) + grid_bytes
    t = r["grid_kernel_ms"] * 1e-3
    hbm = bytes_ / HBM_PEAK >= flops / PEAK[form]
    traffic = (None if traffic_workload is None
               else traffic_per_launch(traffic_workload, kern, form))
    # the vector-ALU roof in complex multiply-adds (8 flops each) per second,
    # for the taps the method takes per sample and for those the merged
    # groups execute
    valu = {"peak_cmac_per_s": PEAK[form] / 8.0,
            "per_sample_cmac_per_s": r["sample_taps"] / t,
            "per_sample_frac": r["sample_taps"] / t / (PEAK[form] / 8.0),
            "executed_cmac_per_s": npol * r["taps"] / t,
            "executed_frac": npol * r["taps"] / t / (PEAK[form] / 8.0)}
    if hbm:
        return {"bound": "hbm", "kernel": kern, "achieved": bytes_ / t / 1e9,
                "peak": HBM_PEAK / 1e9, "unit": "GB/s", "frac": bytes_ / t / HBM_PEAK,
                "traffic": traffic, "algorithmic_bytes_per_launch": bytes_,
                "algorithmic_flops_per_launch": flops,
                "alu_frac": flops / t / PEAK[form], "valu": valu, "kernel_ms": r["grid_kernel_ms"]}
    return {"bound": "alu", "kernel": kern, "achieved": flops / t / 1e12,
            "peak": PEAK[form] / 1e12, "unit": "TFLOP/s", "frac": flops / t / PEAK[form],
            "traffic": traffic, "algorithmic_bytes_per_launch": bytes_,
            "algorithmic_flops_per_launch": flops, "hbm_frac": bytes_ / t / HBM_PEAK,
            "valu": valu, "kernel_ms": r["grid_kernel_ms"]}


def gridding_roofline(wl, form, r):
    """HBM roofline of the whole gridding call (clear of shared tiles,
    presum, gridder) on a shape where bandwidth binds: algorithmic bytes are
    the visibilities and weights read once, the per-pair group map, the
    group sums and kernel taps, and the grid written once."""
    npol = wl.grid.npol
    cplx = 16 if form == "f64" else 8
    real = cplx // 2
    n_pairs = wl.obs.nrow * wl.obs.nchan
    grid_bytes = wl.grid.nplane * npol * wl.grid.nx * wl.grid.ny * cplx
    bytes_ = (n_pairs * npol * (cplx + real) + 4 * n_pairs + r["n_groups"] * npol * cplx
              + cf_read_bytes(form, r) + grid_bytes)
    t = r["grid_call_ms"] * 1e-3
    return {"bound": "hbm", "scope": "lr_grid_overwrite call (presum + gridder)",
            "achieved": bytes_ / t / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
            "frac": bytes_ / t / HBM_PEAK, "algorithmic_bytes_per_call": bytes_,
            "call_ms": r["grid_call_ms"]}


def cf_cache_bench(wl, form):
    """The CF cache on the W-projection table: build alone, build and write
    to disk, load back from disk (page cache warm: the file was just
    written) and a resident hit."""
    import shutil
    import tempfile
    import torch
    from paper_2508_17187_amd import cfcache
    from paper_2508_17187_amd import lr
    from paper_2508_17187_amd import workload as W
    p = lr.PRECISIONS[form]
    g, s = W.grid_spec(wl.grid), W.cf_spec(wl.cf, p)

    def timed(f):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = f()
        torch.cuda.synchronize()
        return r, time.perf_counter() - t0

    d = tempfile.mkdtemp(prefix="lrcf_")
    try:
        cf, t_build = timed(lambda: lr.lr_cf_build(g, dict(s)))
        nbytes = cf.nbytes
        del cf
        c1 = cfcache.CFCache(d)
        _, t_build_save = timed(lambda: c1.get(g, s))
        del c1
        c2 = cfcache.CFCache(d)
        _, t_load = timed(lambda: c2.get(g, s))
        _, t_hit = timed(lambda: c2.get(g, s))
        assert c2.stats["loads"] == 1 and c2.stats["hits"] == 1
    finally:
        shutil.rmtree(d, ignore_errors=True)
    return {"table_bytes": int(nbytes), "build_s": t_build, "build_and_save_s": t_build_save,
            "load_s": t_load, "load_gb_per_s": nbytes / t_load / 1e9, "hit_s": t_hit,
            "form": form}


def calibration_bench(wl, form, steps):
    """Diagonal G-Jones solve on the W-projection data: model visibilities of
    the sky's sources predicted by the degridder, observed data = those
    times known per-antenna gains plus noise, 10 time x 4 frequency
    intervals, both parallel hands (80 problems of 27 antennas).  Times the
    ratio averages (one lr_cal_vavg call: clear, sums, finalise) and the
    solve; the bytes rated are the observed, model and weight records read
    once plus the antenna ids and intervals of every row."""
    import numpy as np
    import torch
    from paper_2508_17187_amd import calibration as cal
    from paper_2508_17187_amd import lr
    from paper_2508_17187_amd import workload as W
    from paper_2508_17187_amd.imaging import predict
    p = lr.PRECISIONS[form]
    cf = W.build_cf(wl, p)
    v = W.device_vis(wl, p)
    g = wl.grid
    # model image: the sky's point sources that fall in the inner half of
    # the image, at their nearest pixels, and a few fixed ones
    model = torch.zeros((g.nplane, g.npol, g.ny, g.nx), dtype=torch.float64, device="cuda")
    px = np.rint(wl.sky.l / g.cell_l).astype(int) + g.nx // 2
    py = np.rint(wl.sky.m / g.cell_m).astype(int) + g.ny // 2
    pts = [(x, y, f) for x, y, f in zip(px, py, wl.sky.flux)
           if g.nx // 4 <= x < 3 * g.nx // 4 and g.ny // 4 <= y < 3 * g.ny // 4]
    pts += [(g.nx // 2 + 37 * k, g.ny // 2 - 29 * k, 1.0 / (1 + k)) for k in range(5)]
    for x, y, f in pts:
        for pp in (0, 3):
            model[0, pp, y, x] += f
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    vmod = predict(cf, v, p, model)
    torch.cuda.synchronize()
    t_pred = time.perf_counter() - t0
    nant = int(max(wl.obs.ant1.max(), wl.obs.ant2.max())) + 1
    nrow, nchan = wl.obs.nrow, wl.obs.nchan
    nbl = nant * (nant - 1) // 2
    n_tsol, n_fsol = 10, 4
    a1 = torch.as_tensor(wl.obs.ant1.astype(np.int32), device="cuda")
    a2 = torch.as_tensor(wl.obs.ant2.astype(np.int32), device="cuda")
    ndump = nrow // nbl
    row_sol = torch.as_tensor((np.arange(nrow) // nbl * n_tsol // ndump).astype(np.int32),
                              device="cuda")
    chan_sol = torch.as_tensor((np.arange(nchan) * n_fsol // nchan).astype(np.int32),
                               device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(7007)
    amp = 1.0 + 0.1 * torch.randn((n_tsol, n_fsol, 2, nant), generator=gen, device="cuda",
                                  dtype=torch.float64)
    ph = 3.0 * (torch.rand((n_tsol, n_fsol, 2, nant), generator=gen, device="cuda",
                           dtype=torch.float64) - 0.5)
    gt = torch.polar(amp, ph)
    rs, cs = row_sol.long(), chan_sol.long()
    vobs = vmod.clone()
    for q, pp in enumerate((0, 3)):
        gq = gt[:, :, q]                                   # [n_tsol, n_fsol, nant]
        gi = gq[rs][:, cs, :].gather(2, a1.long()[:, None, None].expand(nrow, nchan, 1))[..., 0]
        gj = gq[rs][:, cs, :].gather(2, a2.long()[:, None, None].expand(nrow, nchan, 1))[..., 0]
        noise = 0.01 * torch.complex(torch.randn((nrow, nchan), generator=gen, device="cuda"),
                                     torch.randn((nrow, nchan), generator=gen, device="cuda"))
        vobs[:, :, pp] = (gi * torch.conj(gj)).to(vmod.dtype) * vmod[:, :, pp] + noise.to(vmod.dtype)
    vobs = vobs.contiguous()
    run = lambda: lr.lr_cal_vavg(vobs, vmod, v.weight, a1, a2, nant, row_sol, n_tsol, chan_sol,
                                 n_fsol, rows_per_step=nbl)
    for _ in range(2):
        X, w = run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        X, w = run()
    torch.cuda.synchronize()
    t_vavg = (time.perf_counter() - t0) / steps
    t0 = time.perf_counter()
    gs, it, ch = lr.lr_cal_solve(X, w, alpha=0.5, delta=1e-10, max_iter=1000)
    torch.cuda.synchronize()
    t_solve = time.perf_counter() - t0
    # gain products against the truth (the data cannot see a common phase)
    P = gs[..., :, None] * torch.conj(gs[..., None, :])
    T = gt[..., :, None] * torch.conj(gt[..., None, :])
    off = ~torch.eye(nant, dtype=torch.bool, device="cuda")
    err = float((P - T).abs()[..., off].max())
    cplx = 16 if p == lr.LR_F64 else 8
    byts = nrow * nchan * 4 * (2 * cplx + cplx // 2) + nrow * 12 + nchan * 4
    return {"form": form, "n_problems": int(it.numel()), "nant": nant, "predict_ms": 1e3 * t_pred,
            "vavg_ms": 1e3 * t_vavg, "vavg_gb_per_s": byts / t_vavg / 1e9,
            "vavg_hbm_frac": byts / t_vavg / HBM_PEAK,
            "solve_ms": 1e3 * t_solve, "iterations_max": int(it.max()),
            "iterations_mean": float(it.float().mean()), "gain_product_max_error": err,
            "noise_per_sample": 0.01}


def mosaic_bench(wl, form, steps):
    """The W-projection data split into three fields (thirds of the
    observation in time) whose phase centres lie 60 arcsec from the image
    centre: the change of phase centre (lr_rephase, in place on a copy) and
    the mosaic gridding call (pointing phasor on virtual antennas), against
    the single-pointing gridding call of the same data."""
    import numpy as np
    import torch
    from paper_2508_17187_amd import lr
    from paper_2508_17187_amd import workload as W
    from paper_2508_17187_amd.mosaic import Mosaic
    p = lr.PRECISIONS[form]
    cf = W.build_cf(wl, p)
    v = W.device_vis(wl, p, pointing=False)
    nrow = wl.obs.nrow
    nant = int(max(wl.obs.ant1.max(), wl.obs.ant2.max())) + 1
    a = 60.0 * np.pi / (180.0 * 3600.0)
    offs = torch.tensor([[a, 0.0], [-a, 0.5 * a], [0.0, -a]], dtype=torch.float64, device="cuda")
    field = torch.as_tensor((np.arange(nrow) * 3 // nrow).astype(np.int32), device="cuda")
    mos = Mosaic(field, offs, torch.as_tensor(wl.obs.ant1.astype(np.int32), device="cuda"),
                 torch.as_tensor(wl.obs.ant2.astype(np.int32), device="cuda"), nant)
    moved = v.vis.clone()

    def timed(f, n):
        f()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            f()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / n

    t_re = timed(lambda: lr.lr_rephase(moved, v.uvw, v.freq, mos.field, mos.field_dlm), steps)
    vm = mos.vis(v, moved)
    t0 = time.perf_counter()
    vm.plan = lr.Plan(cf, vm)
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    g = W.empty_grid(wl, p)
    wg = lr._work(lr.LR_OP_GRID, cf, vm, p, None)
    t_grid = timed(lambda: lr.lr_grid_overwrite(cf, vm, p, g, work=wg), steps)
    info = vm.plan.info()
    cplx = 16 if p == lr.LR_F64 else 8
    byts = 2 * nrow * wl.obs.nchan * wl.grid.npol * cplx + nrow * 28
    return {"form": form, "fields": 3, "field_offset_arcsec": 60.0,
            "rephase_ms": 1e3 * t_re, "rephase_gb_per_s": byts / t_re / 1e9,
            "mosaic_grid_call_ms": 1e3 * t_grid, "mosaic_plan_build_ms": 1e3 * t_plan,
            "mosaic_groups": info["n_groups"], "kept_pairs": info["n_kept"]}


def deterministic_bench(wl, form, steps):
    """The gridding call (lr_grid_overwrite with sums of weights) on the
    W-projection data in the default and in the deterministic order
    (lr_set_deterministic), and whether two deterministic calls agree bit
    for bit."""
    import torch
    from paper_2508_17187_amd import lr
    from paper_2508_17187_amd import workload as W
    p = lr.PRECISIONS[form]
    cf = W.build_cf(wl, p)
    v = W.device_vis(wl, p)
    v.plan = lr.Plan(cf, v)
    g = W.empty_grid(wl, p)
    sw = torch.zeros((wl.grid.nplane, wl.grid.npol), dtype=torch.float64, device="cuda")
    wg = lr._work(lr.LR_OP_GRID, cf, v, p, None)

    def call():
        lr.lr_grid_overwrite(cf, v, p, g, sumwt=sw, work=wg)

    def timed(n):
        call()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            call()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / n

    t_default = timed(steps)
    prev = lr.set_deterministic(True)
    try:
        t_det = timed(steps)
        call()
        g1, s1 = g.clone(), sw.clone()
        call()
        torch.cuda.synchronize()
        same = bool(torch.equal(g1.view(torch.uint8), g.view(torch.uint8))
                    and torch.equal(s1.view(torch.uint8), sw.view(torch.uint8)))
    finally:
        lr.set_deterministic(prev)
    return {"form": form, "grid_call_ms": 1e3 * t_default,
            "deterministic_grid_call_ms": 1e3 * t_det, "slowdown": t_det / t_default,
            "repeat_bit_identical": same}


C5_WORKLOAD = ("large single image: 351 baselines (36 km) x 14,400 dumps (8 h at 2 s) x 64 "
               "channels (2-4 GHz) x 4 pols = 1,293,926,400 visibilities in 13 chunks of "
               "1e8; A+W kernels, 128 w-planes x 8 frequency groups, supports 17-129, O=20; "
               "8192x8192x4 grid at 0.3 arcsec")


def large_image_resident(form, steps, warmup, ev, rows=None):
    """The large single image with every input resident in HBM: all
    1,293,926,400 samples (sample values drawn on the device: they do not
    change the work), 13 chunks of 390,625 rows with one packed plan each.
    A step grids every chunk into one grid (lr_grid_overwrite for the
    first chunk, lr_grid for the rest) and then degrids every chunk from
    it.  The CF build (PreCompute) and the plans (PreSolvePrep) are built
    once before the timed steps and reported separately."""
    import numpy as np
    import torch
    import synth
    from paper_2508_17187_amd import lr
    from paper_2508_17187_amd import workload as W
    p = lr.PRECISIONS[form]
    wl = synth.config5()
    nrow = wl.obs.nrow if rows is None else rows
    nchan, npol = wl.obs.nchan, wl.grid.npol
    cdt, rdt = (torch.complex128, torch.float64) if p == lr.LR_F64 else (torch.complex64,
                                                                         torch.float32)
    torch.cuda.synchronize()
    torch.cuda.reset_peak_memory_stats()
    t0 = time.perf_counter()
    cf = W.build_cf(wl, p)
    torch.cuda.synchronize()
    t_cf = time.perf_counter() - t0
    R = synth.C5_CHUNK_ROWS
    chunks = [(r, min(r + R, nrow)) for r in range(0, nrow, R)]
    # one uvw array per chunk: a chunk of an odd number of rows would leave
    # the next chunk's uvw rows off the 16-byte alignment the library needs
    uvw = {r0: torch.as_tensor(np.ascontiguousarray(wl.obs.uvw[r0:r1]), device="cuda")
           for r0, r1 in chunks}
    vis = torch.empty((nrow, nchan, npol), dtype=cdt, device="cuda")
    wt = torch.empty((nrow, nchan, npol), dtype=rdt, device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5008)
    for r0, r1 in chunks:
        # FP32 draws (exact in FP64 too): every form grids the same values
        sh = (r1 - r0, nchan, npol)
        vis[r0:r1] = torch.complex(torch.randn(sh, generator=gen, device="cuda"),
                                   torch.randn(sh, generator=gen, device="cuda"))
        wt[r0:r1] = torch.rand(sh, generator=gen, device="cuda") + 0.5
    vout = torch.empty_like(vis)
    freq = wl.obs.freq_hz

    def vdesc(r0, r1, data, plan=None):
        return lr.Vis(uvw[r0], freq, wl.chan_plane, wl.chan_fg, vis=data[r0:r1],
                      weight=wt[r0:r1], npol=npol, plan=plan)

    # plans: built chunk by chunk in one worst-case build buffer, then packed
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plans, buf = [], None
    for r0, r1 in chunks:
        pl = lr.Plan(cf, vdesc(r0, r1, vis), buf=buf)
        buf = pl.buf
        plans.append(pl.packed())
        del pl
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    build_bytes = int(buf.numel())
    del buf
    torch.cuda.empty_cache()
    vs = [vdesc(r0, r1, vis, pl) for (r0, r1), pl in zip(chunks, plans)]
    vo = [vdesc(r0, r1, vout, pl) for (r0, r1), pl in zip(chunks, plans)]
    infos = [pl.info() for pl in plans]
    sample_taps = sum(per_sample_taps(cf, v.with_(plan=None)) for v in vs)
    g = W.empty_grid(wl, p)
    sw = torch.zeros((wl.grid.nplane, npol), dtype=torch.float64, device="cuda")
    # one workspace per operation, sized for the chunk that needs most
    wg = torch.empty(max(lr.workspace_bytes(lr.LR_OP_GRID, cf, v, p) for v in vs),
                     dtype=torch.uint8, device="cuda")
    wd = torch.empty(max(lr.workspace_bytes(lr.LR_OP_DEGRID, cf, v, p) for v in vo),
                     dtype=torch.uint8, device="cuda")

    def step(prof=None):
        for i, v in enumerate(vs):
            if prof:
                lr.lr_set_profile_events(*prof[0][i])
            if i == 0:
                lr.lr_grid_overwrite(cf, v, p, g, sumwt=sw, work=wg)
            else:
                lr.lr_grid(cf, v, p, g, sumwt=sw, work=wg)
        for i, v in enumerate(vo):
            if prof:
                lr.lr_set_profile_events(*prof[1][i])
            lr.lr_degrid(cf, v, p, g, work=wd)

    for _ in range(warmup):
        step()
    n = len(vs)
    prof = [([ev.pair() for _ in range(n)], [ev.pair() for _ in range(n)])
            for _ in range(steps)]
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    a.record()
    for i in range(steps):
        step(prof[i])
    b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    t_step = a.elapsed_time(b) / steps * 1e-3
    kg = [[ev.ms(*pr) for pr in st[0]] for st in prof]
    kd = [[ev.ms(*pr) for pr in st[1]] for st in prof]
    for st in prof:
        for pr in st[0] + st[1]:
            ev.free(*pr)
    nvis = nrow * nchan * npol
    grid_k = float(np.median([sum(x) for x in kg])) * 1e-3
    degrid_k = float(np.median([sum(x) for x in kd])) * 1e-3
    res = {
        "form": form, "samples": nvis, "chunks": n, "steps": steps, "warmup": warmup,
        "vis_per_s": nvis / t_step, "ms_per_step": 1e3 * t_step,
        "wall_ms_per_step": 1e3 * wall / steps,
        "grid_vis_per_s_kernels": nvis / grid_k, "degrid_vis_per_s_kernels": nvis / degrid_k,
        "gridder_ms_per_step": 1e3 * grid_k, "degridder_ms_per_step": 1e3 * degrid_k,
        "gridder_ms_per_chunk": [float(np.median([x[i] for x in kg])) for i in range(n)],
        "degridder_ms_per_chunk": [float(np.median([x[i] for x in kd])) for i in range(n)],
        "cf_build_s": t_cf, "cf_table_bytes": int(cf.nbytes),
        "plan_build_s": t_plan, "plan_build_buffer_bytes": build_bytes,
        "plan_packed_bytes": int(sum(pl.buf.numel() for pl in plans)),
        "n_groups": int(sum(i["n_groups"] for i in infos)),
        "n_kept_pairs": int(sum(i["n_kept"] for i in infos)),
        "n_pairs": int(sum(i["n_pairs"] for i in infos)),
        "taps": int(sum(i["taps"] for i in infos)),
        "sample_taps": int(sample_taps),
        "peak_hbm_bytes": int(torch.cuda.max_memory_allocated()),
    }
    # the grid of all chunks and the degridded values of the first chunk,
    # for the error of one form against another
    return res, g, vout[:chunks[0][1]].clone()


def large_image_roofline(res):
    """Vector-ALU roofline of the kernel that takes the larger share of a
    large-image step (the gridder or the degridder).  Algorithmic flops per
    launch: 8 per complex multiply-add for every kernel tap of every kept
    sample (S_k^2 per (row, channel, pol), no merging), summed over the
    chunk; the rate is the step's total over the kernel's total time (13
    launches, one per chunk).  The peak is the published FP32 (FP64) vector
    rate.  `traffic` is the measured HBM bytes per launch (mean over the 13
    chunks) from the committed counter summary, when it matches the source."""
    form = res["form"]
    k = "gridder" if res["gridder_ms_per_step"] >= res["degridder_ms_per_step"] else "degridder"
    kern = "k_grid_tile" if k == "gridder" else "k_degrid"
    t = res[k + "_ms_per_step"] * 1e-3
    n = res["chunks"]
    flops = 8.0 * res["sample_taps"]
    peak = PEAK[form]
    traffic = traffic_per_launch("large_image", kern, form)
    out = {"bound": "alu", "kernel": kern, "achieved": flops / t / 1e12, "peak": peak / 1e12,
           "unit": "TFLOP/s", "frac": flops / t / peak, "traffic": traffic,
           "algorithmic_flops_per_launch": flops / n, "launches_per_step": n,
           "kernel_ms_per_launch": 1e3 * t / n,
           # packed FP32 instructions are not used, so the FP32 vector rate
           # reachable here is the non-packed one, equal to the FP64 peak
           "frac_of_non_packed_rate": flops / t / PEAK["f64"],
           "executed_frac": 8.0 * 4 * res["taps"] / t / peak,
           # every group reads its S x S sub-kernel: bytes the kernel must
           # fetch when no table plane stays in cache between groups
           "kernel_tap_bytes_per_launch": res["taps"] * ELEM[form] / n}
    # bytes the kernel's vector loads return per launch: every tap's kernel
    # value, and for the degridder the four pols' grid values of the tap
    # (the gridder keeps its grid in registers), per clock and CU
    gbytes = 16 if form == "f64" else 8
    vm = res["taps"] * (ELEM[form] + (4 * gbytes if k == "degridder" else 0)) / n
    out["vmem_bytes_per_launch"] = vm
    out["vmem_bytes_per_clk_per_cu"] = vm / (t / n) / (N_CU * CLOCK_HZ)
    if traffic is not None:
        out["traffic_rate_gbps"] = traffic / (t / n) / 1e9
        out["traffic_frac_of_hbm_peak"] = traffic / (t / n) / HBM_PEAK
    return out


def large_image_streamed(steps, warmup, ev):
    """The large single image streamed from pinned host memory: every chunk
    copied host to device (the copy of chunk i + 1 overlapped with chunk i),
    planned and gridded, FP32: the PCIe-inclusive end-to-end rate."""
    import torch
    import synth
    from paper_2508_17187_amd import lr
    from paper_2508_17187_amd import workload as W
    from paper_2508_17187_amd.stream import ChunkStreamer
    p = lr.LR_F32
    wl = synth.config5()
    out = {"workload": C5_WORKLOAD + "; FP32; streamed from pinned host memory"}
    cf = W.build_cf(wl, p)
    n, nchan, npol = wl.obs.nrow, wl.obs.nchan, wl.grid.npol
    uvw_p = torch.from_numpy(wl.obs.uvw).pin_memory()
    vis_p = torch.empty((n, nchan, npol), dtype=torch.complex64).pin_memory()
    wt_p = torch.empty((n, nchan, npol), dtype=torch.float32).pin_memory()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5008)
    R = synth.C5_CHUNK_ROWS
    for r0 in range(0, n, R):
        r1 = min(n, r0 + R)
        sh = (r1 - r0, nchan, npol)
        vis_p[r0:r1].copy_(torch.complex(torch.randn(sh, generator=gen, device="cuda"),
                                         torch.randn(sh, generator=gen, device="cuda")))
        wt_p[r0:r1].copy_(torch.rand(sh, generator=gen, device="cuda") + 0.5)
    st = ChunkStreamer(cf, p, uvw_p, wl.obs.freq_hz, wl.chan_plane, wl.chan_fg, weight=wt_p,
                       chunk_rows=R)
    g = W.empty_grid(wl, p)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st.grid(vis_p, g)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    out.update({"samples": n * nchan * npol, "chunks": len(st.chunks()),
                "grid_s": t, "grid_vis_per_s": n * nchan * npol / t,
                "includes": "H2D of every chunk, a plan build per chunk, presum, gridder"})
    return out


def standard_kernel_chunk(steps, warmup, ev):
    """One 1e8-visibility chunk of the large-image layout through the
    Standard kernel (PS, S=7, O=100): the shape on which HBM bandwidth
    binds."""
    import synth
    wps = synth.config5_ps()
    R = synth.C5_CHUNK_ROWS
    vals, wts = synth.chunk_values(R, wps.obs.nchan, wps.grid.npol, seed=5009)
    wps.obs.uvw = wps.obs.uvw[:R]
    wps.obs.ant1, wps.obs.ant2 = wps.obs.ant1[:R], wps.obs.ant2[:R]
    wps.vis, wps.weight = vals, wts
    r, _, _ = run_form(wps, "f32", steps, warmup, ev)
    return {"workload": "one 1e8-visibility chunk of the large-image layout, Standard kernel "
                        "(PS, S=7, O=100), 8192x8192x4 grid, FP32", "result": r,
            "roofline": gridding_roofline(wps, "f32", r),
            "roofline_gridder_kernel": gridder_roofline(wps, "f32", r,
                                                        traffic_workload="standard_chunk")}


def image_bench(wl, form, steps, ev):
    """Residual image of the W-projection data against a 20-component model
    (Eq. ResIm): predict (F, degrid), subtract, grid, F^dagger (rocFFT) and
    normalise by the grid correction of the w = 0 plane and the sums of
    weights."""
    import torch
    from paper_2508_17187_amd import lr
    from paper_2508_17187_amd import workload as W
    from paper_2508_17187_amd.autograd import DegridOp
    from paper_2508_17187_amd.imaging import dirty_image, grid_correction, residual_image
    p = lr.PRECISIONS[form]
    cf = W.build_cf(wl, p)
    v = W.device_vis(wl, p)
    v.plan = lr.Plan(cf, v)
    g = wl.grid
    rdt = torch.float64 if p == lr.LR_F64 else torch.float32
    model = torch.zeros((g.nplane, g.npol, g.ny, g.nx), dtype=rdt, device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(2100)
    iy = torch.randint(g.ny // 4, 3 * g.ny // 4, (20,), generator=gen, device="cuda")
    ix = torch.randint(g.nx // 4, 3 * g.nx // 4, (20,), generator=gen, device="cuda")
    model[:, :, iy, ix] = 0.5
    gcf = grid_correction(cf)
    op = DegridOp(cf, v, p)
    out = {}
    for name, fn in (("dirty_image_ms", lambda: dirty_image(cf, v, p, gcf=gcf)),
                     ("residual_image_ms",
                      lambda: residual_image(cf, v, p, model, gcf=gcf, op=op))):
        fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        for _ in range(steps):
            fn()
        b.record()
        torch.cuda.synchronize()
        out[name] = a.elapsed_time(b) / steps
    img, _ = dirty_image(cf, v, p, gcf=gcf)
    out["dirty_peak_jy"] = float(img[0, 0].max().item())
    # PSF image and a minor cycle on the Stokes-I-like first plane
    cdt = torch.complex128 if p == lr.LR_F64 else torch.complex64
    psfg = torch.zeros((g.nplane, g.npol, g.ny, g.nx), dtype=cdt, device="cuda")
    sw = torch.zeros((g.nplane, g.npol), dtype=torch.float64, device="cuda")
    vp = v.with_(plan=None)
    lr.lr_make_psf(cf, vp.with_(plan=lr.Plan(cf, vp, psf=True)), p, psfg, sumwt=sw)
    from paper_2508_17187_amd.autograd import centred_ifft2
    psf = lr.lr_image_normalize(cf, p, centred_ifft2(psfg).contiguous(), gcf[0], gcf[1], sw)
    res = img[0, 0].contiguous()
    model = torch.zeros_like(res)
    niter = 1000
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it = lr.lr_hogbom(psf[0, 0].contiguous(), res, model, 0.1, 0.0, niter)
    out["hogbom_iterations"] = it
    out["hogbom_ms_per_iteration"] = 1e3 * (time.perf_counter() - t0) / max(it, 1)
    out["form"] = form
    return out


def autograd_bench(steps, warmup):
    """The differentiable degrid on the A+W data with pointing offsets (351
    baselines x 600 dumps x 64 channels x 4 pols = 53,913,600 visibilities,
    Airy A terms in 8 frequency groups, 32 w-planes, 4096^2 x 4 model of
    1000 point components): one iteration is chi^2 (F, degrid, residual;
    Eq. ImChisq) and its gradient through the hand-written gridding adjoint
    (grid, F^dagger; Eq. ResIm), in FP32 and FP64, timed with the degrid
    and adjoint calls on their own; the FP32 gradient against the FP64 one."""
    import torch
    import synth
    from paper_2508_17187_amd import lr
    from paper_2508_17187_amd import workload as W
    from paper_2508_17187_amd.autograd import DegridOp, centred_fft2, chi2
    wl = synth.config3_awproj(dft_device="cuda")
    g = wl.grid
    gen = torch.Generator(device="cuda")
    gen.manual_seed(3100)
    base = torch.zeros((g.nplane, g.npol, g.ny, g.nx), dtype=torch.float64, device="cuda")
    iy = torch.randint(g.ny // 8, g.ny - g.ny // 8, (1000,), generator=gen, device="cuda")
    ix = torch.randint(g.nx // 8, g.nx - g.nx // 8, (1000,), generator=gen, device="cuda")
    base[0, 0, iy, ix] = 1e-3 * torch.rand(1000, generator=gen, device="cuda",
                                           dtype=torch.float64)
    base[0, 3] = base[0, 0]
    n = int(wl.nsamples)
    out = {"workload": "A+W projection with pointing offsets: 351 baselines x 600 dumps x "
                       "64 channels x 4 pols = 53,913,600 visibilities; Airy A terms in 8 "
                       "frequency groups, 32 w-planes, supports 17-65, O=20; 4096x4096x4 "
                       "model", "samples": n, "forms": {}}
    grads = {}

    def timed(fn, k):
        for _ in range(warmup):
            fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        for _ in range(k):
            r = fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / k, r

    for f in ("f32", "f64"):
        p = lr.PRECISIONS[f]
        cf = W.build_cf(wl, p)
        v = W.device_vis(wl, p)
        op = DegridOp(cf, v, p)
        img = base.to(op.rdt).requires_grad_(True)

        def step():
            (gr,) = torch.autograd.grad(chi2(img, op, v.vis, v.weight), img)
            return gr

        ms, gr = timed(step, steps)
        grads[f] = gr.detach().double()
        grid = centred_fft2(base.to(op.cdt))
        ms_d, vm = timed(lambda: op.degrid(grid), steps)
        ms_g, _ = timed(lambda: op.grid_adjoint(vm), steps)
        out["forms"][f] = {"ms_per_iteration": ms, "vis_per_s": n / (ms * 1e-3),
                           "degrid_call_ms": ms_d, "grid_adjoint_call_ms": ms_g,
                           "kernel_calls_vis_per_s": n / ((ms_d + ms_g) * 1e-3)}
        del cf, v, op, img, grid, vm
        torch.cuda.empty_cache()
    out["speedup_f32_vs_f64"] = out["forms"]["f32"]["vis_per_s"] / out["forms"]["f64"]["vis_per_s"]
    out["gradient_rel_rms_f32_vs_f64"] = float(
        (torch.linalg.vector_norm(grads["f32"] - grads["f64"])
         / torch.linalg.vector_norm(grads["f64"])).item())
    return out


def serving_jobs(n_jobs, rate, form):
    """The serving stream (configuration 4): visibility counts log-uniform
    in [1e4, 2e7] (4 pols, one 3 GHz channel), grids of 512^2 .. 4096^2 x 4
    at 0.2 arcsec, 1 .. 64 w-planes (w_max fixed from the 36 km layout at
    4 GHz), 5-source skies, grid or degrid with probability 1/2; one model
    grid per grid size, shared by that size's degrid jobs.  Inputs are
    staged in pinned host memory; footprints are the executor's exact
    allocations."""
    import math
    import numpy as np
    import torch
    import synth
    from paper_2508_17187_amd import lr
    from paper_2508_17187_amd import serving as S
    p = lr.PRECISIONS[form]
    specs = synth.config4_jobs(n_jobs, rate)
    enu = synth.antenna_layout(27, 36000.0, seed=1004)
    full, _, _, nbl = synth.uvw_tracks(enu, 480, 60.0, 30.0)
    w_max = float(np.max(np.abs(full[:, 2])) * 4.0e9 / synth.C_LIGHT)
    cell = 0.2 * synth.ARCSEC
    rng = np.random.default_rng(4005)
    models = {}
    jobs = []
    for sp in specs:
        nrow = max(1, math.ceil(sp.n_samples / 4))
        n_time = math.ceil(nrow / nbl)
        uvw, _, _, _ = synth.uvw_tracks(enu, n_time, 2.0, 30.0)
        uvw = np.ascontiguousarray(uvw[:nrow])
        freq = np.array([3.0e9])
        sky = synth.random_point_sky(5, seed=sp.seed, half_width_deg=0.05)
        vis = synth.dft_visibilities(uvw, freq, sky, 4, device="cuda").astype(np.complex64)
        N = sp.n_grid
        gs = lr.GridSpec(N, N, 4, 1, cell, cell)
        if sp.n_w == 1:
            cs = dict(terms=1, oversample=100, ps_support=7, n_w=1, w_max=0.0, h_min=3,
                      h_max=3, n_fg=1, fg_hz=np.array([3e9]), dish_m=25.0, screen_m=0,
                      storage=p)
        else:
            cs = dict(terms=3, oversample=20, ps_support=7, n_w=sp.n_w, w_max=w_max, h_min=8,
                      h_max=32, n_fg=1, fg_hz=np.array([3e9]), dish_m=25.0, screen_m=0,
                      storage=p)
        g, mkey = None, None
        if sp.op == "degrid":
            mkey = N
            if N not in models:
                models[N] = torch.complex(torch.randn((1, 4, N, N)), torch.randn((1, 4, N, N))
                                          ).pin_memory()
            g = models[N]
        payload = dict(grid_spec=gs, cf_spec=cs, uvw=torch.from_numpy(uvw).pin_memory(),
                       freq=freq, chan_plane=np.zeros(1, np.int32),
                       vis=torch.from_numpy(vis).pin_memory(),
                       weight=torch.ones(vis.shape, dtype=torch.float32).pin_memory(), grid=g)
        cfb, cfw = S.cf_footprint(gs, cs)
        jobs.append(S.Job(sp.job_id, sp.op, (N, sp.n_w),
                          S.job_footprint(sp.op, gs, cs, nrow, 1, 4, p,
                                          resident_model=mkey is not None),
                          cfb, payload=payload, n_vis=vis.size, t_arrival=sp.arrival_s,
                          model_key=mkey,
                          model_bytes=S.model_footprint(gs, p) if mkey is not None else 0,
                          cf_build_bytes=cfw))
    return jobs


def serving_bench(n_jobs=256, rate=20.0, budget_gb=16.0, slots=4, form="f32", jobs=None):
    """The serving stream submitted at its arrival times to a
    continuous-batching server with an HBM budget that binds (16 GB: jobs
    wait for memory as well as for slots); returns its stats.  rate=None
    submits every job at once (arrivals far above capacity: throughput is
    then the server's capacity)."""
    import threading
    import torch
    from paper_2508_17187_amd import lr
    from paper_2508_17187_amd import serving as S
    p = lr.PRECISIONS[form]
    if jobs is None:
        jobs = serving_jobs(n_jobs, rate or 20.0, form)
    arrivals = [0.0 if rate is None else j.t_arrival for j in jobs]
    exe = S.GPUExecutor(slots, p)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    base = torch.cuda.memory_allocated()
    torch.cuda.reset_peak_memory_stats()
    srv = S.Server(exe, hbm_budget=int(budget_gb * (1 << 30)), n_slots=slots)
    t0 = time.perf_counter()

    def consume(fut):
        # the client takes each result as its job completes and lets it go
        # (results held to the end would pin host memory for the whole run)
        if fut.exception() is None:
            fut.result().result = None

    def submit_all():
        for j, ta in zip(jobs, arrivals):
            d = t0 + ta - time.perf_counter()
            if d > 0:
                time.sleep(d)
            srv.submit(j).add_done_callback(consume)

    th = threading.Thread(target=submit_all)
    th.start()
    th.join()
    srv.drain(timeout=900)
    st = srv.stats()
    srv.close()
    torch.cuda.synchronize()
    st["allocator_peak_bytes"] = int(torch.cuda.max_memory_allocated() - base)
    st["n_jobs"] = len(jobs)
    st["arrival_rate_hz"] = rate if rate is not None else "all at once"
    st["slots"] = slots
    st["form"] = form
    st["total_vis"] = int(sum(j.n_vis for j in jobs))
    del exe
    torch.cuda.empty_cache()
    return st


def cpu_baseline_large(sample_taps_per_vis, seconds=15.0, n_planes=12):
    """The CPU FP64 oracle, as it stands, on a bounded sample of the large
    image: the channels of the first frequency group, one at a time, each
    with the rows whose samples fall on one of
    the n_planes kernel planes most used among those whose support is near
    the workload's root-mean-square support, all 4 pols (the oracle's table
    holds only those planes).  Grid + degrid on all host threads, channels
    added until about `seconds` of work; the rate in kernel taps per second
    is turned into visibilities per second with the large image's mean taps
    per visibility (its cost is linear in N_vis x C_sup)."""
    import numpy as np
    import oracle
    import synth
    from oracle.native import Problem
    wl = synth.config5()
    cores = os.cpu_count() or 1
    try:
        cores = len(os.sched_getaffinity(0))
    except Exception:
        pass
    g = wl.grid
    nchan, npol = wl.obs.nchan, g.npol
    chans = [c for c in range(nchan) if wl.chan_fg[c] == 0]
    dummy = oracle.build_cf(g, wl.cf, planes=set(), compact=True)
    h = dummy.h
    S = 2 * h.astype(np.int64) + 1

    def problem(uvw, c, ocf):
        # one channel of the observation (its frequency and A-term group)
        return Problem(uvw, wl.obs.freq_hz[c:c + 1], np.zeros(1, np.int32),
                       np.asarray(wl.chan_fg[c:c + 1], np.int32), g.nx, g.ny, npol, g.nplane,
                       g.cell_l, g.cell_m, ocf)

    def chan_map(c, nrows):
        m = problem(wl.obs.uvw[:nrows], c, dummy).map()[:, 0]
        return m[:, 6] == 1, m[:, 4].copy()

    nprobe = wl.obs.nrow
    c_mid = chans[len(chans) // 2]
    keep, kk = chan_map(c_mid, nprobe)
    s_rms = np.sqrt(sample_taps_per_vis)
    near = (S >= 0.8 * s_rms) & (S <= 1.25 * s_rms)
    counts = np.bincount(kk[keep], minlength=len(h))
    counts[~near] = 0
    top = np.argsort(-counts)[:n_planes]
    top = top[counts[top] > 0]
    planes = {(0, int(k)) for k in top}
    t0 = time.perf_counter()
    ocf = oracle.build_cf(g, wl.cf, planes=planes, compact=True)
    t_cf = time.perf_counter() - t0
    rng = np.random.default_rng(5010)
    t, taps, nv, used = 0.0, 0, 0, []
    for c in [c_mid] + [c for c in chans if c != c_mid]:
        if t >= seconds:
            break
        if c != c_mid:
            keep, kk = chan_map(c, nprobe)
        sel = np.nonzero(keep & np.isin(kk, top))[0]
        if len(sel) == 0:
            continue
        if t > 0:
            # rows of this channel that fill the remaining time at the rate so far
            sel = sel[:max(1, int((seconds - t) * nv / npol / t))]
        pr = problem(np.ascontiguousarray(wl.obs.uvw[sel]), c, ocf)
        shape = (len(sel), 1, npol)
        wt = np.ones(shape)
        vis = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
        t0 = time.perf_counter()
        gr = pr.grid(vis, wt, nthreads=cores)
        pr.degrid(gr, wt, nthreads=cores)
        t += time.perf_counter() - t0
        del gr
        taps += int(np.sum(S[kk[sel]] ** 2)) * npol
        nv += len(sel) * npol
        used.append(c)
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": taps / t / sample_taps_per_vis, "unit": "visibilities gridded+degridded/s",
            "cores": cores, "kind": "oracle", "cpu_model": model,
            "host_cpus": os.cpu_count(),
            "sample": "large image, channels %s one at a time: the rows (of %d) whose "
                      "samples lie on the %d kernel planes most used near the workload's rms "
                      "support (w-planes %s, supports %s-%s), 4 pols = %d visibilities; grid + "
                      "degrid in FP64 in %.1f s = %.3g taps/s, divided by the workload's %.1f "
                      "taps per visibility (oracle table build %.1f s, not timed)"
                      % (used, nprobe, len(planes), sorted(int(k) for k in top),
                         int(S[top].min()), int(S[top].max()), nv, t, taps / t,
                         sample_taps_per_vis, t_cf)}


def rel_rms(a, b):
    import torch
    d = (a.to(torch.complex128) - b).flatten()
    return float((d.abs().pow(2).sum() / b.flatten().abs().pow(2).sum()).sqrt().item())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--large-forms", default="f16cf,f64",
                    help="forms of the large image measured beside FP32 (min(steps, 3) "
                         "steps each)")
    ap.add_argument("--forms", default="f32,f16cf,bf16cf,f64",
                    help="forms of the W-projection workload")
    ap.add_argument("--large-rows", type=int, default=0,
                    help="rows of the large image (0 = all 5,054,400)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--serving-jobs", type=int, default=256,
                    help="jobs in the serving stream (0 = skip it)")
    ap.add_argument("--legs", default="all",
                    help="comma list of legs after the headline (wproj, image, cf_cache, "
                         "calibration, mosaic, deterministic, autograd, standard, "
                         "standard_chunk, streamed, serving), 'all' or ''")
    ap.add_argument("--no-legs", dest="legs", action="store_const", const="",
                    help="only the large image (headline) and the CPU baseline")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the headline (profiling runs of single legs)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="run one 1 GiB device copy first (scale of the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: there is no multi-GPU path (each GPU would "
              "grid its share of the rows into a private grid, followed by one sum of grids)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    torch.cuda.set_device(0)
    if args.copy_calib:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    ev = HipEvents()
    rows = args.large_rows or None
    legs = set(x for x in args.legs.split(",") if x)

    def want(name):
        return "all" in legs or name in legs

    out = {}
    if not args.no_large:
        out = headline(args, ev, rows)
    run_legs(args, ev, want, out)
    if not args.no_cpu_baseline and "large_image_forms" in out:
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline_large(
            out["large_image_forms"]["f32"]["sample_taps"]
            / out["large_image_forms"]["f32"]["samples"], args.cpu_seconds)
    print(json.dumps(out), flush=True)


def headline(args, ev, rows):
    """The large single image, inputs resident in HBM: FP32 (the value)
    and the other forms asked for."""
    import torch
    log("large image, FP32, %d steps after %d warm-up" % (args.steps, args.warmup))
    head, g32, v32 = large_image_resident("f32", args.steps, args.warmup, ev, rows=rows)
    log("  ", json.dumps(head))
    large = {"f32": head}
    g32h = g32
    for f in [f for f in args.large_forms.split(",") if f and f != "f32"]:
        torch.cuda.empty_cache()
        log("large image,", f)
        r, gf, vf = large_image_resident(f, min(args.steps, 3), 1, ev, rows=rows)
        large[f] = r
        if f == "f64":
            large["f32"]["grid_rel_rms_vs_f64"] = rel_rms(g32h, gf)
            large["f32"]["degrid_rel_rms_vs_f64_first_chunk"] = rel_rms(v32, vf)
            if "_f16" in large:
                gh, vh = large.pop("_f16")
                large["f16cf"]["grid_rel_rms_vs_f64"] = rel_rms(gh, gf)
                large["f16cf"]["degrid_rel_rms_vs_f64_first_chunk"] = rel_rms(vh, vf)
        elif f in ("f16cf", "bf16cf"):
            large["_f16"] = (gf, vf)
        del gf, vf
        log("  ", json.dumps(r))
    large.pop("_f16", None)
    if "f64" in large:
        for f in list(large):
            large[f]["speedup_vs_f64"] = large[f]["vis_per_s"] / large["f64"]["vis_per_s"]
    del g32, g32h, v32
    torch.cuda.empty_cache()
    roof = large_image_roofline(head)
    out = {
        "metric": METRIC,
        "value": head["vis_per_s"],
        "unit": "visibilities/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded antenna layout and tracks; sample values drawn on the "
                "device, which do not change the work)",
        "config": {"workload": C5_WORKLOAD + ("" if rows is None else "; first %d rows" % rows),
                   "form": "f32"},
        "roofline": roof,
        "large_image_forms": large,
    }
    return out


def run_legs(args, ev, want, out):
    import torch
    import synth
    if any(want(x) for x in ("wproj", "image", "cf_cache", "calibration", "mosaic",
                             "deterministic")):
        log("generating the W-projection workload")
        wl = synth.config2_wproj(dft_device="cuda")
        if want("wproj"):
            res, grids = {}, {}
            forms = [f for f in args.forms.split(",") if f]
            for f in forms:
                log("W-projection form", f)
                r, g, dv = run_form(wl, f, args.steps, args.warmup, ev)
                res[f] = r
                grids[f] = (g, dv)
                log("  ", json.dumps(r))
            if "f64" in grids:
                g64, v64 = grids["f64"]
                for f in forms:
                    g, dv = grids[f]
                    res[f]["grid_rel_rms_vs_f64"] = rel_rms(g, g64)
                    res[f]["degrid_rel_rms_vs_f64"] = rel_rms(dv, v64)
                for f in forms:
                    res[f]["speedup_vs_f64"] = res[f]["vis_per_s"] / res["f64"]["vis_per_s"]
            del grids
            wproj = {"workload": "W-projection: 351 baselines x 600 dumps x 16 channels x 4 "
                                 "pols = 13,478,400 visibilities; 32 w-planes, supports 17-65, "
                                 "O=20; 2048x2048x4 grid at 0.2 arcsec", "forms": res}
            if "f32" in res:
                wproj["roofline"] = gridder_roofline(wl, "f32", res["f32"],
                                                     traffic_workload="wproj2048")
            out["wproj"] = wproj
        if want("image"):
            log("residual image")
            out["image"] = image_bench(wl, "f32", args.steps, ev)
        if want("cf_cache"):
            log("CF cache")
            out["cf_cache"] = cf_cache_bench(wl, "f32")
        if want("calibration"):
            log("calibration")
            out["calibration"] = calibration_bench(wl, "f32", args.steps)
        if want("mosaic"):
            log("mosaic")
            out["mosaic"] = mosaic_bench(wl, "f32", args.steps)
        if want("deterministic"):
            log("deterministic order")
            out["deterministic"] = deterministic_bench(wl, "f32", args.steps)
        del wl
        torch.cuda.empty_cache()
    if want("autograd"):
        log("differentiable degrid on the A+W data")
        out["autograd"] = autograd_bench(args.steps, args.warmup)
        log("  ", json.dumps(out["autograd"]))
        torch.cuda.empty_cache()
    if want("standard"):
        log("standard-kernel (PS) workloads")
        wps = synth.config2_ps(dft_device="cuda")
        hbm = {"workload": "W-projection data with the Standard kernel: PS only, S=7, "
                           "O=100, 2048x2048x4 grid", "forms": {}}
        for f in ("f32", "f64"):
            r, _, _ = run_form(wps, f, args.steps, args.warmup, ev)
            hbm["forms"][f] = r
            log("  ", f, json.dumps(r))
        hbm["speedup_f32_vs_f64"] = (hbm["forms"]["f32"]["vis_per_s"]
                                     / hbm["forms"]["f64"]["vis_per_s"])
        hbm["roofline"] = gridding_roofline(wps, "f32", hbm["forms"]["f32"])
        hbm["roofline_gridder_kernel"] = gridder_roofline(wps, "f32", hbm["forms"]["f32"],
                                                          traffic_workload="standard2048")
        out["hbm_bound_workload"] = hbm
        del wps
        torch.cuda.empty_cache()
    if want("standard_chunk"):
        log("standard-kernel chunk of the large image")
        out["standard_kernel_chunk"] = standard_kernel_chunk(args.steps, args.warmup, ev)
        log("  ", json.dumps(out["standard_kernel_chunk"]))
        torch.cuda.empty_cache()
    if want("streamed"):
        log("large image streamed from host memory")
        out["large_image_streamed"] = large_image_streamed(args.steps, args.warmup, ev)
        log("  ", json.dumps(out["large_image_streamed"]))
        torch.cuda.empty_cache()
        # hand the leg's 16 GB of pinned host buffers back to the system
        gc.collect()
        if hasattr(torch._C, "_host_emptyCache"):
            torch._C._host_emptyCache()
    if want("serving") and args.serving_jobs > 0:
        log("serving stream of %d jobs" % args.serving_jobs)
        jobs = serving_jobs(args.serving_jobs, 20.0, "f32")
        serving = {"stream_20_per_s": serving_bench(rate=20.0, jobs=jobs)}
        log("  ", json.dumps(serving["stream_20_per_s"]))
        for j in jobs:
            j.t_admit = j.t_done = j.error = j.result = None
            j.cf_cold = j.model_cold = False
            j.charged = 0
        serving["all_at_once"] = serving_bench(rate=None, jobs=jobs)
        log("  ", json.dumps(serving["all_at_once"]))
        out["serving"] = serving


if __name__ == "__main__":
    main()
