#!/usr/bin/env python3
"""Benchmark of the gridding / degridding hot path on one MI355X.

A step = grid every visibility into a fresh grid (lr_grid_overwrite: clear
of the tiles no chunk owns, presum, gridder), then degrid every visibility
from that grid (degridder + expand), over the W-projection
workload: 351 baselines, 600 dumps, 16 channels, 4 correlations
(13,478,400 visibilities), 32 w-planes with supports 17..65, O = 20, onto a
2048 x 2048 x 4 grid.  Inputs are resident in HBM; the CF table
(PreCompute) and the binning plan (PreSolvePrep) are built once before the
timed region and reported separately.

Prints one JSON line; `value` is visibilities gridded + degridded per second
in the headline precision form.
"""

import argparse
import ctypes as C
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"f64": 78.6e12, "f32": 157.3e12, "f16cf": 157.3e12, "bf16cf": 157.3e12}
HBM_PEAK = 8.0e12


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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_grid_tile_wproj2048_traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2508_17187_amd", "csrc", "k_grid.hip")


def cf_read_bytes(form, r):
    """Kernel bytes a gridding or degridding pass must read: every group's
    sub-kernel once, but no more than the whole table (a small table, such
    as the Standard kernel's, is read once and then served from cache)."""
    return min(r["taps"] * ELEM[form], r["cf_table_bytes"])


def gridder_roofline(wl, form, r, with_traffic=True):
    """Roofline of the gridder kernel (one launch grids all groups).

    Algorithmic flops: 8 per complex multiply-add, npol per kernel tap of
    every group.  Algorithmic bytes: the presummed group values (npol
    complex), every group's S x S sub-kernel once, the grid written once.
    The binding roof is the one with the longer time at peak."""
    import hashlib
    npol = wl.grid.npol
    cplx = 16 if form == "f64" else 8
    flops = 8.0 * npol * r["taps"]
    grid_bytes = wl.grid.nplane * npol * wl.grid.nx * wl.grid.ny * cplx
    bytes_ = r["n_groups"] * npol * cplx + cf_read_bytes(form, r) + grid_bytes
    t = r["grid_kernel_ms"] * 1e-3
    hbm = bytes_ / HBM_PEAK >= flops / PEAK[form]
    traffic = None
    try:
        if not with_traffic:        # the counter summary covers the W-projection run
            raise OSError
        tr = json.load(open(TRAFFIC_FILE))
        sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
        if tr.get("kernel_source_sha256") == sha and tr.get("form") == form:
            traffic = tr["hbm_bytes_per_launch"]
    except (OSError, ValueError, KeyError):
        pass
    # the vector-ALU roof in complex multiply-adds (8 flops each) per second,
    # for the taps the method takes per sample and for those the merged
    # groups execute
    valu = {"peak_cmac_per_s": PEAK[form] / 8.0,
            "per_sample_cmac_per_s": r["sample_taps"] / t,
            "per_sample_frac": r["sample_taps"] / t / (PEAK[form] / 8.0),
            "executed_cmac_per_s": npol * r["taps"] / t,
            "executed_frac": npol * r["taps"] / t / (PEAK[form] / 8.0)}
    if hbm:
        return {"bound": "hbm", "kernel": "k_grid_tile (gridder)", "achieved": bytes_ / t / 1e9,
                "peak": HBM_PEAK / 1e9, "unit": "GB/s", "frac": bytes_ / t / HBM_PEAK,
                "traffic": traffic, "algorithmic_bytes_per_launch": bytes_,
                "algorithmic_flops_per_launch": flops,
                "alu_frac": flops / t / PEAK[form], "valu": valu, "kernel_ms": r["grid_kernel_ms"]}
    return {"bound": "alu", "kernel": "k_grid_tile (gridder)", "achieved": flops / t / 1e12,
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


def large_image_bench(steps, warmup, ev):
    """The large single image: all 1,293,926,400 samples of the 8 h
    observation streamed from pinned host memory in 13 chunks of 1e8
    (copy of chunk i + 1 overlapped with planning and gridding of chunk i),
    FP32, A+W kernels (128 planes, supports to 129, 8 frequency groups),
    onto 8192^2 x 4.  Then one 1e8 chunk of the same layout through the
    Standard kernel, where HBM bandwidth binds."""
    import torch
    import synth
    from paper_2508_17187_amd import lr
    from paper_2508_17187_amd import workload as W
    from paper_2508_17187_amd.stream import ChunkStreamer
    p = lr.LR_F32
    wl = synth.config5()
    out = {"workload": "8 h at 2 s, 351 baselines, 64 channels, 4 pols = 1,293,926,400 "
                       "visibilities in 13 chunks; A+W CF 128 planes x 8 frequency groups, "
                       "supports 17-129, O=20; 8192x8192x4 grid at 0.3 arcsec; FP32"}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cf = W.build_cf(wl, p)
    torch.cuda.synchronize()
    out["cf_build_s"] = time.perf_counter() - t0
    out["cf_gb"] = cf.nbytes / 1e9
    n, nchan, npol = wl.obs.nrow, wl.obs.nchan, wl.grid.npol
    # sample values drawn on the device and staged in pinned host memory
    # (their values do not change the work)
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
    del st, cf, g, vis_p, wt_p, uvw_p
    torch.cuda.empty_cache()
    # one chunk through the Standard kernel
    wps = synth.config5_ps()
    vals, wts = synth.chunk_values(R, nchan, npol, seed=5009)
    wps.obs.uvw = wps.obs.uvw[:R]
    wps.vis, wps.weight = vals, wts
    r, _, _ = run_form(wps, "f32", steps, warmup, ev)
    roof = gridding_roofline(wps, "f32", r)
    out["standard_kernel_chunk"] = {
        "workload": "one 1e8-visibility chunk of the same layout, Standard kernel (PS, S=7, "
                    "O=100), 8192x8192x4 grid, FP32", "result": r, "roofline": roof,
        "roofline_gridder_kernel": gridder_roofline(wps, "f32", r, with_traffic=False)}
    return out


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


def serving_bench(n_jobs=256, rate=20.0, budget_gb=64.0, slots=4, form="f32"):
    """Poisson stream of grid / degrid jobs (configuration 4): visibility
    counts log-uniform in [1e4, 2e7] (4 pols, one 3 GHz channel), grids of
    512^2 .. 4096^2 x 4 at 0.2 arcsec, 1 .. 64 w-planes (w_max fixed from the
    36 km layout at 4 GHz), 5-source skies.  Jobs are submitted at their
    arrival times to a continuous-batching server; returns its stats."""
    import math
    import threading
    import numpy as np
    import torch
    import synth
    from paper_2508_17187_amd import lr
    from paper_2508_17187_amd import serving as S
    from paper_2508_17187_amd import workload as W
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
        wt = np.ones(vis.shape, np.float32)
        N = sp.n_grid
        gs = lr.GridSpec(N, N, 4, 1, cell, cell)
        if sp.n_w == 1:
            cs = dict(terms=1, oversample=100, ps_support=7, n_w=1, w_max=0.0, h_min=3,
                      h_max=3, n_fg=1, fg_hz=np.array([3e9]), dish_m=25.0, screen_m=0,
                      storage=p)
            cfb = S.cf_bytes(1, 3, 3, 100)
        else:
            cs = dict(terms=3, oversample=20, ps_support=7, n_w=sp.n_w, w_max=w_max, h_min=8,
                      h_max=32, n_fg=1, fg_hz=np.array([3e9]), dish_m=25.0, screen_m=0,
                      storage=p)
            cfb = S.cf_bytes(sp.n_w, 8, 32, 20)
        g = None
        if sp.op == "degrid":
            if N not in models:
                models[N] = (rng.standard_normal((1, 4, N, N), np.float32)
                             + 1j * rng.standard_normal((1, 4, N, N), np.float32)
                             ).astype(np.complex64)
            g = models[N]
        payload = dict(grid_spec=gs, cf_spec=cs, uvw=uvw, freq=freq,
                       chan_plane=np.zeros(1, np.int32), vis=vis, weight=wt, grid=g)
        jobs.append(S.Job(sp.job_id, sp.op, (N, sp.n_w), S.job_bytes(nrow, 1, 4, N) +
                          600 * nrow, cfb, payload=payload, n_vis=vis.size,
                          t_arrival=sp.arrival_s))
    arrivals = [j.t_arrival for j in jobs]
    exe = S.GPUExecutor(slots, p)
    srv = S.Server(exe, hbm_budget=int(budget_gb * (1 << 30)), n_slots=slots)
    t0 = time.perf_counter()

    def submit_all():
        for j, ta in zip(jobs, arrivals):
            d = t0 + ta - time.perf_counter()
            if d > 0:
                time.sleep(d)
            srv.submit(j)

    th = threading.Thread(target=submit_all)
    th.start()
    th.join()
    srv.drain(timeout=900)
    st = srv.stats()
    srv.close()
    st["n_jobs"] = n_jobs
    st["arrival_rate_hz"] = rate
    st["slots"] = slots
    st["form"] = form
    st["total_vis"] = int(sum(j.n_vis for j in jobs))
    return st


def cpu_baseline(wl, seconds=15.0):
    """The CPU FP64 oracle, as it stands, on the first rows of the same
    workload: grid + degrid, all host threads."""
    import numpy as np
    import oracle
    from oracle.native import Problem
    ocf = oracle.build_cf(wl.grid, wl.cf)
    cores = os.cpu_count() or 1
    try:
        cores = len(os.sched_getaffinity(0))
    except Exception:
        pass

    def run(rows):
        pr = Problem(wl.obs.uvw[:rows], wl.obs.freq_hz, wl.chan_plane, wl.chan_fg, wl.grid.nx,
                     wl.grid.ny, wl.grid.npol, wl.grid.nplane, wl.grid.cell_l, wl.grid.cell_m,
                     ocf)
        t0 = time.perf_counter()
        g = pr.grid(wl.vis[:rows], wl.weight[:rows], nthreads=cores)
        pr.degrid(g, wl.weight[:rows], nthreads=cores)
        return time.perf_counter() - t0

    rows = 351
    t = run(rows)
    while t < 1.0 and rows < wl.obs.nrow:
        rows = min(wl.obs.nrow, rows * 4)
        t = run(rows)
    rows = int(min(wl.obs.nrow, max(rows, rows * seconds / max(t, 1e-3))))
    t = run(rows)
    n = rows * wl.obs.nchan * wl.grid.npol
    return {"value": n / t, "unit": "visibilities gridded+degridded/s", "cores": cores,
            "kind": "oracle",
            "sample": "first %d of %d rows (all 16 channels, 4 pols): %d visibilities, "
                      "grid + degrid in FP64, %.1f s" % (rows, wl.obs.nrow, n, t)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--form", default="f32", choices=["f64", "f32", "f16cf", "bf16cf"])
    ap.add_argument("--forms", default="f32,f16cf,bf16cf,f64",
                    help="forms measured beside the headline one")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--serving-jobs", type=int, default=256,
                    help="jobs in the serving stream (0 = skip it)")
    ap.add_argument("--no-large", dest="large", action="store_false",
                    help="skip the large single image (1.3e9 visibilities streamed)")
    ap.add_argument("--no-ps", dest="ps", action="store_false",
                    help="skip the Standard-kernel (HBM-bound) workload")
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
    log("generating the W-projection workload")
    t0 = time.perf_counter()
    wl = synth.config2_wproj(dft_device="cuda")
    log("  %d visibilities in %.1f s" % (wl.nsamples, time.perf_counter() - t0))
    ev = HipEvents()
    forms = [args.form] + [f for f in args.forms.split(",") if f and f != args.form]
    res, grids = {}, {}
    for f in forms:
        log("form", f)
        r, g, dv = run_form(wl, f, args.steps, args.warmup, ev)
        res[f] = r
        grids[f] = (g, dv)
        log("  ", json.dumps(r))
    if "f64" in grids:
        g64, v64 = grids["f64"]
        for f in forms:
            g, dv = grids[f]
            res[f]["grid_rel_rms_vs_f64"] = float(
                ((g.to(torch.complex128) - g64).norm() / g64.norm()).item())
            res[f]["degrid_rel_rms_vs_f64"] = float(
                ((dv.to(torch.complex128) - v64).norm() / v64.norm()).item())
        for f in forms:
            res[f]["speedup_vs_f64"] = res[f]["vis_per_s"] / res["f64"]["vis_per_s"]
    del grids
    log("residual image")
    images = image_bench(wl, args.form, args.steps, ev)
    log("  ", json.dumps(images))
    log("CF cache")
    cache = cf_cache_bench(wl, args.form)
    log("  ", json.dumps(cache))
    log("calibration")
    calib = calibration_bench(wl, args.form, args.steps)
    log("  ", json.dumps(calib))
    log("mosaic")
    mosaic = mosaic_bench(wl, args.form, args.steps)
    log("  ", json.dumps(mosaic))
    log("deterministic order")
    determ = deterministic_bench(wl, args.form, args.steps)
    log("  ", json.dumps(determ))
    hbm = None
    if args.ps:
        # the same data through the Standard kernel (PS, S = 7, O = 100, one
        # plane): the shape on which HBM bandwidth binds
        log("standard-kernel (PS) workload")
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
                                                          with_traffic=False)
        del wps
    head = res[args.form]
    roof = gridder_roofline(wl, args.form, head)
    out = {
        "metric": "visibilities gridded+degridded/sec",
        "value": head["vis_per_s"],
        "unit": "visibilities/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f64": "f64", "f32": "f32", "f16cf": "f32 (fp16 CF)",
                  "bf16cf": "f32 (bf16 CF)"}[args.form],
        "data": "synthetic (seeded 200-source sky, direct-sum visibilities, Gaussian noise)",
        "config": {"workload": "W-projection: 351 baselines x 600 dumps x 16 channels x 4 "
                               "pols = 13,478,400 visibilities; 32 w-planes, supports 17-65, "
                               "O=20; 2048x2048x4 grid at 0.2 arcsec",
                   "form": args.form},
        "roofline": roof,
        "forms": res,
    }
    out["image"] = images
    out["cf_cache"] = cache
    out["calibration"] = calib
    out["mosaic"] = mosaic
    out["deterministic"] = determ
    if hbm is not None:
        out["hbm_bound_workload"] = hbm
    if args.large:
        log("large single image")
        del wl
        torch.cuda.empty_cache()
        out["large_image"] = large_image_bench(args.steps, args.warmup, ev)
        log("  ", json.dumps(out["large_image"]))
        wl = None
    if args.serving_jobs > 0:
        log("serving stream of %d jobs" % args.serving_jobs)
        wl = None
        torch.cuda.empty_cache()
        out["serving"] = serving_bench(args.serving_jobs, form=args.form)
        log("  ", json.dumps(out["serving"]))
        wl = None
    if not args.no_cpu_baseline:
        log("cpu baseline")
        if wl is None:
            wl = synth.config2_wproj(dft_device="cuda")
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
