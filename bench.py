#!/usr/bin/env python3
"""Benchmark of the gridding / degridding hot path on one MI355X.

A step = zero the grid, grid every visibility (presum + gridder), degrid
every visibility from that grid (degridder + expand), over the W-projection
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

    def step(prof=None):
        g.zero_()
        if prof:
            lr.lr_set_profile_events(*prof[0])
        lr.lr_grid(cf, v, p, g, work=wg)
        if prof:
            lr.lr_set_profile_events(*prof[1])
        lr.lr_degrid(cf, vout, p, g, work=wd)

    for _ in range(warmup):
        step()
    pairs = [(ev.pair(), ev.pair()) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        step(pairs[i])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kg = [ev.ms(*pr[0]) for pr in pairs]
    kd = [ev.ms(*pr[1]) for pr in pairs]
    for pr in pairs:
        ev.free(*pr[0])
        ev.free(*pr[1])
    n = wl.nsamples
    res = {
        "vis_per_s": n * steps / dt,
        "ms_per_step": 1e3 * dt / steps,
        "grid_kernel_ms": sum(kg) / len(kg),
        "degrid_kernel_ms": sum(kd) / len(kd),
        "cf_build_ms": 1e3 * t_cf,
        "plan_build_ms": 1e3 * t_plan,
        "n_groups": info["n_groups"],
        "n_kept_pairs": info["n_kept"],
        "taps": info["taps"],
    }
    return res, g, vout.vis


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
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (each GPU would "
              "grid its share of the rows into a private grid, followed by one sum of grids)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    torch.cuda.set_device(0)
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
    head = res[args.form]
    npol = wl.grid.npol
    flops = 8.0 * npol * head["taps"]
    t_k = head["grid_kernel_ms"] * 1e-3
    roof = {"bound": "alu", "kernel": "k_grid (gridder)", "achieved": flops / t_k / 1e12,
            "peak": PEAK[args.form] / 1e12, "unit": "TFLOP/s",
            "frac": (flops / t_k) / PEAK[args.form], "traffic": None,
            "algorithmic_flops_per_launch": flops,
            "unit_of_work": "8 flops x 4 pols per kernel tap of each sample group"}
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
    if not args.no_cpu_baseline:
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
