"""The gridding step captured in a HIP graph: every replay, with eager work
and synchronisations in between, equals the eager result (no allocation,
memset or synchronisation is recorded by a call that has a plan)."""

import numpy as np
import pytest

import synth
from oracle.cfbuild import TERM_PS, TERM_W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2508_17187_amd import lr  # noqa: E402
from paper_2508_17187_amd import workload as W  # noqa: E402


def test_graph_replays_match_eager():
    wl = synth.tiny_workload(n_w=4, h_min=3, h_max=6, oversample=8, terms=TERM_PS | TERM_W,
                             nchan=3, n_time=20, nx=96, ny=96, cell_arcsec=6.0,
                             diameter_m=5000.0, cfg_id=301)
    p = lr.LR_F32
    cf = W.build_cf(wl, p)
    v = W.device_vis(wl, p)
    v.plan = lr.Plan(cf, v)
    vout = v.with_(vis=torch.empty_like(v.vis))
    g = W.empty_grid(wl, p)
    wg = lr._work(lr.LR_OP_GRID, cf, v, p, None)
    wd = lr._work(lr.LR_OP_DEGRID, cf, vout, p, None)

    def step():
        g.zero_()
        lr.lr_grid(cf, v, p, g, work=wg)
        lr.lr_degrid(cf, vout, p, g, work=wd)

    step()
    torch.cuda.synchronize()
    ref_g, ref_v = g.clone(), vout.vis.clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    for r in range(4):
        # eager work between replays: scribble over the outputs
        g.fill_(3.0)
        vout.vis.fill_(-1.0)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        eg = ((g - ref_g).abs().max() / ref_g.abs().max()).item()
        ev = ((vout.vis - ref_v).abs().max() / ref_v.abs().max()).item()
        assert eg < 1e-5 and ev < 1e-5, (r, eg, ev)
