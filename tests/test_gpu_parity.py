"""GPU parity: the HIP path through the C ABI against the CPU FP64 oracle on
the same seeded inputs.

Bars: index map, counters and PSF symmetry bit-exact; grid / degrid values
within rel-RMS 1e-12 (FP64), 1e-5 (FP32), 3e-3 (FP16 CF); BF16 CF is
reported against 2e-2 (its 8-bit mantissa gives ~1e-3..1e-2); sumwt within
1e-12 relative.
"""

import numpy as np
import pytest

import synth
import oracle
from oracle.cfbuild import TERM_A, TERM_PS, TERM_W, quantised_table, plane_scale_exponents
from oracle.native import Problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2508_17187_amd import lr  # noqa: E402
from paper_2508_17187_amd import workload as W  # noqa: E402

DEV = "cuda"
PREC = {"f64": lr.LR_F64, "f32": lr.LR_F32, "f16cf": lr.LR_F32_CF16, "bf16cf": lr.LR_F32_CFBF16}
TOL = {"f64": 1e-12, "f32": 1e-5, "f16cf": 3e-3, "bf16cf": 2e-2}


def rel(a, b):
    a = np.asarray(a, np.complex128).ravel()
    b = np.asarray(b, np.complex128).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def say(*a):
    print(*a, flush=True)


def awp_workload(nx=128, ny=96, pointing=0.0, seed_id=91, h_max=7):
    wl = synth.tiny_workload(n_w=6, h_min=3, h_max=h_max, oversample=8,
                             terms=TERM_PS | TERM_W | TERM_A, nchan=4, n_time=16, nx=nx,
                             ny=ny, cell_arcsec=6.0, diameter_m=6000.0, nplane=2,
                             chan_plane=[0, 1, -1, 0], chan_fg=[0, 0, 1, 1],
                             fg_hz=[2.4e9, 3.6e9], cfg_id=seed_id, pointing_sigma=pointing)
    rng = np.random.default_rng(seed_id)
    wl.weight[rng.random(wl.weight.shape) < 0.05] = 0.0
    return wl


# widest support 15 (within one 32-cell tile plus a band) and 19
KERNELS = [7, 9]
KERNEL_IDS = ["S15", "S19"]


@pytest.fixture(scope="module", params=KERNELS, ids=KERNEL_IDS)
def awp(request):
    wl = awp_workload(h_max=request.param)
    return wl, oracle.build_cf(wl.grid, wl.cf)


@pytest.fixture(scope="module", params=KERNELS, ids=KERNEL_IDS)
def awp_po(request):
    wl = awp_workload(pointing=3e-5, seed_id=92, h_max=request.param)
    return wl, oracle.build_cf(wl.grid, wl.cf)


# --- index map -------------------------------------------------------------------

@pytest.mark.parametrize("psf", [False, True])
def test_map_bitexact_small(awp, psf):
    wl, ocf = awp
    say("map", wl.obs.nrow, wl.obs.nchan, "psf", psf)
    cf = W.build_cf(wl, lr.LR_F64)
    v = W.device_vis(wl, lr.LR_F64, with_vis=False)
    got = lr.lr_debug_map(cf, v, psf=psf).cpu().numpy()
    pr = Problem.from_workload(wl, ocf, psf=psf)
    ref = pr.map()
    keep = ref[..., 6] == 1
    assert np.array_equal(got[..., 6], ref[..., 6])
    assert np.array_equal(got[keep], ref[keep])
    assert 0 < keep.sum() < keep.size


def test_map_bitexact_ties_and_edges():
    # samples placed on 1/O boundaries, next to them, at the grid edge and
    # beyond, with w on plane boundaries and of both signs
    rng = np.random.default_rng(11)
    nx, O, n_w = 64, 20, 8
    cell = 4.0 * synth.ARCSEC
    freq = np.array([2.2e9, 3.3e9, 3.9e9])
    du_m = synth.C_LIGHT / freq[0] / (nx * cell)
    u = np.concatenate([np.arange(-700, 700) / O * du_m, rng.uniform(-40, 40, 3000) * du_m])
    u = np.concatenate([u, np.nextafter(u, np.inf), np.nextafter(u, -np.inf)])
    v = rng.permutation(u)
    w_max = 5e4
    wl_m = w_max * synth.C_LIGHT / freq[-1]
    w = np.concatenate([np.linspace(-1.1 * wl_m, 1.1 * wl_m, len(u) - 4), [0.0, -0.0, wl_m, -wl_m]])
    uvw = np.stack([u, v, w], 1)
    wl = synth.tiny_workload(nx=nx, ny=nx, cell_arcsec=4.0, oversample=O, n_w=n_w, h_min=2,
                             h_max=5, terms=TERM_PS | TERM_W, nchan=3, n_time=2)
    wl.obs.uvw = uvw
    wl.obs.freq_hz = freq
    wl.cf.w_max = w_max
    wl.vis = np.zeros((len(u), 3, 4), np.complex128)
    wl.weight = np.ones((len(u), 3, 4))
    ocf = oracle.build_cf(wl.grid, wl.cf, planes=set())
    cf = W.build_cf(wl, lr.LR_F32)
    vv = W.device_vis(wl, lr.LR_F32, with_vis=False)
    got = lr.lr_debug_map(cf, vv).cpu().numpy()
    ref = Problem.from_workload(wl, ocf).map()
    keep = ref[..., 6] == 1
    assert np.array_equal(got[..., 6], ref[..., 6])
    assert np.array_equal(got[keep], ref[keep])
    assert keep.sum() > 1000 and (~keep).sum() > 100


@pytest.mark.parametrize("form", ["f64", "f32", "f16cf", "bf16cf"])
def test_grid_and_degrid_with_footprints_at_the_grid_edges(form):
    """Samples dense near the edges of a 64 x 64 grid, so that kept
    footprints touch the first and last rows and columns (the FP32
    degridder's two-cell loads there start at column 0 or end at column
    nx - 1): G and D against the oracle."""
    rng = np.random.default_rng(12)
    nx, O = 64, 20
    cell = 4.0 * synth.ARCSEC
    freq = np.array([2.2e9, 3.3e9, 3.9e9])
    du_m = synth.C_LIGHT / freq[-1] / (nx * cell)
    u = rng.uniform(-34, 34, 4000) * du_m
    v = rng.uniform(-34, 34, 4000) * du_m
    w_max = 5e4
    w = rng.uniform(-1, 1, 4000) * w_max * synth.C_LIGHT / freq[-1]
    wl = synth.tiny_workload(nx=nx, ny=nx, cell_arcsec=4.0, oversample=O, n_w=8, h_min=2,
                             h_max=5, terms=TERM_PS | TERM_W, nchan=3, n_time=2)
    wl.obs.uvw = np.stack([u, v, w], 1)
    wl.obs.freq_hz = freq
    wl.cf.w_max = w_max
    wl.vis = rng.standard_normal((4000, 3, 4)) + 1j * rng.standard_normal((4000, 3, 4))
    wl.weight = rng.uniform(0.5, 1.5, (4000, 3, 4))
    ocf = oracle.build_cf(wl.grid, wl.cf)
    pr = Problem.from_workload(wl, ocf)
    m = pr.map()
    keep = m[..., 6] == 1
    h = oracle.half_widths(wl.cf.n_w, wl.cf.h_min, wl.cf.h_max)[m[..., 4]]
    for lo, hi in ((m[..., 0] - h, m[..., 0] + h), (m[..., 1] - h, m[..., 1] + h)):
        assert (keep & (lo == 0)).sum() > 10 and (keep & (hi == nx - 1)).sum() > 10
    assert (~keep).sum() > 100
    p = PREC[form]
    cf = W.build_cf(wl, p)
    vd = W.device_vis(wl, p)
    g = W.empty_grid(wl, p)
    lr.lr_grid(cf, vd, p, g)
    e = rel(g.cpu().numpy(), pr.grid(wl.vis, wl.weight))
    x = rng.standard_normal((1, 4, nx, nx)) + 1j * rng.standard_normal((1, 4, nx, nx))
    lr.lr_degrid(cf, vd, p, torch.as_tensor(x, device=DEV).to(g.dtype))
    ref = pr.degrid(x, wl.weight)
    got = vd.vis.cpu().numpy()
    e2 = rel(got, ref)
    say("edges", form, e, e2)
    assert e <= TOL[form] and e2 <= TOL[form]
    assert np.all(got[ref == 0] == 0)


def test_map_bitexact_config1():
    wl = synth.config1_plain()
    ocf = oracle.build_cf(wl.grid, wl.cf)
    cf = W.build_cf(wl, lr.LR_F64)
    got = lr.lr_debug_map(cf, W.device_vis(wl, lr.LR_F64, with_vis=False)).cpu().numpy()
    ref = Problem.from_workload(wl, ocf).map()
    assert np.array_equal(got, ref)
    assert ref[..., 6].all()


# --- CF tables ----------------------------------------------------------------------

def check_cf_table(wl, ocf, form):
    cf = W.build_cf(wl, PREC[form])
    got = cf.table_host()
    ref = ocf.table
    scale = np.abs(ref).max()
    if form == "f64":
        # the two PSWF constructions (Nystrom vs Legendre series) agree to
        # ~1e-13, and that sets the floor here
        assert np.max(np.abs(got - ref)) < 5e-13 * scale
        return
    q = quantised_table(ocf, {"f32": "f32", "f16cf": "f16", "bf16cf": "bf16"}[form])
    if form != "f32":
        assert np.array_equal(cf.scale_exponents(), plane_scale_exponents(ocf))
    diff = np.abs(got - q)
    # identical except where the two FP64 tables (which differ by <5e-13 of
    # the peak) straddle a rounding boundary of the storage format: a
    # component that differs must have the oracle's FP64 value within that
    # bound of the midpoint of the two stored neighbours (the boundary)
    for gc, qc, rc in ((got.real, q.real, ref.real), (got.imag, q.imag, ref.imag)):
        d = gc != qc
        assert np.all(np.abs(rc[d] - 0.5 * (gc[d] + qc[d])) <= 5e-13 * scale)
    ulp = {"f32": 2.0 ** -23, "f16cf": 2.0 ** -10, "bf16cf": 2.0 ** -7}[form]
    sub = 2.0 ** -24 * scale if form == "f16cf" else 0.0     # fp16 subnormal step
    assert np.all(diff <= ulp * np.abs(ref) * 1.01 + 2 * sub + 1e-12 * scale)


@pytest.mark.parametrize("form", ["f64", "f32", "f16cf", "bf16cf"])
def test_cf_table_matches_oracle(awp, form):
    wl, ocf = awp
    say("cf", form)
    check_cf_table(wl, ocf, form)


# --- gridding, degridding, PSF --------------------------------------------------------

def run_grid(wl, form, plan=False, pointing=None):
    p = PREC[form]
    cf = W.build_cf(wl, p)
    v = W.device_vis(wl, p, pointing=pointing)
    if plan:
        v.plan = lr.Plan(cf, v)
    g = W.empty_grid(wl, p)
    sw = torch.zeros((wl.grid.nplane, wl.grid.npol), dtype=torch.float64, device=DEV)
    cnt = torch.zeros(3, dtype=torch.int64, device=DEV)
    lr.lr_grid(cf, v, p, g, sumwt=sw, counters=cnt)
    torch.cuda.synchronize()
    return g.cpu().numpy(), sw.cpu().numpy(), cnt.cpu().numpy()


def check_grid(wl, ocf, form):
    g, sw, cnt = run_grid(wl, form)
    pr = Problem.from_workload(wl, ocf)
    ref = pr.grid(wl.vis, wl.weight)
    s_ref, c_ref = pr.sumwt(wl.weight)
    e = rel(g, ref)
    say("grid rel-rms", form, e)
    assert e <= TOL[form]
    assert np.array_equal(cnt, c_ref)
    assert np.max(np.abs(sw - s_ref) / np.abs(s_ref).max()) < 1e-12
    assert c_ref[0] > 0 and c_ref[1] > 0 and c_ref[2] > 0


@pytest.mark.parametrize("form", ["f64", "f32"])
@pytest.mark.parametrize("plan", [False, True], ids=["transient", "plan"])
def test_sumwt_default_mode_matches_oracle(awp, form, plan):
    """lr_sumwt in the default (scheduling-dependent) order: FP64 sums of the
    kept weights per (plane, pol) and the class counts, added to what the
    outputs held (the oracle sums the weights the GPU was given: FP32
    weights rounded first)."""
    wl, ocf = awp
    p = PREC[form]
    cf = W.build_cf(wl, p)
    v = W.device_vis(wl, p)
    if plan:
        v.plan = lr.Plan(cf, v)
    sw = torch.full((wl.grid.nplane, wl.grid.npol), 0.25, dtype=torch.float64, device=DEV)
    cnt = torch.tensor([5, 6, 7], dtype=torch.int64, device=DEV)
    lr.lr_sumwt(cf, v, p, sw, counters=cnt)
    torch.cuda.synchronize()
    w = wl.weight if form == "f64" else wl.weight.astype(np.float32).astype(np.float64)
    s_ref, c_ref = Problem.from_workload(wl, ocf).sumwt(w)
    assert np.array_equal(cnt.cpu().numpy(), c_ref + np.array([5, 6, 7]))
    got = sw.cpu().numpy() - 0.25
    assert np.max(np.abs(got - s_ref)) <= 1e-12 * np.abs(s_ref).max()
    assert c_ref[0] > 0 and c_ref[1] > 0 and c_ref[2] > 0


@pytest.mark.parametrize("form", ["f64", "f32", "f16cf", "bf16cf"])
def test_grid_parity(awp, form):
    wl, ocf = awp
    say("grid", form)
    check_grid(wl, ocf, form)


def test_rows_in_any_order(awp):
    """Time-major rows let presum / expand walk tracks in natural order; a
    shuffled row order has no period and takes the sorted-gather path.  Both
    agree with the oracle."""
    wl, ocf = awp
    perm = np.random.default_rng(12).permutation(wl.obs.nrow)
    import copy
    ws = copy.deepcopy(wl)
    ws.obs.uvw = wl.obs.uvw[perm]
    ws.vis = wl.vis[perm]
    ws.weight = wl.weight[perm]
    for form in ("f64", "f32"):
        p = PREC[form]
        cf = W.build_cf(ws, p)
        v = W.device_vis(ws, p)
        plan = lr.Plan(cf, v)
        v.plan = plan
        g = W.empty_grid(ws, p)
        cnt = torch.zeros(3, dtype=torch.int64, device=DEV)
        lr.lr_grid(cf, v, p, g, counters=cnt)
        pr = Problem.from_workload(ws, ocf)
        assert rel(g.cpu().numpy(), pr.grid(ws.vis, ws.weight)) <= TOL[form]
        assert np.array_equal(cnt.cpu().numpy(), pr.sumwt(ws.weight)[1])
        lr.lr_degrid(cf, v, p, g)
        ref = pr.degrid(g.cpu().numpy().astype(np.complex128), ws.weight)
        assert rel(v.vis.cpu().numpy(), ref) <= TOL[form]


def test_grid_with_plan_equals_transient_plan(awp):
    wl, _ = awp
    a, sa, ca = run_grid(wl, "f64")
    b, sb, cb = run_grid(wl, "f64", plan=True)
    assert rel(b, a) < 1e-14
    assert np.array_equal(ca, cb) and np.allclose(sa, sb, rtol=1e-15, atol=0)


def check_degrid(wl, ocf, form):
    p = PREC[form]
    rng = np.random.default_rng(5)
    shape = (wl.grid.nplane, wl.grid.npol, wl.grid.ny, wl.grid.nx)
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    cf = W.build_cf(wl, p)
    v = W.device_vis(wl, p)
    v.vis = torch.full_like(v.vis, 7.0)       # overwritten everywhere
    cdt = torch.complex128 if p == lr.LR_F64 else torch.complex64
    xg = torch.as_tensor(x, device=DEV).to(cdt)
    cnt = torch.zeros(3, dtype=torch.int64, device=DEV)
    lr.lr_degrid(cf, v, p, xg, counters=cnt)
    got = v.vis.cpu().numpy()
    pr = Problem.from_workload(wl, ocf)
    ref = pr.degrid(x, wl.weight)
    e = rel(got, ref)
    say("degrid rel-rms", form, e)
    assert e <= TOL[form]
    assert np.all(got[ref == 0] == 0)
    assert np.array_equal(cnt.cpu().numpy(), pr.sumwt(wl.weight)[1])


@pytest.mark.parametrize("form", ["f64", "f32", "f16cf", "bf16cf"])
def test_degrid_parity(awp, form):
    wl, ocf = awp
    say("degrid", form)
    check_degrid(wl, ocf, form)


# --- every row of Table AWP-CFSETUP -------------------------------------------------
# The kernel compositions of the table: PS*A*W, A*W, PS*A (A-Projection),
# A alone and W without the PS taper are the PSTerm-off rows, PS*W
# (W-Projection) and PS alone (Standard).

TERM_ROWS = {"PSxAxW": TERM_PS | TERM_A | TERM_W, "AxW": TERM_A | TERM_W,
             "PSxA": TERM_PS | TERM_A, "A": TERM_A, "PSxW": TERM_PS | TERM_W, "PS": TERM_PS}


@pytest.fixture(scope="module", params=list(TERM_ROWS), ids=list(TERM_ROWS))
def awp_row(request):
    import dataclasses
    wl = awp_workload(seed_id=93, h_max=7)
    wl.cf = dataclasses.replace(wl.cf, terms=TERM_ROWS[request.param])
    return wl, oracle.build_cf(wl.grid, wl.cf)


@pytest.mark.parametrize("form", ["f64", "f32", "f16cf", "bf16cf"])
def test_cf_table_every_row(awp_row, form):
    wl, ocf = awp_row
    say("cf row", wl.cf.terms, form)
    check_cf_table(wl, ocf, form)


@pytest.mark.parametrize("form", ["f64", "f32", "f16cf", "bf16cf"])
def test_grid_parity_every_row(awp_row, form):
    wl, ocf = awp_row
    say("grid row", wl.cf.terms, form)
    check_grid(wl, ocf, form)


@pytest.mark.parametrize("form", ["f64", "f32", "f16cf", "bf16cf"])
def test_degrid_parity_every_row(awp_row, form):
    wl, ocf = awp_row
    say("degrid row", wl.cf.terms, form)
    check_degrid(wl, ocf, form)


@pytest.mark.parametrize("form", ["f64", "f32", "f16cf"])
def test_psf_parity_and_hermitian(awp, form):
    wl, ocf = awp
    say("psf", form)
    p = PREC[form]
    cf = W.build_cf(wl, p)
    v = W.device_vis(wl, p, with_vis=False)
    g = W.empty_grid(wl, p)
    sw = torch.zeros((wl.grid.nplane, wl.grid.npol), dtype=torch.float64, device=DEV)
    cnt = torch.zeros(3, dtype=torch.int64, device=DEV)
    lr.lr_make_psf(cf, v, p, g, sumwt=sw, counters=cnt)
    got = g.cpu().numpy()
    pr = Problem.from_workload(wl, ocf)
    ref, s_ref, c_ref = pr.psf(wl.weight)
    e = rel(got, ref)
    say("psf rel-rms", form, e)
    assert e <= TOL[form]
    assert np.array_equal(cnt.cpu().numpy(), c_ref)
    assert np.allclose(sw.cpu().numpy(), s_ref, rtol=1e-12, atol=0)
    # Hermitian: psf[ny - i][nx - j] = conj psf[i][j] up to the atomics' order
    a = got[..., 1:, 1:]
    b = np.conj(a[..., ::-1, ::-1])
    assert rel(a, b) <= (1e-14 if form == "f64" else 1e-6)


@pytest.mark.parametrize("form", ["f64", "f32"])
def test_pointing_phasor_parity(awp_po, form):
    wl, ocf = awp_po
    say("pointing", form)
    g, _, cnt = run_grid(wl, form)
    pr = Problem.from_workload(wl, ocf)
    assert pr.po
    ref = pr.grid(wl.vis, wl.weight)
    e = rel(g, ref)
    say("pointing grid rel-rms", form, e)
    assert e <= TOL[form]
    plain = Problem.from_workload(wl, ocf, pointing=False).grid(wl.vis, wl.weight)
    assert rel(plain, ref) > 1e-4          # the phasor is not a no-op here
    # degrid through the phasor
    p = PREC[form]
    rng = np.random.default_rng(6)
    x = rng.standard_normal(pr.grid_shape()) + 1j * rng.standard_normal(pr.grid_shape())
    cf = W.build_cf(wl, p)
    v = W.device_vis(wl, p)
    cdt = torch.complex128 if p == lr.LR_F64 else torch.complex64
    lr.lr_degrid(cf, v, p, torch.as_tensor(x, device=DEV).to(cdt))
    e2 = rel(v.vis.cpu().numpy(), pr.degrid(x, wl.weight))
    say("pointing degrid rel-rms", form, e2)
    assert e2 <= TOL[form]


def test_adjoint_identity_on_gpu(awp_po):
    wl, _ = awp_po
    p = lr.LR_F64
    cf = W.build_cf(wl, p)
    v = W.device_vis(wl, p)
    rng = np.random.default_rng(8)
    shape = (wl.grid.nplane, wl.grid.npol, wl.grid.ny, wl.grid.nx)
    x = torch.as_tensor(rng.standard_normal(shape) + 1j * rng.standard_normal(shape), device=DEV)
    y = torch.as_tensor(rng.standard_normal(wl.vis.shape) + 1j * rng.standard_normal(wl.vis.shape),
                        device=DEV)
    lr.lr_degrid(cf, v, p, x)
    dx = v.vis.clone()
    unit = (v.weight != 0).to(torch.float64)
    gy = torch.zeros_like(x)
    lr.lr_grid(cf, v.with_(vis=y, weight=unit), p, gy)
    lhs = torch.vdot(dx.flatten(), y.flatten()).item()
    rhs = torch.vdot(x.flatten(), gy.flatten()).item()
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


@pytest.mark.parametrize("form", ["f64", "f32"])
def test_config1_full(form):
    wl = synth.config1_plain()
    say("config1", form)
    ocf = oracle.build_cf(wl.grid, wl.cf)
    g, sw, cnt = run_grid(wl, form)
    pr = Problem.from_workload(wl, ocf)
    ref = pr.grid(wl.vis, wl.weight)
    assert rel(g, ref) <= TOL[form]
    assert cnt[0] == wl.vis.size


def test_empty_and_fully_flagged_inputs(awp):
    wl, _ = awp
    p = lr.LR_F32
    cf = W.build_cf(wl, p)
    v = W.device_vis(wl, p, rows=slice(0, 0))
    g = W.empty_grid(wl, p)
    cnt = torch.zeros(3, dtype=torch.int64, device=DEV)
    lr.lr_grid(cf, v, p, g, counters=cnt)
    lr.lr_degrid(cf, v, p, g)
    assert cnt.sum().item() == 0 and g.abs().sum().item() == 0
    v = W.device_vis(wl, p)
    v.weight.zero_()
    lr.lr_grid(cf, v, p, g, counters=cnt)
    assert g.abs().sum().item() == 0
    assert cnt[1].item() == wl.weight.size


def test_errors_leave_outputs_untouched(awp):
    wl, _ = awp
    cf = W.build_cf(wl, lr.LR_F32)
    v = W.device_vis(wl, lr.LR_F64)
    g = W.empty_grid(wl, lr.LR_F64)
    with pytest.raises(lr.LRError) as ei:
        lr.lr_grid(cf, v, lr.LR_F64, g)       # storage f32 vs precision f64
    assert ei.value.status == lr.LR_E_DTYPE
    assert g.abs().sum().item() == 0


@pytest.mark.parametrize("dt_s", [0.5, 20.0])
def test_tracks_longer_than_one_wavefront(dt_s):
    """Time-major rows with 400 dumps: the track presum cuts each track into
    several wavefront segments, so group runs cross segment boundaries (they
    are added atomically) or lie inside one (a single-run group is stored).
    Short dumps give long runs, long dumps mostly one-sample groups."""
    wl = synth.tiny_workload(n_ant=5, n_time=400, dt_s=dt_s, nchan=2, nx=96, ny=96,
                             cell_arcsec=4.0, diameter_m=3000.0, n_w=4, h_min=3, h_max=5,
                             oversample=8, terms=TERM_PS | TERM_W, cfg_id=96)
    ocf = oracle.build_cf(wl.grid, wl.cf)
    pr = Problem.from_workload(wl, ocf)
    ref = pr.grid(wl.vis, wl.weight)
    s_ref, c_ref = pr.sumwt(wl.weight)
    for form in ("f64", "f32"):
        g, sw, cnt = run_grid(wl, form, plan=True)
        say("long tracks", dt_s, form, rel(g, ref))
        assert rel(g, ref) <= TOL[form]
        assert np.array_equal(cnt, c_ref)
        assert np.max(np.abs(sw - s_ref) / np.abs(s_ref).max()) < 1e-12
    p = lr.LR_F64
    cf = W.build_cf(wl, p)
    v = W.device_vis(wl, p)
    v.plan = lr.Plan(cf, v)
    assert v.plan.info()["n_groups"] < v.plan.info()["n_kept"] or dt_s > 1
