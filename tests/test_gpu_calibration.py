"""GPU: diagonal G-Jones calibration (calibration section) against the oracle.

lr_cal_vavg must reproduce the oracle's ratio averages (Eq. VAvg) on data
with both baseline orientations, autocorrelations, flags, zero model
samples, rows and channels outside every interval, several intervals and
one, two or four correlations, for complex128 and complex64 inputs (sums in
FP64 either way, so the bar is FP64 rounding) and for any rows-per-step
value; lr_cal_solve must take the oracle's iterations (Eqs. CalUpdateDir,
CalUpdateModel) to the same gains in the same number of steps.  The whole
solver, with model visibilities predicted by the library's degridder,
recovers known gains.
"""

import numpy as np
import pytest

import synth
from oracle import calibration as ocal
from oracle.cfbuild import TERM_PS, TERM_W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2508_17187_amd import calibration as cal  # noqa: E402
from paper_2508_17187_amd import lr  # noqa: E402
from paper_2508_17187_amd import workload as W  # noqa: E402

DEV = "cuda"


def rel(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def dataset(npol=4, nant=9, ndump=41, nchan=6, n_tsol=3, n_fsol=2, seed=160):
    rng = np.random.default_rng(seed)
    a1, a2 = np.triu_indices(nant, 1)
    nbl = len(a1)
    ant1 = np.tile(a1, ndump).astype(np.int32)
    ant2 = np.tile(a2, ndump).astype(np.int32)
    nrow = len(ant1)
    # some rows in the other orientation, a few autocorrelations
    flip = rng.random(nrow) < 0.2
    ant1[flip], ant2[flip] = ant2[flip].copy(), ant1[flip].copy()
    auto = rng.random(nrow) < 0.02
    ant2[auto] = ant1[auto]
    row_sol = (np.arange(nrow) // nbl * n_tsol // ndump).astype(np.int32)
    row_sol[rng.random(nrow) < 0.03] = -1
    chan_sol = (np.arange(nchan) * n_fsol // nchan).astype(np.int32)
    chan_sol[-1] = -1                                   # a channel outside every interval
    g = (1.0 + 0.2 * rng.standard_normal((n_tsol, n_fsol, 2, nant))) * \
        np.exp(1j * rng.uniform(-np.pi, np.pi, (n_tsol, n_fsol, 2, nant)))
    vmod = rng.standard_normal((nrow, nchan, npol)) + 1j * rng.standard_normal((nrow, nchan, npol))
    vmod[rng.random(vmod.shape) < 0.02] = 0.0
    hands = ocal.parallel_hands(npol)
    vobs = 0.05 * (rng.standard_normal(vmod.shape) + 1j * rng.standard_normal(vmod.shape))
    for r in range(nrow):
        ts = max(row_sol[r], 0)
        for c in range(nchan):
            fs = max(chan_sol[c], 0)
            for q, p in enumerate(hands):
                gg = g[ts, fs, q]
                vobs[r, c, p] += gg[ant1[r]] * np.conj(gg[ant2[r]]) * vmod[r, c, p]
    w = rng.uniform(0.5, 2.0, vmod.shape)
    w[rng.random(w.shape) < 0.05] = 0.0
    return dict(vobs=vobs, vmod=vmod, w=w, ant1=ant1, ant2=ant2, nant=nant, row_sol=row_sol,
                n_tsol=n_tsol, chan_sol=chan_sol, n_fsol=n_fsol, nbl=nbl, g=g)


def to_dev(d, f64):
    cdt, rdt = (torch.complex128, torch.float64) if f64 else (torch.complex64, torch.float32)
    t = {k: torch.as_tensor(d[k], device=DEV) for k in ("ant1", "ant2", "row_sol", "chan_sol")}
    t["vobs"] = torch.as_tensor(d["vobs"], device=DEV).to(cdt).contiguous()
    t["vmod"] = torch.as_tensor(d["vmod"], device=DEV).to(cdt).contiguous()
    t["w"] = torch.as_tensor(d["w"], device=DEV).to(rdt).contiguous()
    return t


def oracle_vavg(d, t):
    # the oracle sees exactly the values the device holds
    return ocal.vavg(t["vobs"].cpu().numpy(), t["vmod"].cpu().numpy(), t["w"].cpu().numpy(),
                     d["ant1"], d["ant2"], d["nant"], d["row_sol"], d["n_tsol"], d["chan_sol"],
                     d["n_fsol"])


def gpu_vavg(d, t, rows_per_step):
    return lr.lr_cal_vavg(t["vobs"], t["vmod"], t["w"], t["ant1"], t["ant2"], d["nant"],
                          t["row_sol"], d["n_tsol"], t["chan_sol"], d["n_fsol"],
                          rows_per_step=rows_per_step)


@pytest.mark.parametrize("npol", [1, 2, 4])
@pytest.mark.parametrize("f64", [True, False], ids=["c128", "c64"])
def test_vavg_matches_oracle(npol, f64):
    d = dataset(npol=npol, seed=160 + npol)
    t = to_dev(d, f64)
    Xo, wo = oracle_vavg(d, t)
    for rps in (d["nbl"], 1, 7):
        X, w = gpu_vavg(d, t, rps)
        torch.cuda.synchronize()
        Xg, wg = X.cpu().numpy(), w.cpu().numpy()
        print("vavg", npol, f64, rps, rel(Xg, Xo), rel(wg, wo), flush=True)
        assert Xg.shape == Xo.shape
        assert rel(wg, wo) < 1e-13 and rel(Xg, Xo) < 1e-13
        assert np.array_equal(wg == 0, wo == 0)          # the same bins hold samples
        assert np.array_equal(Xg, np.conj(np.swapaxes(Xg, -1, -2)))


def test_vavg_interleaved_intervals():
    """Frequency intervals that interleave channels, so that equal bins are
    not neighbours: same averages as the oracle."""
    d = dataset(seed=175)
    d["chan_sol"] = np.array([1, 0, 1, 0, -1, 1], np.int32)
    t = to_dev(d, True)
    Xo, wo = oracle_vavg(d, t)
    for rps in (d["nbl"], 1):
        X, w = gpu_vavg(d, t, rps)
        torch.cuda.synchronize()
        assert rel(X.cpu().numpy(), Xo) < 1e-13 and rel(w.cpu().numpy(), wo) < 1e-13


def test_ids_out_of_range_are_ignored():
    d = dataset(seed=170)
    t = to_dev(d, True)
    X0, w0 = gpu_vavg(d, t, d["nbl"])
    a1 = t["ant1"].clone()
    a1[::17] = d["nant"] + 3
    a2 = t["ant2"].clone()
    a2[5::23] = -2
    # the oracle without those rows
    keep = np.ones(len(d["ant1"]), bool)
    keep[::17] = False
    keep[5::23] = False
    dk = dict(d, vobs=d["vobs"][keep], vmod=d["vmod"][keep], w=d["w"][keep],
              ant1=d["ant1"][keep], ant2=d["ant2"][keep], row_sol=d["row_sol"][keep])
    tk = to_dev(dk, True)
    Xo, wo = oracle_vavg(dk, tk)
    X, w = lr.lr_cal_vavg(t["vobs"], t["vmod"], t["w"], a1, a2, d["nant"], t["row_sol"],
                          d["n_tsol"], t["chan_sol"], d["n_fsol"], rows_per_step=d["nbl"])
    torch.cuda.synchronize()
    assert rel(X.cpu().numpy(), Xo) < 1e-13 and rel(w.cpu().numpy(), wo) < 1e-13


def test_solve_matches_oracle():
    d = dataset(seed=171)
    t = to_dev(d, True)
    Xo, wo = oracle_vavg(d, t)
    X = torch.as_tensor(Xo, device=DEV)
    w = torch.as_tensor(wo, device=DEV)
    for alpha, delta, max_iter in ((0.5, 1e-9, 1000), (0.3, 1e-6, 1000), (0.5, 0.0, 25)):
        g, it, ch = lr.lr_cal_solve(X, w, alpha=alpha, delta=delta, max_iter=max_iter)
        torch.cuda.synchronize()
        g, it, ch = g.cpu().numpy(), it.cpu().numpy(), ch.cpu().numpy()
        for idx in np.ndindex(it.shape):
            go, ito, cho = ocal.solve(Xo[idx], wo[idx], np.ones(d["nant"], complex), alpha,
                                      delta, max_iter)
            assert abs(int(it[idx]) - ito) <= 1, (idx, it[idx], ito)
            if int(it[idx]) == ito:
                assert np.max(np.abs(g[idx] - go)) < 1e-10
                assert abs(ch[idx] - cho) <= 1e-10 * max(cho, 1e-300) + 1e-14
        print("solve", alpha, delta, max_iter, it.ravel()[:6], flush=True)


def test_solve_recovers_true_gains():
    d = dataset(seed=172)
    t = to_dev(d, True)
    X, w = gpu_vavg(d, t, d["nbl"])
    g, it, ch = lr.lr_cal_solve(X, w, alpha=0.5, delta=1e-12, max_iter=3000)
    torch.cuda.synchronize()
    g = g.cpu().numpy()
    assert (ch.cpu().numpy() < 1e-12).all()
    for idx in np.ndindex(g.shape[:-1]):
        P = g[idx][:, None] * np.conj(g[idx][None, :])
        T = d["g"][idx][:, None] * np.conj(d["g"][idx][None, :])
        off = ~np.eye(d["nant"], dtype=bool)
        # noise 0.05 on unit model amplitudes, averaged over many samples
        assert np.max(np.abs(P - T)[off]) < 0.05


def test_whole_solver_with_degridded_model():
    """Model visibilities from lr_degrid of a point-source model image; the
    observed data are those times known gains, so the gain products are
    recovered to rounding."""
    wl = synth.tiny_workload(n_ant=10, n_time=24, nchan=4, nx=128, ny=128, cell_arcsec=4.0,
                             diameter_m=1500.0, oversample=16, terms=TERM_PS | TERM_W, n_w=4,
                             h_min=3, h_max=5, cfg_id=173)
    p = lr.LR_F64
    cf = W.build_cf(wl, p)
    v = W.device_vis(wl, p)
    nant = 10
    model = torch.zeros((1, 4, 128, 128), dtype=torch.float64, device=DEV)
    model[0, 0, 60, 70] = 1.0
    model[0, 3, 60, 70] = 1.0
    model[0, 0, 75, 50] = 0.5
    model[0, 3, 75, 50] = 0.5
    from paper_2508_17187_amd.imaging import predict
    vmod = predict(cf, v, p, model)
    rng = np.random.default_rng(174)
    gt = (1.0 + 0.2 * rng.standard_normal((2, nant))) * np.exp(1j * rng.uniform(-3, 3, (2, nant)))
    a1 = torch.as_tensor(wl.obs.ant1.astype(np.int32), device=DEV)
    a2 = torch.as_tensor(wl.obs.ant2.astype(np.int32), device=DEV)
    G = torch.as_tensor(gt, device=DEV)
    vobs = vmod.clone()
    for q, pp in enumerate((0, 3)):
        vobs[:, :, pp] = G[q][a1.long()][:, None] * torch.conj(G[q][a2.long()])[:, None] * \
            vmod[:, :, pp]
    nbl = nant * (nant - 1) // 2
    row_sol = torch.zeros(wl.obs.nrow, dtype=torch.int32, device=DEV)
    chan_sol = torch.zeros(wl.obs.nchan, dtype=torch.int32, device=DEV)
    sol = cal.solve_gains(vobs, vmod, v.weight, a1, a2, nant, row_sol, 1, chan_sol, 1,
                          rows_per_step=nbl, delta=1e-13, max_iter=5000)
    torch.cuda.synchronize()
    g = sol.g.cpu().numpy()[0, 0]
    for q in range(2):
        P = g[q][:, None] * np.conj(g[q][None, :])
        T = gt[q][:, None] * np.conj(gt[q][None, :])
        off = ~np.eye(nant, dtype=bool)
        assert np.max(np.abs(P - T)[off]) < 1e-9
    # the oracle on the same device data gives the same averages
    Xo, wo = ocal.vavg(vobs.cpu().numpy(), vmod.cpu().numpy(), v.weight.cpu().numpy(),
                       wl.obs.ant1, wl.obs.ant2, nant, np.zeros(wl.obs.nrow, np.int32), 1,
                       np.zeros(wl.obs.nchan, np.int32), 1)
    assert rel(sol.X.cpu().numpy(), Xo) < 1e-13
