"""Pins of the oracle's G-Jones calibration (calibration section: Eqs. VAvg,
XChisq, CalUpdateDir, CalUpdateModel), CPU only.

They rest on what the mathematics fixes: data made exactly as
g_i conj(g_j) V^Mod average to exactly g_i conj(g_j) and are solved back to
the true gains up to the one phase the data cannot see; the true gains are
a fixed point of the update; the converged gains make chi^2 stationary;
the ratio average is invariant under weight scaling and scales as 1/s when
the model scales by s; flags, autocorrelations and unused intervals take no
part."""

import numpy as np

from oracle import calibration as cal


def layout(nant, ndump, rng):
    a1, a2 = np.triu_indices(nant, 1)
    ant1 = np.tile(a1, ndump).astype(np.int32)
    ant2 = np.tile(a2, ndump).astype(np.int32)
    return ant1, ant2


def make(nant=7, ndump=6, nchan=5, npol=4, n_tsol=2, n_fsol=2, seed=0, noise=0.0):
    rng = np.random.default_rng(seed)
    ant1, ant2 = layout(nant, ndump, rng)
    nrow = len(ant1)
    g = (1.0 + 0.3 * rng.standard_normal((n_tsol, n_fsol, 2, nant))) * \
        np.exp(1j * rng.uniform(-np.pi, np.pi, (n_tsol, n_fsol, 2, nant)))
    row_sol = (np.arange(nrow) * n_tsol // nrow).astype(np.int32)
    chan_sol = (np.arange(nchan) * n_fsol // nchan).astype(np.int32)
    vmod = (rng.standard_normal((nrow, nchan, npol)) + 1j * rng.standard_normal((nrow, nchan, npol)))
    vobs = np.zeros_like(vmod)
    hands = cal.parallel_hands(npol)
    for r in range(nrow):
        for c in range(nchan):
            for q, p in enumerate(hands):
                gg = g[row_sol[r], chan_sol[c], q]
                vobs[r, c, p] = gg[ant1[r]] * np.conj(gg[ant2[r]]) * vmod[r, c, p]
    vobs += noise * (rng.standard_normal(vobs.shape) + 1j * rng.standard_normal(vobs.shape))
    w = rng.uniform(0.5, 2.0, (nrow, nchan, npol))
    return dict(vobs=vobs, vmod=vmod, w=w, ant1=ant1, ant2=ant2, nant=nant, row_sol=row_sol,
                n_tsol=n_tsol, chan_sol=chan_sol, n_fsol=n_fsol, g=g)


def run_vavg(d, **over):
    a = dict(d, **over)
    return cal.vavg(a["vobs"], a["vmod"], a["w"], a["ant1"], a["ant2"], a["nant"],
                    a["row_sol"], a["n_tsol"], a["chan_sol"], a["n_fsol"])


def products(g):
    return g[:, None] * np.conj(g[None, :])


def test_exact_data_average_to_the_gain_products():
    d = make()
    X, w = run_vavg(d)
    nant = d["nant"]
    off = ~np.eye(nant, dtype=bool)
    for ts in range(2):
        for fs in range(2):
            for q in range(2):
                P = products(d["g"][ts, fs, q])
                assert np.max(np.abs(X[ts, fs, q][off] - P[off])) < 1e-13
                assert np.all(w[ts, fs, q][off] > 0) and np.all(np.diag(w[ts, fs, q]) == 0)
                assert np.allclose(X[ts, fs, q], np.conj(X[ts, fs, q].T), rtol=0, atol=0)


def test_true_gains_are_a_fixed_point_and_are_recovered():
    d = make(seed=1)
    X, w = run_vavg(d)
    g = d["g"][1, 0, 1]
    assert np.max(np.abs(cal.update_dir(g, X[1, 0, 1], w[1, 0, 1]) - g)) < 1e-13
    # the undamped update (alpha = 1) oscillates between two states; the
    # step size of Eq. CalUpdateModel is what makes it converge
    for alpha in (0.5, 0.3):
        sol, it, change = cal.solve(X[1, 0, 1], w[1, 0, 1], np.ones(d["nant"], complex), alpha,
                                    1e-13, 2000)
        assert change < 1e-13 and it < 2000
        # only g_i conj(g_j) is seen by the data: compare those
        assert np.max(np.abs(products(sol) - products(g))) < 1e-10


def test_noisy_solution_is_a_stationary_point_of_chi2():
    d = make(seed=2, noise=0.05)
    X, w = run_vavg(d)
    Xp, wp = X[0, 1, 0], w[0, 1, 0]
    g, it, change = cal.solve(Xp, wp, np.ones(d["nant"], complex), 0.5, 1e-14, 5000)
    assert change < 1e-14
    c0 = cal.chi2(Xp, wp, g)
    rng = np.random.default_rng(3)
    for _ in range(20):
        dirn = rng.standard_normal(len(g)) + 1j * rng.standard_normal(len(g))
        dirn /= np.linalg.norm(dirn)
        eps = 1e-4
        cp, cm = cal.chi2(Xp, wp, g + eps * dirn), cal.chi2(Xp, wp, g - eps * dirn)
        # first-order term vanishes: the symmetric difference is O(eps^2)
        assert abs(cp - cm) < 1e-6 * max(c0, 1.0)
        assert cp > c0 - 1e-12 and cm > c0 - 1e-12


def test_weight_and_model_scaling():
    d = make(seed=4, noise=0.1)
    X, w = run_vavg(d)
    X2, w2 = run_vavg(d, w=3.0 * d["w"])
    assert np.allclose(X2, X, rtol=1e-13, atol=1e-15) and np.allclose(w2, 3.0 * w, rtol=1e-13)
    s = 2.5
    X3, w3 = run_vavg(d, vmod=s * d["vmod"])
    assert np.allclose(X3, X / s, rtol=1e-13, atol=1e-15)
    assert np.allclose(w3, s * s * w, rtol=1e-13)


def test_flags_autocorrelations_and_unused_intervals_take_no_part():
    d = make(seed=5, noise=0.1)
    X, w = run_vavg(d)
    # extra autocorrelation rows and rows / channels outside every interval
    nrow, nchan, npol = d["vobs"].shape
    rng = np.random.default_rng(6)
    extra = 10
    junk = rng.standard_normal((extra, nchan, npol)) * (1 + 1j)
    ant = rng.integers(0, d["nant"], extra).astype(np.int32)
    d2 = dict(d, vobs=np.concatenate([d["vobs"], junk]), vmod=np.concatenate([d["vmod"], junk]),
              w=np.concatenate([d["w"], np.ones((extra, nchan, npol))]),
              ant1=np.concatenate([d["ant1"], ant]), ant2=np.concatenate([d["ant2"], ant]),
              row_sol=np.concatenate([d["row_sol"], np.zeros(extra, np.int32)]))
    X2, w2 = run_vavg(d2)
    assert np.array_equal(X2, X) and np.array_equal(w2, w)
    d3 = dict(d2, ant2=np.concatenate([d["ant2"], (ant + 1) % d["nant"]]),
              row_sol=np.concatenate([d["row_sol"], -np.ones(extra, np.int32)]))
    X3, w3 = run_vavg(d3)
    assert np.array_equal(X3, X) and np.array_equal(w3, w)
    # a zero weight, or a zero model, removes exactly that sample
    wz = d["w"].copy()
    wz[3, 2, 0] = 0.0
    vz = d["vmod"].copy()
    vz[3, 2, 0] = 0.0
    Xa, wa = run_vavg(d, w=wz)
    Xb, wb = run_vavg(d, vmod=vz)
    assert np.allclose(Xa, Xb, rtol=1e-14, atol=0) and np.allclose(wa, wb, rtol=1e-14, atol=0)
    i, j = d["ant1"][3], d["ant2"][3]
    assert wa[d["row_sol"][3], d["chan_sol"][2], 0, i, j] < w[d["row_sol"][3], d["chan_sol"][2], 0, i, j]


def test_exit_criteria():
    d = make(seed=7, noise=0.05)
    X, w = run_vavg(d)
    g, it, _ = cal.solve(X[0, 0, 0], w[0, 0, 0], np.ones(d["nant"], complex), 0.5, 1e9, 100)
    assert it == 1
    g, it, change = cal.solve(X[0, 0, 0], w[0, 0, 0], np.ones(d["nant"], complex), 0.5, 0.0, 7)
    assert it == 7 and change > 0.0
