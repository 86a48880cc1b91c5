"""Diagonal G-Jones calibration (the calibration section: Eqs. VAvg, XChisq,
CalUpdateDir, CalUpdateModel) -- test infrastructure only.

Plain FP64 numpy, one solution problem at a time, in the paper's order:

PreSolvePrep (Eq. VAvg)
    per solution interval (a time interval of rows x a frequency interval of
    channels), parallel-hand polarisation p and baseline (i, j), i != j:
        X_ij = sum W V^c conj(V^Mod) / sum W |V^Mod|^2,
        w_ij = sum W |V^Mod|^2,
    the sums over the interval's (row, channel) samples with W > 0 and
    V^Mod != 0.  This is the weighted mean of the ratios V^c / V^Mod, each
    ratio weighted by its inverse variance W |V^Mod|^2 (the paper's sum of
    ratios, normalised so that X_ij estimates g_i conj(g_j)); w_ij is the
    weight of X_ij in chi^2 (Eq. XChisq).  X_ji = conj(X_ij), w_ji = w_ij;
    autocorrelations take no part.  V^c is the observed data (no earlier
    calibration term is applied).
UpdateDir (Eq. CalUpdateDir)
    dg_i = sum_{j != i} g_j X_ij w_ij / sum_{j != i} |g_j|^2 w_ij,
    every antenna from the same iterate g^k; an antenna with no weight
    keeps its gain.
ModelUpdate (Eq. CalUpdateModel)
    g^{k+1} = (1 - alpha) g^k + alpha dg.
ExitCriteria
    stop when max_i |g_i^{k+1} - g_i^k| < delta, or after max_iter
    iterations.
"""

import numpy as np


def parallel_hands(npol):
    """Indices of the parallel-hand correlations: XX and YY of four, both of
    two, the one of one."""
    return {1: [0], 2: [0, 1], 4: [0, 3]}[npol]


def vavg(v_obs, v_mod, weight, ant1, ant2, nant, row_sol, n_tsol, chan_sol, n_fsol):
    """X [n_tsol, n_fsol, npar, nant, nant] complex128 and w (same shape,
    float64) from [nrow, nchan, npol] data.  row_sol [nrow] and chan_sol
    [nchan] give each row's and channel's interval (< 0: not used)."""
    v_obs = np.asarray(v_obs, np.complex128)
    v_mod = np.asarray(v_mod, np.complex128)
    weight = np.asarray(weight, np.float64)
    nrow, nchan, npol = v_obs.shape
    hands = parallel_hands(npol)
    num = np.zeros((n_tsol, n_fsol, len(hands), nant, nant), np.complex128)
    den = np.zeros((n_tsol, n_fsol, len(hands), nant, nant), np.float64)
    for r in range(nrow):
        i, j, ts = int(ant1[r]), int(ant2[r]), int(row_sol[r])
        if i == j or ts < 0:
            continue
        for c in range(nchan):
            fs = int(chan_sol[c])
            if fs < 0:
                continue
            for q, p in enumerate(hands):
                W = weight[r, c, p]
                M = v_mod[r, c, p]
                if W <= 0.0 or M == 0:
                    continue
                num[ts, fs, q, i, j] += W * v_obs[r, c, p] * np.conj(M)
                den[ts, fs, q, i, j] += W * abs(M) ** 2
    # both orientations of each baseline
    num_h = num + np.conj(np.swapaxes(num, -1, -2))
    den_h = den + np.swapaxes(den, -1, -2)
    X = np.zeros_like(num_h)
    ok = den_h > 0
    X[ok] = num_h[ok] / den_h[ok]
    return X, den_h


def update_dir(g, X, w):
    """Eq. CalUpdateDir for every antenna from the same iterate g."""
    nant = len(g)
    out = np.array(g, np.complex128, copy=True)
    for i in range(nant):
        top = 0j
        bot = 0.0
        for j in range(nant):
            if j == i:
                continue
            top += g[j] * X[i, j] * w[i, j]
            bot += abs(g[j]) ** 2 * w[i, j]
        if bot > 0.0:
            out[i] = top / bot
    return out


def solve(X, w, g0, alpha, delta, max_iter):
    """One problem: (g, iterations, last max |change|)."""
    g = np.array(g0, np.complex128, copy=True)
    it = 0
    change = np.inf
    while it < max_iter:
        dg = update_dir(g, X, w)
        g_new = (1.0 - alpha) * g + alpha * dg
        change = float(np.max(np.abs(g_new - g))) if len(g) else 0.0
        g = g_new
        it += 1
        if change < delta:
            break
    return g, it, change


def chi2(X, w, g):
    """Eq. XChisq over baselines i < j."""
    nant = len(g)
    s = 0.0
    for i in range(nant):
        for j in range(i + 1, nant):
            R = X[i, j] - g[i] * np.conj(g[j])
            s += w[i, j] * abs(R) ** 2
    return s
