"""Zeroth prolate spheroidal wave function psi_0(c, eta) on [-1, 1].

The paper's Standard convolution function is the anti-aliasing prolate
spheroidal (Table AWP-CFSETUP, "PS").  psi_0 is the eigenfunction of largest
eigenvalue of the finite Fourier operator restricted to even functions,

    integral_{-1}^{1} cos(c x t) psi(t) dt = mu psi(x),

discretised here by Gauss-Legendre quadrature (Nystrom): the symmetric matrix
sqrt(w_i) cos(c t_i t_j) sqrt(w_j) is diagonalised with a library eigen
solver, its top eigenvector gives psi at the nodes, and the Nystrom formula
interpolates psi(x) = (1/mu) sum_j w_j cos(c x t_j) psi(t_j).  Normalised to
psi_0(c, 0) = 1.  c = pi * S_ps / 2 for a taper whose uv support is S_ps
cells.
"""

import numpy as np


def pswf_nystrom(c, n_nodes=64):
    """Return (psi(x) callable normalised to psi(0) = 1, mu, nodes, psi at nodes)."""
    t, w = np.polynomial.legendre.leggauss(n_nodes)
    sw = np.sqrt(w)
    a = sw[:, None] * np.cos(c * np.outer(t, t)) * sw[None, :]
    ev, vec = np.linalg.eigh(a)
    mu = ev[-1]
    v = vec[:, -1]
    if v.sum() < 0:
        v = -v
    psi_nodes = v / sw

    def raw(x):
        x = np.atleast_1d(np.asarray(x, dtype=np.float64))
        return (np.cos(c * np.outer(x, t)) @ (w * psi_nodes)) / mu

    p0 = raw(0.0)[0]

    def psi(x):
        return raw(x) / p0

    return psi, mu, t, psi_nodes / p0


def pswf0(c, x, n_nodes=64):
    psi, _, _, _ = pswf_nystrom(c, n_nodes)
    return psi(x)
