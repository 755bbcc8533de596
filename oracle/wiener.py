"""Closed-form Wiener filter for linear Gaussian data (test infrastructure only).

With the distances and sigma_NL held fixed, the posterior of Section 2 is
Gaussian in the independent mode coordinates x (eq:q order): the prior is
N(0, S) with S = diag(sigma_k^2 / 2) per real coordinate (eq:prior-k), and the
data y_i = v_obs,i (eq:vrobs) depend linearly on x through y = A x + noise,
noise ~ N(0, K), K = diag(kappa_i^2) (eqn:lvr, eq:kappa).  Its mean and
covariance are the Wiener filter
    x_WF = S A^T (A S A^T + K)^-1 y,   C = S - S A^T (A S A^T + K)^-1 A S,
which an HMC chain on that posterior must reproduce (eq:int_mc).

A is built column by column by applying the oracle's own forward operator
(modes -> projected, interpolated velocity) to each basis vector, and the
system is solved densely in FP64.  Practical on 8^3 - 16^3 grids only.
"""
import numpy as np

from . import hmc, model


def forward_matrix(prob, d):
    """Dense A (n_gal x n_dof) of u(x) at fixed distances d."""
    n = prob.n_grid
    ndof = 2 * int(hmc.canonical_mask(n).sum())
    cols = []
    for a in range(ndof):
        e = np.zeros(ndof)
        e[a] = 1.0
        cols.append(model.project_gather(prob, hmc.unpack_modes(n, e), d))
    return np.stack(cols, axis=1)


def wiener_filter(prob, d, s):
    """Returns (x_wf, diag C, A, S) in the flat coordinates of hmc.pack_modes."""
    n = prob.n_grid
    var = model.mode_variance(prob)
    sv = hmc.pack_modes(n, var.astype(np.complex128))
    m = len(sv) // 2
    s_diag = 0.5 * sv[:m]
    s_diag = np.concatenate([s_diag, s_diag])
    a = forward_matrix(prob, d)
    zb = model.zbar(d, prob.omega_m)
    snl = model.SIGMA_NL_UNIT * s
    kappa2 = snl * snl + prob.sigma_cz ** 2 / (1.0 + zb) ** 2
    y = model.v_obs(prob.cz, d, prob.omega_m)
    sat = s_diag[:, None] * a.T
    gram = a @ sat + np.diag(kappa2)
    x_wf = sat @ np.linalg.solve(gram, y)
    cov_diag = s_diag - np.einsum("ij,ji->i", sat, np.linalg.solve(gram, sat.T))
    return x_wf, cov_diag, a, s_diag
