"""Oracle Hamiltonian Monte Carlo sampler (test infrastructure only).

Follows Section 3 of the paper: the Hamiltonian eq:Hamiltonian with the
diagonal mass matrix eq:M_ab, Hamilton's equations eq:hamilton integrated by
leapfrog (Section 3.3), fresh momenta for every trajectory and a
Metropolis-Hastings test of the end point (Section 3.2), step-size tuning to
an acceptance rate of 0.65 by dual averaging (Section 3.3, after Hoffman &
Gelman's NUTS paper), and the Monte-Carlo mean eq:int_mc.

Readings used here:
  * Leapfrog is kick-drift-kick; the gradient at the end of a trajectory is
    reused at the start of the next one (L gradients per trajectory).
  * A rejected trajectory repeats the current state as a chain sample and
    new momenta are drawn next iteration (standard Metropolis-Hastings; the
    "start all over" wording of Section 3.2 read as retry-until-accept would
    bias the chain).  The Monte-Carlo mean counts the repeats.
  * Accept iff ln u < -dH with u in (0, 1]; a non-finite dH rejects.
  * Mass matrix per real coordinate: M^-1 = sigma_k^2/2 for each of Re and Im
    of a mode (P(k_j)/2 of eq:M_ab in discrete units), sigma_v^2/H0^2 for a
    distance, 1 for s = sigma_NL/100.  Frozen distances or sigma_NL get no
    momentum and do not move.
"""
import math
from dataclasses import dataclass

import numpy as np

from . import philox
from .model import (H0, exact_sum, logpost_grad, mode_indices, mode_variance, pair_weight,
                    retained_mask)
from .model import mode_dof as model_mode_dof


# ----------------------------------------------------------------------------
# Independent coordinates of the half spectrum
# ----------------------------------------------------------------------------

def mirror_mask(n):
    """kz = 0 entries whose Hermitian partner is the canonical one.

    Canonical half of the kz = 0 plane: ny > 0, or ny = 0 and nx > 0.
    """
    nx, ny, nz = mode_indices(n)
    return retained_mask(n) & (nz == 0) & ((ny < 0) | ((ny == 0) & (nx < 0)))


def canonical_mask(n):
    return retained_mask(n) & ~mirror_mask(n)


def partner_flat_index(n):
    """Flat half-spectrum index of (-kx, -ky, kz) for every entry (kz = 0 use)."""
    j = np.arange(n)
    neg = (-j) % n
    nh = n // 2 + 1
    kz = np.arange(nh)
    return (neg[:, None, None] * n + neg[None, :, None]) * nh + kz[None, None, :]


def symmetrise(n, arr):
    """Overwrite mirror entries with the conjugate of their canonical partner."""
    out = np.array(arr, dtype=np.complex128, copy=True)
    mm = mirror_mask(n)
    flat = out.reshape(-1)
    part = partner_flat_index(n).reshape(-1)
    idx = np.nonzero(mm.reshape(-1))[0]
    flat[idx] = np.conj(flat[part[idx]])
    out[~retained_mask(n)] = 0.0
    return out


def pack_modes(n, dhat):
    """Paper's flat order (eq:q): (Re of independent modes, Im of them)."""
    sel = canonical_mask(n).reshape(-1)
    v = np.asarray(dhat).reshape(-1)[sel]
    return np.concatenate([v.real, v.imag])


def unpack_modes(n, vec):
    sel = canonical_mask(n).reshape(-1)
    m = int(sel.sum())
    out = np.zeros(n * n * (n // 2 + 1), dtype=np.complex128)
    out[sel] = vec[:m] + 1j * vec[m:2 * m]
    return symmetrise(n, out.reshape(n, n, n // 2 + 1))


def pack_state(n, modes, dist, s, cosmo=None):
    """The whole flat parameter vector of Section 3.1 (eq:q): Re and Im of
    the independent modes, then the n distances, then s = sigma_NL/100 (and
    u8, phi, eta when the cosmological parameters are sampled)."""
    tail = [float(s)] + ([] if cosmo is None else [float(c) for c in cosmo])
    return np.concatenate([pack_modes(n, modes), np.asarray(dist, dtype=float), tail])


def unpack_state(n, vec, n_gal, cosmo=False):
    """Inverse of pack_state: (modes with mirror entries filled, dist, s[,
    (u8, phi, eta)])."""
    m2 = (n - 1) ** 3 - 1
    vec = np.asarray(vec, dtype=float)
    assert vec.size == m2 + n_gal + (4 if cosmo else 1)
    out = (unpack_modes(n, vec[:m2]), vec[m2:m2 + n_gal].copy(), float(vec[m2 + n_gal]))
    return out + (vec[m2 + n_gal + 1:].copy(),) if cosmo else out


# ----------------------------------------------------------------------------
# Phase-space state
# ----------------------------------------------------------------------------

@dataclass
class State:
    modes: np.ndarray     # complex (N, N, N/2+1)
    dist: np.ndarray      # (n,)
    s: float              # sigma_NL / 100 km/s
    cosmo: np.ndarray = None   # (u8, phi, eta) when the cosmological parameters are sampled

    def copy(self):
        return State(self.modes.copy(), self.dist.copy(), float(self.s),
                     None if self.cosmo is None else np.array(self.cosmo, dtype=float))


def inverse_mass(prob):
    """Diagonal M^-1 of eq:M_ab: (per real part of each mode, per distance, s)."""
    var = mode_variance(prob)
    minv_modes = 0.5 * var
    minv_d = (prob.sigma_v / H0) ** 2 if prob.sample_distances else 0.0
    minv_s = 1.0 if prob.sample_sigma_nl else 0.0
    return minv_modes, minv_d, minv_s


def cosmo_inverse_mass(prob):
    """M^-1 of (u8, phi, eta) (a reading; eq:M_ab has no such coordinates):
    the inverse curvature of the prior in u8 at the fiducial amplitude,
    1 / (2 D) with D real mode coordinates; 1 / n for phi (each point carries
    information of order one on the amplitude of its velocity); and for eta
    the inverse curvature of the distance-modulus terms at eta = 1 with the
    distances held, 1 / sum_i (5 / ln 10)^2 / sigma_mu,i^2 (1 without points)."""
    if not prob.sample_cosmology:
        return np.zeros(3)
    c = (5.0 / math.log(10.0)) ** 2
    curv = float(np.sum(c / np.asarray(prob.sigma_mu, dtype=float) ** 2)) if prob.n_gal > 0 else 1.0
    return np.array([1.0 / (2.0 * model_mode_dof(prob.n_grid)), 1.0 / max(prob.n_gal, 1), 1.0 / curv])


def draw_momenta(prob, seed, iteration):
    """p ~ N(0, M): variance 2/sigma_k^2 per real part of a mode, etc."""
    n = prob.n_grid
    var = mode_variance(prob)
    nh = n // 2 + 1
    # Stream index of entry (kx, ky, kz): its flat position in the layout
    # without the kz = N/2 plane (which holds only excluded modes),
    # (kx N + ky) N/2 + kz; a mirror entry draws at its canonical partner.
    kx, ky, kz = np.meshgrid(np.arange(n), np.arange(n), np.arange(nh), indexing="ij")
    stream_idx = ((kx * n + ky) * (n // 2) + kz).reshape(-1)
    partner_idx = ((((-kx) % n) * n + ((-ky) % n)) * (n // 2)).reshape(-1)
    mm = mirror_mask(n).reshape(-1)
    src = np.where(mm, partner_idx, stream_idx)
    z0, z1 = philox.normal_pair(philox.draw_words(seed, iteration, philox.PURPOSE_MODES, src))
    scale = np.sqrt(2.0 / np.where(var > 0, var, 1.0)).reshape(-1)
    pm = scale * (z0 + 1j * z1)
    pm = np.where(mm, np.conj(pm), pm)
    pm = np.where(retained_mask(n).reshape(-1), pm, 0.0).reshape(n, n, nh)
    if prob.sample_distances:
        zd, _ = philox.normal_pair(philox.draw_words(seed, iteration, philox.PURPOSE_DIST,
                                                     np.arange(prob.n_gal)))
        pd = (H0 / prob.sigma_v) * zd
    else:
        pd = np.zeros(prob.n_gal)
    if prob.sample_sigma_nl:
        zs, _ = philox.normal_pair(philox.draw_words(seed, iteration, philox.PURPOSE_SNL, [0]))
        ps = float(zs[0])
    else:
        ps = 0.0
    pc = None
    if prob.sample_cosmology:
        # u8 and phi from the pair at index 0, eta from the first of index 1
        z0, z1 = philox.normal_pair(philox.draw_words(seed, iteration, philox.PURPOSE_COSMO, [0, 1]))
        pc = np.array([float(z0[0]), float(z1[0]), float(z0[1])]) / np.sqrt(cosmo_inverse_mass(prob))
    return State(pm, pd, ps, pc)


def kinetic(prob, p):
    """K = (1/2) p^T M^-1 p over independent real coordinates (eq:Hamiltonian).

    Per stored mode entry: (w_k / 8) sigma_k^2 |p_k|^2.
    """
    var = mode_variance(prob)
    w = pair_weight(prob.n_grid)
    _, minv_d, minv_s = inverse_mass(prob)
    terms = [(w * var * np.abs(p.modes) ** 2 / 8.0).ravel(), 0.5 * minv_d * np.asarray(p.dist) ** 2,
             [0.5 * minv_s * p.s * p.s]]
    if prob.sample_cosmology:
        terms.append(0.5 * cosmo_inverse_mass(prob) * np.asarray(p.cosmo) ** 2)
    return exact_sum(np.concatenate(terms))


def gradient(prob, q):
    """(Psi, dPsi/dmodes, dPsi/dd, dPsi/ds, dPsi/d(u8, phi, eta) or None) at q."""
    if prob.sample_cosmology:
        return logpost_grad(prob, q.modes, q.dist, q.s, cosmo=q.cosmo)
    return logpost_grad(prob, q.modes, q.dist, q.s) + (None,)


def leapfrog(prob, q, p, eps, n_steps, cached=None):
    """Kick-drift-kick integration of eq:hamilton.

    cached: (psi, g_modes, g_d, g_s) at q, else computed.  Returns
    (q, p, (psi, g_modes, g_d, g_s)) at the end point.
    """
    q = q.copy()
    p = p.copy()
    if cached is None:
        cached = gradient(prob, q)
    psi, gm, gd, gs, gc = cached
    minv_m, minv_d, minv_s = inverse_mass(prob)
    minv_c = cosmo_inverse_mass(prob)
    for _ in range(n_steps):
        p.modes = p.modes - 0.5 * eps * gm
        p.dist = p.dist - 0.5 * eps * gd if prob.sample_distances else p.dist
        p.s = p.s - 0.5 * eps * gs if prob.sample_sigma_nl else p.s
        if prob.sample_cosmology:
            p.cosmo = p.cosmo - 0.5 * eps * gc
        q.modes = q.modes + eps * minv_m * p.modes
        q.dist = q.dist + eps * minv_d * p.dist
        q.s = q.s + eps * minv_s * p.s
        if prob.sample_cosmology:
            q.cosmo = q.cosmo + eps * minv_c * p.cosmo
        psi, gm, gd, gs, gc = gradient(prob, q)
        p.modes = p.modes - 0.5 * eps * gm
        p.dist = p.dist - 0.5 * eps * gd if prob.sample_distances else p.dist
        p.s = p.s - 0.5 * eps * gs if prob.sample_sigma_nl else p.s
        if prob.sample_cosmology:
            p.cosmo = p.cosmo - 0.5 * eps * gc
    return q, p, (psi, gm, gd, gs, gc)


# ----------------------------------------------------------------------------
# Dual averaging of the step size (Hoffman & Gelman, NUTS paper, Sec. 3.2.1)
# ----------------------------------------------------------------------------

@dataclass
class DualAveraging:
    eps0: float
    target: float = 0.65
    gamma: float = 0.05
    t0: float = 10.0
    kappa: float = 0.75

    def __post_init__(self):
        self.mu = math.log(10.0 * self.eps0)
        self.hbar = 0.0
        self.log_eps_bar = 0.0
        self.m = 0

    def update(self, accept_prob):
        """One adaptation step; returns the step size for the next iteration."""
        self.m += 1
        m = float(self.m)
        eta = 1.0 / (m + self.t0)
        self.hbar = (1.0 - eta) * self.hbar + eta * (self.target - accept_prob)
        log_eps = self.mu - math.sqrt(m) / self.gamma * self.hbar
        wgt = m ** (-self.kappa)
        self.log_eps_bar = wgt * log_eps + (1.0 - wgt) * self.log_eps_bar
        return math.exp(log_eps)

    def final(self):
        return math.exp(self.log_eps_bar)


def accept_probability(dh):
    """min(1, exp(-dH)); 0 for a non-finite dH."""
    if not math.isfinite(dh):
        return 0.0
    return 1.0 if dh <= 0.0 else math.exp(-dh)


# ----------------------------------------------------------------------------
# The chain (Section 3.2, eq:int_mc)
# ----------------------------------------------------------------------------

@dataclass
class ChainResult:
    state: State
    dh: np.ndarray
    accepted: np.ndarray
    eps: float
    mode_sum: np.ndarray
    n_mean: int


def hmc_run(prob, q0, n_iter, n_leapfrog, eps0, seed, warmup=0, target=0.65,
            jitter=False, callback=None):
    """Run n_iter HMC iterations from q0.

    Iterations < warmup adapt the step size by dual averaging; from then on it
    is frozen at the averaged value.  Post-warm-up chain states (repeats
    included) are summed into mode_sum.  With jitter the step of an iteration
    is eps * (0.9 + 0.2 u), u uniform from the Philox stream.
    """
    q = q0.copy()
    cached = gradient(prob, q)
    eps = float(eps0)
    da = DualAveraging(eps0, target) if warmup > 0 else None
    dh_rec = np.zeros(n_iter)
    acc_rec = np.zeros(n_iter, dtype=np.int32)
    mode_sum = np.zeros_like(q.modes)
    n_mean = 0
    for it in range(n_iter):
        eps_it = eps
        if jitter:
            w = philox.draw_words(seed, it, philox.PURPOSE_JITTER, [0])
            eps_it = eps * (0.9 + 0.2 * float(philox.uniform53(w[0, 0], w[0, 1])))
        p = draw_momenta(prob, seed, it)
        h_start = kinetic(prob, p) + cached[0]
        q1, p1, cached1 = leapfrog(prob, q, p, eps_it, n_leapfrog, cached)
        h_end = kinetic(prob, p1) + cached1[0]
        dh = h_end - h_start
        if not math.isfinite(dh):
            dh = math.inf
        w = philox.draw_words(seed, it, philox.PURPOSE_ACCEPT, [0])
        u = float(philox.uniform53(w[0, 0], w[0, 1]))
        accept = math.log(u) < -dh
        if accept:
            q, cached = q1, cached1
        dh_rec[it] = dh
        acc_rec[it] = int(accept)
        if it < warmup:
            eps = da.update(accept_probability(dh))
            if it == warmup - 1:
                eps = da.final()
        else:
            mode_sum += q.modes
            n_mean += 1
        if callback is not None:
            callback(it, q, dh, accept, eps_it)
    return ChainResult(q, dh_rec, acc_rec, eps, mode_sum, n_mean)
