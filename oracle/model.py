"""Oracle posterior of the HAMLET reconstruction: Psi(q) and its gradient.

TEST INFRASTRUCTURE ONLY.  Plain, slow FP64 numpy code that defines what the
GPU path must compute.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import it; the product never does.

Everything follows Section 2 of the paper (eq:covfefe:bay .. eq:D) with the
readings listed below wherever the paper is silent or garbled.

Units: distances in Mpc/h, velocities in km/s, H0 = 100 km/s per Mpc/h.

Parameters q (eq:q): the Fourier modes delta_k of the density contrast, the
true distances d_i of the n catalogue points, and sigma_NL.

Readings of the paper used here (each is also listed in the design notes):
  * Fourier convention.  delta(x) = N^-3 sum_k dhat_k exp(+i k.x) with the
    unnormalised forward transform.  eq:vel-field writes the multiplier as
    -i H0 f k/k^2 without fixing the sign of the transform; with this
    convention the same field (divergence -H0 f delta, i.e. infall onto
    overdensities) needs m_c(k) = +i a H0 f k_c / k^2 (a = 1).
  * Mode variance.  P(k_j) in eq:prior-k is the variance of the complex
    mode; for the unnormalised discrete transform on a box of volume V this
    is sigma_k^2 = <|dhat_k|^2> = N^6 P(|k|) / V.  The normalisation
    constant of eq:prior-k (garbled as 1/(2P)) is a constant and dropped.
  * Retained modes.  k = 0 and every mode with a Nyquist index |n_c| = N/2
    are excluded (zero and not sampled); (N-1)^3 - 1 real degrees of freedom
    remain.  Storage is the half spectrum (kx, ky, kz) with 0 <= kz <= N/2,
    kz fastest; on the kz = 0 plane both members of each Hermitian pair are
    stored, and the pair counts once.
  * Interpolation.  v(d_i r_i) in eqn:lvr is cloud-in-cell (trilinear)
    interpolation on nodes x_j = j*Delta with periodic wrap; the observer sits
    at the box centre o = (L/2)(1,1,1) (Section 5.1).
  * sigma_NL is sampled as s = sigma_NL / (100 km/s) with a flat prior
    (P(sigma_NL) is never given); Psi depends on s^2 only.
  * Constants: ln(2 pi) and ln sigma_mu terms are dropped; the parameter
    dependent ln kappa_i of eqn:lvr is kept.
  * Domain.  zbar(d) needs d < c/(3 Omega0 H0) and mu(d) needs d > 0; outside
    it (or outside the support of the distance histogram) Psi = +inf.
  * Sums.  Psi, dPsi/ds and the kinetic energy are the exact sums of their
    terms rounded once (math.fsum): the Metropolis test takes the difference
    of two such totals of millions of terms, and an exactly rounded sum is
    the plain definition, free of any summation order.
  * Cosmological parameters in q (Section 6, item 3: H0, sigma_8 and the
    growth rate estimated with the field).  With `sample_cosmology` three
    more coordinates join s: u8 = sigma_8 / sigma_8,fid, which scales P(k)
    by u8^2, phi = f / f_fid, which scales the velocity multiplier, and
    eta = h / h_fid.  All three have flat priors on (0, inf) (Psi = +inf
    elsewhere).  The prior of the modes is then the normalised Gaussian of
    variance u8^2 sigma_k^2, whose u8-dependent part is E / u8^2 + D ln u8
    with E the fiducial prior energy and D = (N-1)^3 - 1 the number of real
    mode coordinates.  With distances in Mpc/h and H0 = 100 h km/s/Mpc, h
    enters only the distance modulus (d_L / h in Mpc): mu(d) moves by
    -5 log10 eta, the zero point of every distance modulus at once
    (Section 6, item 4's calibration by a Hubble parameter).
"""
import math
from dataclasses import dataclass, field

import numpy as np

from .fft import fftn, ifftn_unnormalised

C_KMS = 299792.458          # speed of light, km/s
H0 = 100.0                  # Hubble constant, km/s per Mpc/h
SIGMA_NL_UNIT = 100.0       # s = sigma_NL / SIGMA_NL_UNIT


# ----------------------------------------------------------------------------
# Cosmological distance relations (Section 2.2)
# ----------------------------------------------------------------------------

def zbar(d, om):
    """Second-order cosmological redshift of proper distance d (Section 2.2)."""
    return (2.0 / (3.0 * om)) * (1.0 - np.sqrt(1.0 - 3.0 * om * H0 * d / C_KMS))


def zbar_prime(d, om):
    """d zbar / d d = (H0/c) / sqrt(1 - 3 Omega0 H0 d / c)."""
    return (H0 / C_KMS) / np.sqrt(1.0 - 3.0 * om * H0 * d / C_KMS)


def distance_modulus(d, om, h):
    """mu(d) = 5 log10(d_L / 10 pc), d_L = d (1 + zbar(d)) (Section 2.2).

    d is in Mpc/h, so d_L / h is in Mpc and 10 pc = 1e-5 Mpc.
    """
    dl_mpc = d * (1.0 + zbar(d, om)) / h
    return 5.0 * np.log10(dl_mpc) + 25.0


def distance_modulus_prime(d, om):
    """d mu / d d."""
    zb = zbar(d, om)
    zp = zbar_prime(d, om)
    return (5.0 / math.log(10.0)) * (1.0 + zb + d * zp) / (d * (1.0 + zb))


def v_obs(cz, d, om):
    """Observed radial velocity c (z - zbar)/(1 + zbar) (eq:vrobs), z = cz/c."""
    zb = zbar(d, om)
    return C_KMS * (cz / C_KMS - zb) / (1.0 + zb)


def v_obs_prime(cz, d, om):
    """d v_obs / d d = -c zbar' (1 + z) / (1 + zbar)^2."""
    zb = zbar(d, om)
    return -C_KMS * zbar_prime(d, om) * (1.0 + cz / C_KMS) / (1.0 + zb) ** 2


def redshift_distance(z, om, intervals=2000):
    """d_z of eq:e:dz: (c/H0) * int_0^z dz'/sqrt(Om (1+z')^3 + 1 - Om).

    Composite Simpson rule with `intervals` (even) sub-intervals per point.
    """
    z = np.atleast_1d(np.asarray(z, dtype=np.float64))
    j = np.arange(intervals + 1)
    coef = np.where((j == 0) | (j == intervals), 1.0, np.where(j % 2 == 1, 4.0, 2.0))
    hstep = z[:, None] / intervals
    zz = hstep * j[None, :]
    integrand = 1.0 / np.sqrt(om * (1.0 + zz) ** 3 + (1.0 - om))
    return (C_KMS / H0) * (hstep[:, 0] / 3.0) * (integrand * coef[None, :]).sum(axis=1)


# ----------------------------------------------------------------------------
# The distance prior: histogram of redshift distances (eq:D)
# ----------------------------------------------------------------------------

@dataclass
class DistanceHistogram:
    """N^obs_{d_z}: density histogram of the catalogue's redshift distances.

    Reading: bins of width w on [0, max(d_z) + 15 Mpc/h), one pseudo-count per
    bin so that the prior never vanishes inside the support; redshift
    distances below zero are counted in the first bin.
    """
    width: float
    density: np.ndarray

    @classmethod
    def from_catalogue(cls, cz, om, width):
        dz = redshift_distance(np.asarray(cz, dtype=np.float64) / C_KMS, om)
        top = float(dz.max()) if len(dz) else 0.0
        nbins = int(math.ceil((max(top, 0.0) + 15.0) / width))
        b = np.clip(np.floor(dz / width).astype(np.int64), 0, nbins - 1)
        counts = np.bincount(b, minlength=nbins).astype(np.float64)
        density = (counts + 1.0) / ((len(dz) + nbins) * width)
        return cls(width=float(width), density=density)

    def log_density(self, d):
        d = np.asarray(d, dtype=np.float64)
        out = np.full(d.shape, -np.inf)
        ok = np.isfinite(d) & (d >= 0.0)
        b = np.zeros(d.shape, dtype=np.int64)
        b[ok] = np.floor(d[ok] / self.width).astype(np.int64)
        ok &= b < len(self.density)
        out[ok] = np.log(self.density[b[ok]])
        return out


# ----------------------------------------------------------------------------
# Problem statement
# ----------------------------------------------------------------------------

@dataclass
class Problem:
    """One reconstruction problem: grid, cosmology, P(k) and catalogue.

    pk_n2[j] is the power spectrum at |k| = (2 pi / L) sqrt(j) for
    j = 0 .. 3 (N/2)^2 (every value that |n|^2 takes on the grid).
    rhat is (n, 3): the unit vector (cos b cos l, cos b sin l, sin b) of
    supergalactic latitude b and longitude l.
    """
    n_grid: int
    box: float
    omega_m: float
    h: float
    f_growth: float
    sigma_v: float
    pk_n2: np.ndarray
    rhat: np.ndarray
    mu: np.ndarray
    sigma_mu: np.ndarray
    cz: np.ndarray
    sigma_cz: np.ndarray
    hist_width: float = 5.0
    sample_distances: bool = True
    sample_sigma_nl: bool = True
    sample_cosmology: bool = False
    hist: DistanceHistogram = field(default=None)

    def __post_init__(self):
        if self.hist is None:
            self.hist = DistanceHistogram.from_catalogue(self.cz, self.omega_m, self.hist_width)

    @property
    def spacing(self):
        return self.box / self.n_grid

    @property
    def n_gal(self):
        return len(self.mu)


# ----------------------------------------------------------------------------
# Fourier-mode bookkeeping (eq:prior-k, eq:q)
# ----------------------------------------------------------------------------

def signed_index(n):
    """Signed frequency index of array index j on an axis of length n."""
    j = np.arange(n)
    return np.where(j < n // 2, j, j - n)


def half_shape(n):
    return (n, n, n // 2 + 1)


def mode_indices(n):
    """Signed integer wave-vector components (nx, ny, nz) on the half spectrum."""
    s = signed_index(n)
    nx = s[:, None, None] * np.ones(half_shape(n), dtype=np.int64)
    ny = s[None, :, None] * np.ones(half_shape(n), dtype=np.int64)
    nz = np.arange(n // 2 + 1)[None, None, :] * np.ones(half_shape(n), dtype=np.int64)
    return nx, ny, nz


def retained_mask(n):
    """True for retained modes: not k = 0, no component on the Nyquist index."""
    nx, ny, nz = mode_indices(n)
    half = n // 2
    nyq = (np.abs(nx) == half) | (np.abs(ny) == half) | (nz == half)
    zero = (nx == 0) & (ny == 0) & (nz == 0)
    return ~(nyq | zero)


def pair_weight(n):
    """w_k: 2 for 0 < kz < N/2 (partner -k not stored), 1 on kz = 0."""
    _, _, nz = mode_indices(n)
    return np.where(nz == 0, 1.0, 2.0) * retained_mask(n)


def mode_variance(prob):
    """sigma_k^2 = N^6 P(|k|) / V on the half spectrum; 0 where excluded."""
    n = prob.n_grid
    nx, ny, nz = mode_indices(n)
    n2 = nx * nx + ny * ny + nz * nz
    var = (float(n) ** 6 / prob.box ** 3) * np.asarray(prob.pk_n2)[n2]
    return np.where(retained_mask(n), var, 0.0)


def full_spectrum(dhat):
    """Extend a half spectrum to all N^3 modes with dhat(-k) = conj dhat(k)."""
    n = dhat.shape[0]
    full = np.zeros((n, n, n), dtype=np.complex128)
    full[:, :, : n // 2 + 1] = dhat
    j = np.arange(n)
    neg = (-j) % n
    for kz in range(n // 2 + 1, n):
        full[:, :, kz] = np.conj(dhat[np.ix_(neg, neg, [n - kz])][:, :, 0])
    return full


def hermitian_partner_index(n):
    """For each half-spectrum entry on kz = 0, the flat index of (-kx, -ky, 0)."""
    j = np.arange(n)
    neg = (-j) % n
    nh = n // 2 + 1
    return (neg[:, None] * n + neg[None, :]) * nh


def mode_dof(n):
    """Real coordinates of the retained modes: (N-1)^3 - 1."""
    return (n - 1) ** 3 - 1


def velocity_multiplier(prob, phi=1.0):
    """m_c(k) = i a H0 f k_c / k^2 on the half spectrum (eq:vel-field), a = 1,
    with f = phi f_fid.

    Returns complex array (3, N, N, N/2+1); zero on excluded modes.
    """
    n = prob.n_grid
    kf = 2.0 * math.pi / prob.box
    nx, ny, nz = mode_indices(n)
    kvec = [kf * nx, kf * ny, kf * nz]
    k2 = kvec[0] ** 2 + kvec[1] ** 2 + kvec[2] ** 2
    keep = retained_mask(n)
    safe = np.where(keep, k2, 1.0)
    amp = H0 * prob.f_growth * phi
    return np.stack([np.where(keep, 1j * amp * kc / safe, 0.0) for kc in kvec])


# ----------------------------------------------------------------------------
# The velocity field and its interpolation (eq:vel-field, eqn:lvr)
# ----------------------------------------------------------------------------

def velocity_grids(prob, dhat, phi=1.0):
    """v_c(x_j) = N^-3 sum_k m_c(k) dhat_k exp(+i k.x_j) for c = x, y, z."""
    n = prob.n_grid
    mult = velocity_multiplier(prob, phi)
    out = np.empty((3, n, n, n))
    for c in range(3):
        field_c = ifftn_unnormalised(full_spectrum(mult[c] * dhat)) / float(n) ** 3
        out[c] = field_c.real
    return out


def density_grid(prob, dhat):
    """delta(x_j) = N^-3 sum_k dhat_k exp(+i k.x_j) on every node (the Fourier
    convention of eq:prior-k's modes); excluded modes are zero in dhat."""
    n = prob.n_grid
    return (ifftn_unnormalised(full_spectrum(dhat)) / float(n) ** 3).real


def galaxy_positions(prob, d):
    """x_i = o + d_i rhat_i with the observer at o = (L/2)(1, 1, 1)."""
    return 0.5 * prob.box + np.asarray(d)[:, None] * prob.rhat


def cic_cells(prob, x):
    """Lower node index (mod N) and fractional offset per axis for points x."""
    s = x / prob.spacing
    i0 = np.floor(s)
    t = s - i0
    return np.mod(i0.astype(np.int64), prob.n_grid), t


def _corners():
    for ox in (0, 1):
        for oy in (0, 1):
            for oz in (0, 1):
                yield ox, oy, oz


def cic_gather(prob, grids, d):
    """u_i = rhat_i . v(d_i rhat_i) and u'_i = d u_i / d d_i (CIC, periodic).

    grids: (3, N, N, N).  The derivative differentiates the trilinear weights
    along rhat_i: d/dd = sum_a rhat_ia d/dx_a, with d w/dx = -+1/Delta.
    """
    n = prob.n_grid
    x = galaxy_positions(prob, d)
    i0, t = cic_cells(prob, x)
    vel = np.zeros((len(d), 3))
    dvel = np.zeros((len(d), 3, 3))       # dvel[i, c, a] = d v_c / d x_a
    inv = 1.0 / prob.spacing
    for ox, oy, oz in _corners():
        off = np.array([ox, oy, oz])
        w1 = np.where(off == 1, t, 1.0 - t)                  # (n, 3)
        dw1 = np.where(off == 1, inv, -inv) * np.ones_like(t)
        ix = (i0 + off) % n
        vals = grids[:, ix[:, 0], ix[:, 1], ix[:, 2]].T      # (n, 3)
        w = w1[:, 0] * w1[:, 1] * w1[:, 2]
        vel += w[:, None] * vals
        dw = np.stack([dw1[:, 0] * w1[:, 1] * w1[:, 2],
                       w1[:, 0] * dw1[:, 1] * w1[:, 2],
                       w1[:, 0] * w1[:, 1] * dw1[:, 2]], axis=1)   # (n, 3)
        dvel += vals[:, :, None] * dw[:, None, :]
    u = (vel * prob.rhat).sum(axis=1)
    du = np.einsum("ic,ica,ia->i", prob.rhat, dvel, prob.rhat)
    return u, du


def cic_scatter(prob, d, g):
    """Adjoint of the projected gather: G_c(x_j) = sum_i g_i rhat_ic W_i(x_j)."""
    n = prob.n_grid
    x = galaxy_positions(prob, d)
    i0, t = cic_cells(prob, x)
    out = np.zeros((3, n, n, n))
    for ox, oy, oz in _corners():
        off = np.array([ox, oy, oz])
        w1 = np.where(off == 1, t, 1.0 - t)
        w = w1[:, 0] * w1[:, 1] * w1[:, 2]
        ix = (i0 + off) % n
        for c in range(3):
            np.add.at(out[c], (ix[:, 0], ix[:, 1], ix[:, 2]), g * prob.rhat[:, c] * w)
    return out


def project_gather(prob, dhat, d, phi=1.0):
    """The linear map from modes to u_i = rhat_i . v(d_i rhat_i) at fixed d."""
    u, _ = cic_gather(prob, velocity_grids(prob, dhat, phi), np.asarray(d, dtype=np.float64))
    return u


def modes_adjoint(prob, d, g, phi=1.0):
    """Gradient of sum_i g_i u_i with respect to the modes (at fixed d).

    (2/N^3) sum_c conj(m_c(k)) Ghat_c(k), Ghat_c the forward transform of the
    scatter-added grid G_c, in the complex convention of logpost_grad.
    """
    n = prob.n_grid
    grids = cic_scatter(prob, np.asarray(d, dtype=np.float64), np.asarray(g, dtype=np.float64))
    mult = velocity_multiplier(prob, phi)
    nh = n // 2 + 1
    out = np.zeros(half_shape(n), dtype=np.complex128)
    for c in range(3):
        gk = fftn(grids[c])[:, :, :nh]
        out += (2.0 / float(n) ** 3) * np.conj(mult[c]) * gk
    return out


def modes_adjoint_at(prob, d, g, kidx, phi=1.0):
    """modes_adjoint at a few half-spectrum entries kidx = (ix, iy, iz) arrays,
    by the definition of the forward transform summed directly over the
    nodes the points reach: Ghat_c(k) = sum_i g_i rhat_ic sum_corners
    w_corner exp(-2 pi i n.j_corner / N).  For sampled checks on grids whose
    full transforms are too large for the host."""
    n = prob.n_grid
    d = np.asarray(d, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    ix, iy, iz = (np.asarray(a, dtype=np.int64) for a in kidx)
    x = galaxy_positions(prob, d)
    i0, t = cic_cells(prob, x)
    mult = velocity_multiplier(prob, phi)
    s = signed_index(n)
    nvec = np.stack([s[ix], s[iy], iz], axis=1).astype(np.float64)     # (m, 3) signed wave numbers
    ghat = np.zeros((3, len(ix)), dtype=np.complex128)
    for ox, oy, oz in _corners():
        off = np.array([ox, oy, oz])
        w1 = np.where(off == 1, t, 1.0 - t)
        w = w1[:, 0] * w1[:, 1] * w1[:, 2]
        node = (i0 + off) % n                                            # (npts, 3)
        phase = np.exp(-2j * math.pi * (node.astype(np.float64) @ nvec.T) / n)   # (npts, m)
        for c in range(3):
            ghat[c] += (g * prob.rhat[:, c] * w) @ phase
    out = np.zeros(len(ix), dtype=np.complex128)
    for c in range(3):
        out += (2.0 / float(n) ** 3) * np.conj(mult[c][ix, iy, iz]) * ghat[c]
    return out


def logpost_grad_sampled(prob, dhat, d, s, kidx):
    """Psi, the mode gradient at the entries kidx only (as logpost_grad's at
    those entries), dPsi/dd and dPsi/ds.  The velocity field is the full
    inverse transform; the adjoint is summed directly (modes_adjoint_at)."""
    d = np.asarray(d, dtype=np.float64)
    ok = in_domain(prob, d)
    dsafe = np.where(ok, d, 1.0)
    v = velocity_grids(prob, dhat)
    u, du = cic_gather(prob, v, dsafe)
    del v
    t = galaxy_terms(prob, dsafe, s, u)
    om = prob.omega_m
    kappa2, r = t["kappa2"], t["r"]
    zb = t["zbar"]
    g = -r / kappa2
    dk2 = 0.5 / kappa2 - 0.5 * r * r / kappa2 ** 2
    dkappa2_dd = -2.0 * prob.sigma_cz ** 2 * zbar_prime(dsafe, om) / (1.0 + zb) ** 3
    g_d = (-t["dmu"] * distance_modulus_prime(dsafe, om) / prob.sigma_mu ** 2
           + (r / kappa2) * (v_obs_prime(prob.cz, dsafe, om) - du)
           + dk2 * dkappa2_dd)
    g_s = exact_sum(dk2 * 2.0 * SIGMA_NL_UNIT ** 2 * s)
    ix, iy, iz = (np.asarray(a, dtype=np.int64) for a in kidx)
    var = mode_variance(prob)[ix, iy, iz]
    q = np.asarray(dhat)[ix, iy, iz]
    g_modes = np.where(var > 0, 2.0 * q / np.where(var > 0, var, 1.0), 0.0) + modes_adjoint_at(prob, dsafe, g, kidx)
    psi = exact_sum(np.concatenate([[prior_energy(prob, dhat)], t["psi"]])) if np.all(ok) else math.inf
    if not np.isfinite(psi):
        psi = math.inf
    return psi, g_modes, g_d, g_s


# ----------------------------------------------------------------------------
# Psi and its gradient (eq:Psi with eqn:lmu, eqn:lvr, eq:kappa, eq:prior-k, eq:D)
# ----------------------------------------------------------------------------

def in_domain(prob, d):
    d = np.asarray(d, dtype=np.float64)
    dmax = C_KMS / (3.0 * prob.omega_m * H0)
    return np.isfinite(d) & (d > 0.0) & (d < dmax)


def exact_sum(terms):
    """The sum of the terms rounded once (math.fsum): every sum of the
    Hamiltonian (Psi, dPsi/ds, the kinetic energy) is taken this way, so that
    it does not depend on the order or the number of its terms."""
    return math.fsum(np.asarray(terms, dtype=np.float64).ravel().tolist())


def prior_energy(prob, dhat, u8=1.0):
    """-ln P(Delta_k) up to a constant: sum over independent modes |dhat|^2/sigma^2.

    On the half spectrum: (1/2) sum_k w_k |dhat_k|^2 / sigma_k^2, the energy E
    of the fiducial spectrum.  With P scaled by u8^2 (sigma_8 = u8 sigma_8,fid)
    the Gaussian's normalisation enters: E / u8^2 + D ln u8, D real mode
    coordinates (exactly E at u8 = 1).
    """
    var = mode_variance(prob)
    w = pair_weight(prob.n_grid)
    safe = np.where(var > 0, var, 1.0)
    e = exact_sum(0.5 * w * np.abs(dhat) ** 2 / safe)
    return e / (u8 * u8) + mode_dof(prob.n_grid) * math.log(u8)


def _cosmo(prob, cosmo):
    """(u8, phi, eta) of a state: the fiducial (1, 1, 1) unless the problem
    samples them."""
    if not prob.sample_cosmology or cosmo is None:
        return 1.0, 1.0, 1.0
    return float(cosmo[0]), float(cosmo[1]), float(cosmo[2])


def galaxy_terms(prob, d, s, u, eta=1.0):
    """Per-galaxy pieces of Psi: returns dict of arrays (all FP64); eta =
    h / h_fid."""
    om = prob.omega_m
    zb = zbar(d, om)
    snl = SIGMA_NL_UNIT * s
    kappa2 = snl * snl + prob.sigma_cz ** 2 / (1.0 + zb) ** 2
    dmu = prob.mu - distance_modulus(d, om, prob.h * eta)
    r = v_obs(prob.cz, d, om) - u
    psi = (dmu * dmu / (2.0 * prob.sigma_mu ** 2) + r * r / (2.0 * kappa2)
           + 0.5 * np.log(kappa2) - prob.hist.log_density(d))
    return dict(zbar=zb, kappa2=kappa2, dmu=dmu, r=r, psi=psi)


def logpost(prob, dhat, d, s, cosmo=None):
    """Psi(q) = -ln Pi(q) up to constants (eq:Psi); cosmo = (u8, phi, eta)
    when the problem samples the cosmological parameters."""
    d = np.asarray(d, dtype=np.float64)
    u8, phi, eta = _cosmo(prob, cosmo)
    if not np.all(in_domain(prob, d)) or not (u8 > 0.0 and phi > 0.0 and eta > 0.0):
        return math.inf
    v = velocity_grids(prob, dhat, phi)
    u, _ = cic_gather(prob, v, d)
    terms = galaxy_terms(prob, d, s, u, eta)
    total = exact_sum(np.concatenate([[prior_energy(prob, dhat, u8)], terms["psi"]]))
    return total if np.isfinite(total) else math.inf


def logpost_grad(prob, dhat, d, s, cosmo=None):
    """Psi(q) and its analytic gradient.

    Returns (psi, g_modes, g_d, g_s) where g_modes is on the half spectrum in
    the complex convention G_k = dPsi/dRe dhat_k + i dPsi/dIm dhat_k, taken
    with respect to the independent coordinates of each mode (on the kz = 0
    plane the stored partner carries the conjugate).  When the problem
    samples the cosmological parameters, cosmo = (u8, phi, eta) and a fifth
    entry (dPsi/du8, dPsi/dphi, dPsi/deta) follows:
        dPsi/du8 = -2 E / u8^3 + D / u8      (the prior; E at u8 = 1)
        dPsi/dphi = sum_i g_i u_i / phi      (u_i is linear in phi)
        dPsi/deta = sum_i (dmu_i / sigma_mu,i^2) 5 / (eta ln 10)
                                             (mu_i(d) moves by -5 log10 eta)
    """
    n = prob.n_grid
    d = np.asarray(d, dtype=np.float64)
    ok = in_domain(prob, d)
    dsafe = np.where(ok, d, 1.0)
    u8, phi, eta = _cosmo(prob, cosmo)
    v = velocity_grids(prob, dhat, phi)
    u, du = cic_gather(prob, v, dsafe)
    t = galaxy_terms(prob, dsafe, s, u, eta if eta > 0.0 else 1.0)
    om = prob.omega_m
    kappa2, r = t["kappa2"], t["r"]
    zb = t["zbar"]
    # dPsi/du_i = -r_i / kappa_i^2 (eqn:lvr)
    g = -r / kappa2
    # dPsi/d kappa_i^2
    dk2 = 0.5 / kappa2 - 0.5 * r * r / kappa2 ** 2
    dkappa2_dd = -2.0 * prob.sigma_cz ** 2 * zbar_prime(dsafe, om) / (1.0 + zb) ** 3
    g_d = (-t["dmu"] * distance_modulus_prime(dsafe, om) / prob.sigma_mu ** 2
           + (r / kappa2) * (v_obs_prime(prob.cz, dsafe, om) - du)
           + dk2 * dkappa2_dd)
    g_s = exact_sum(dk2 * 2.0 * SIGMA_NL_UNIT ** 2 * s)
    # Modes: prior term 2 dhat / sigma^2 plus the adjoint of the projected
    # gather through the inverse transform: (2/N^3) sum_c conj(m_c) FFT(G_c).
    var = mode_variance(prob)
    safe = np.where(var > 0, var, 1.0)
    g_modes = np.where(var > 0, 2.0 * dhat / (u8 * u8 * safe), 0.0).astype(np.complex128)
    g_modes += modes_adjoint(prob, dsafe, g, phi)
    good = np.all(ok) and u8 > 0.0 and phi > 0.0 and eta > 0.0
    psi = exact_sum(np.concatenate([[prior_energy(prob, dhat, u8)], t["psi"]])) if good else math.inf
    if not (good and np.isfinite(psi)):
        psi = math.inf
    if cosmo is None or not prob.sample_cosmology:
        return psi, g_modes, g_d, g_s
    e = prior_energy(prob, dhat)
    g_u8 = -2.0 * e / u8 ** 3 + mode_dof(n) / u8
    g_phi = exact_sum(g * u) / phi
    g_eta = exact_sum(t["dmu"] / prob.sigma_mu ** 2) * 5.0 / (eta * math.log(10.0))
    return psi, g_modes, g_d, g_s, np.array([g_u8, g_phi, g_eta])
