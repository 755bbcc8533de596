"""Seeded synthetic inputs: Lambda-CDM power spectrum and mock catalogues.

This module is the only code shared by the GPU library's callers and the
test oracle, and it holds none of the reconstruction's arithmetic: it draws
inputs.  Its "mock universe" (a linear Gaussian random field, its linear
velocities sampled at the galaxies, the observed distance moduli and
redshifts) is a simulation of the observations, written here on its own
with numpy's FFT; neither the oracle nor the GPU path calls into it for
their own results.

Mock recipe (Section 5.1 of the paper, with the shapes and error levels of
the synthetic configurations standing in for the Cosmicflows-3 errors that
are not available):
  * Field: BBKS transfer function (Gamma = Omega_m h, n_s = 1), normalised to
    sigma_8 with a top-hat of radius 8 Mpc/h; a Gaussian random field on the
    periodic N^3 grid of side L, modes with a Nyquist index and k = 0 zeroed.
  * Observer at the box centre, supergalactic axes along the grid axes.
  * Points: isotropic directions; radii uniform in a sphere (r = R u^(1/3)),
    or with number density proportional to 1/r (r = sqrt(rmin^2 + (R^2 -
    rmin^2) u)); an optional zone of avoidance |b| < b_min is redrawn.
  * Errors: a fractional lognormal distance error sigma_lnd per point, so
    sigma_mu = 5 sigma_lnd / ln 10; sigma_cz = 50 km/s.
  * Observed mu = mu(d) + sigma_mu xi and cz = c zbar(d) + v (1 + zbar(d)) +
    sigma_cz xi', with v the linear radial velocity of the field at the point.
"""
import dataclasses
import math
from dataclasses import dataclass

import numpy as np

C_KMS = 299792.458
H100 = 100.0
SEED_BASE = 2203_02369


# ----------------------------------------------------------------------------
# Power spectrum
# ----------------------------------------------------------------------------

def bbks_transfer(k, omega_m, h):
    """BBKS (Bardeen et al. 1986) transfer function; k in h/Mpc."""
    q = np.asarray(k, dtype=np.float64) / (omega_m * h)
    q = np.where(q > 0, q, 1e-30)
    poly = 1.0 + 3.89 * q + (16.1 * q) ** 2 + (5.46 * q) ** 3 + (6.71 * q) ** 4
    return np.log(1.0 + 2.34 * q) / (2.34 * q) * poly ** -0.25


def _tophat(x):
    x = np.asarray(x, dtype=np.float64)
    small = x < 1e-4
    xs = np.where(small, 1.0, x)
    w = 3.0 * (np.sin(xs) - xs * np.cos(xs)) / xs ** 3
    return np.where(small, 1.0 - x * x / 10.0, w)


@dataclass
class PowerSpectrum:
    """P(k) = A k^n_s T_BBKS(k)^2 in (Mpc/h)^3, normalised to sigma_8."""
    omega_m: float = 0.3
    h: float = 0.7
    sigma8: float = 0.8
    n_s: float = 1.0

    def __post_init__(self):
        lk = np.linspace(math.log(1e-5), math.log(1e3), 40001)
        k = np.exp(lk)
        shape = k ** self.n_s * bbks_transfer(k, self.omega_m, self.h) ** 2
        integrand = k ** 3 * shape * _tophat(8.0 * k) ** 2 / (2.0 * math.pi ** 2)
        s8sq = np.trapezoid(integrand, lk)
        self.amp = self.sigma8 ** 2 / s8sq

    def __call__(self, k):
        k = np.asarray(k, dtype=np.float64)
        pk = self.amp * np.where(k > 0, k, 1.0) ** self.n_s * bbks_transfer(k, self.omega_m, self.h) ** 2
        return np.where(k > 0, pk, 0.0)

    def table_n2(self, n_grid, box):
        """P at |k| = (2 pi / L) sqrt(j), j = 0 .. 3 (N/2)^2."""
        j = np.arange(3 * (n_grid // 2) ** 2 + 1, dtype=np.float64)
        return self(2.0 * math.pi / box * np.sqrt(j))


# ----------------------------------------------------------------------------
# Mock catalogue
# ----------------------------------------------------------------------------

@dataclass
class Mock:
    """A synthetic reconstruction problem (grid, cosmology, catalogue).

    rhat[i] = (cos b cos l, cos b sin l, sin b), l = sgl, b = sgb (degrees).
    dhat_true is the mock field's half spectrum (N, N, N/2+1), unnormalised
    forward-transform convention; d_true the true distances; d_init a
    starting guess from the observed distance modulus.
    """
    n_grid: int
    box: float
    omega_m: float
    h: float
    f_growth: float
    sigma_v: float
    pk_n2: np.ndarray
    hist_width: float
    sgl: np.ndarray
    sgb: np.ndarray
    rhat: np.ndarray
    mu: np.ndarray
    sigma_mu: np.ndarray
    cz: np.ndarray
    sigma_cz: np.ndarray
    d_true: np.ndarray
    d_init: np.ndarray
    dhat_true: np.ndarray
    vr_true: np.ndarray

    @property
    def n_gal(self):
        return len(self.mu)

    def problem_kwargs(self):
        """Keyword arguments describing the problem (shared by both sides)."""
        return dict(n_grid=self.n_grid, box=self.box, omega_m=self.omega_m, h=self.h,
                    f_growth=self.f_growth, sigma_v=self.sigma_v, pk_n2=self.pk_n2,
                    rhat=self.rhat, mu=self.mu, sigma_mu=self.sigma_mu, cz=self.cz,
                    sigma_cz=self.sigma_cz, hist_width=self.hist_width)


def _gaussian_field(rng, n_grid, box, pk):
    """Half spectrum of a Gaussian random field with <|dhat|^2> = N^6 P / V."""
    white = rng.standard_normal((n_grid, n_grid, n_grid))
    wk = np.fft.rfftn(white)
    kf = 2.0 * math.pi / box
    f = np.fft.fftfreq(n_grid, d=1.0 / n_grid)
    fz = np.arange(n_grid // 2 + 1)
    kx, ky, kz = np.meshgrid(f, f, fz, indexing="ij")
    kmag = kf * np.sqrt(kx * kx + ky * ky + kz * kz)
    amp = np.sqrt(n_grid ** 3 * pk(kmag) / box ** 3)
    dhat = wk * amp
    half = n_grid // 2
    bad = (np.abs(kx) == half) | (np.abs(ky) == half) | (kz == half) | (kmag == 0)
    dhat[bad] = 0.0
    return hermitian_half(dhat), (kx, ky, kz)


def hermitian_half(dhat):
    """Make the kz = 0 plane of a half spectrum exactly Hermitian.

    The entry (kx, ky, 0) with ky < N/2 taken as signed ky < 0, or ky = 0 and
    kx past N/2, is set to the conjugate of its partner (-kx, -ky, 0).
    """
    out = np.array(dhat, dtype=np.complex128, copy=True)
    n = out.shape[0]
    f = np.fft.fftfreq(n, d=1.0 / n).astype(np.int64)
    plane = out[:, :, 0]
    neg = (-np.arange(n)) % n
    partner = np.conj(plane[np.ix_(neg, neg)])
    mirror = (f[None, :] < 0) | ((f[None, :] == 0) & (f[:, None] < 0))
    plane[mirror] = partner[mirror]
    out[:, :, 0] = plane
    return out


def _linear_velocity(dhat, kvec, n_grid, box, f_growth):
    """The mock field's linear velocity grids (3, N, N, N) via numpy's FFT."""
    kf = 2.0 * math.pi / box
    kx, ky, kz = [kf * c for c in kvec]
    k2 = kx * kx + ky * ky + kz * kz
    k2 = np.where(k2 > 0, k2, 1.0)
    out = []
    for kc in (kx, ky, kz):
        vk = 1j * H100 * f_growth * kc / k2 * dhat
        out.append(np.fft.irfftn(vk, s=(n_grid,) * 3, axes=(0, 1, 2)))
    return np.stack(out)


def _trilinear(grids, pos, box, n_grid):
    d = box / n_grid
    s = pos / d
    i0 = np.floor(s).astype(np.int64)
    t = s - i0
    out = np.zeros((pos.shape[0], grids.shape[0]))
    for ox in (0, 1):
        for oy in (0, 1):
            for oz in (0, 1):
                w = ((t[:, 0] if ox else 1 - t[:, 0]) * (t[:, 1] if oy else 1 - t[:, 1])
                     * (t[:, 2] if oz else 1 - t[:, 2]))
                ix = (i0 + np.array([ox, oy, oz])) % n_grid
                out += w[:, None] * grids[:, ix[:, 0], ix[:, 1], ix[:, 2]].T
    return out


def _zbar(d, om):
    return (2.0 / (3.0 * om)) * (1.0 - np.sqrt(1.0 - 3.0 * om * H100 * d / C_KMS))


def make_mock(n_grid, box, n_gal, radius, radial="sphere", sigma_lnd=(0.2, 0.2),
              sigma_cz=50.0, zoa_deg=0.0, rmin=5.0, seed=0, omega_m=0.3, h=0.7,
              sigma8=0.8, hist_width=5.0):
    """Draw one mock problem.  radial: 'sphere' (uniform) or 'inv_r' (n ~ 1/r)."""
    rng_field = np.random.default_rng(seed)
    rng_cat = np.random.default_rng(seed + 1)
    pk = PowerSpectrum(omega_m=omega_m, h=h, sigma8=sigma8)
    f_growth = omega_m ** 0.55
    dhat, kvec = _gaussian_field(rng_field, n_grid, box, pk)
    vgrid = _linear_velocity(dhat, kvec, n_grid, box, f_growth)
    sigma_v = float(np.sqrt(np.mean(vgrid ** 2)))

    sgl, sgb, r = [], [], []
    have = 0
    while have < n_gal:
        m = 2 * (n_gal - have) + 16
        l = rng_cat.uniform(0.0, 360.0, m)
        b = np.degrees(np.arcsin(rng_cat.uniform(-1.0, 1.0, m)))
        u = rng_cat.uniform(0.0, 1.0, m)
        if radial == "sphere":
            rr = radius * u ** (1.0 / 3.0)
        elif radial == "inv_r":
            rr = np.sqrt(rmin ** 2 + (radius ** 2 - rmin ** 2) * u)
        else:
            raise ValueError(radial)
        keep = (np.abs(b) >= zoa_deg) & (rr > 0.5)
        sgl.append(l[keep]); sgb.append(b[keep]); r.append(rr[keep])
        have += int(keep.sum())
    sgl = np.concatenate(sgl)[:n_gal]
    sgb = np.concatenate(sgb)[:n_gal]
    d_true = np.concatenate(r)[:n_gal]
    lr, br = np.radians(sgl), np.radians(sgb)
    rhat = np.stack([np.cos(br) * np.cos(lr), np.cos(br) * np.sin(lr), np.sin(br)], axis=1)

    pos = 0.5 * box + d_true[:, None] * rhat
    vr = (_trilinear(vgrid, pos, box, n_grid) * rhat).sum(axis=1)

    lo, hi = sigma_lnd
    slnd = rng_cat.uniform(lo, hi, n_gal) if hi > lo else np.full(n_gal, lo)
    sigma_mu = 5.0 * slnd / math.log(10.0)
    zb = _zbar(d_true, omega_m)
    mu_true = 5.0 * np.log10(d_true * (1.0 + zb) / h) + 25.0
    mu = mu_true + sigma_mu * rng_cat.standard_normal(n_gal)
    scz = np.full(n_gal, float(sigma_cz))
    cz = C_KMS * zb + vr * (1.0 + zb) + scz * rng_cat.standard_normal(n_gal)
    d_init = np.clip(10.0 ** ((mu - 25.0) / 5.0) * h, 1.0, 1.8 * radius)
    return Mock(n_grid=n_grid, box=float(box), omega_m=omega_m, h=h, f_growth=f_growth,
                sigma_v=sigma_v, pk_n2=pk.table_n2(n_grid, box), hist_width=hist_width,
                sgl=sgl, sgb=sgb, rhat=rhat, mu=mu, sigma_mu=sigma_mu, cz=cz,
                sigma_cz=scz, d_true=d_true, d_init=d_init, dhat_true=dhat, vr_true=vr)


# ----------------------------------------------------------------------------
# The synthetic workloads
# ----------------------------------------------------------------------------

def config_seed(k):
    return SEED_BASE + 10 * k


def plain_fp64_32():
    """32^3, L = 400, 1000 points uniform in a sphere of 120 Mpc/h, 20 %."""
    return make_mock(32, 400.0, 1000, 120.0, "sphere", (0.20, 0.20), seed=config_seed(1))


def single_chain_128():
    """128^3, L = 500, 10 000 points with n ~ 1/r to 200 Mpc/h, 20-25 %."""
    return make_mock(128, 500.0, 10000, 200.0, "inv_r", (0.20, 0.25), seed=config_seed(2))


def paper_scale_256(n_gal=30000, n_grid=256, seed=None):
    """256^3, L = 500, 30 000 points, n ~ 1/r to 250 Mpc/h, ZoA |b| < 10 deg."""
    return make_mock(n_grid, 500.0, n_gal, 250.0, "inv_r", (0.15, 0.25), zoa_deg=10.0,
                     seed=config_seed(3) if seed is None else seed)


def refine(mock, n_grid):
    """The same universe and catalogue on a finer grid of n_grid^3: the
    field's modes carried over (times (n_grid / N)^3, the unnormalised
    transform), the modes the coarse grid cannot hold left at zero, P(k)
    tabulated for the finer grid."""
    n0 = mock.n_grid
    if n_grid < n0 or n_grid % n0:
        raise ValueError("n_grid must be a multiple of %d" % n0)
    s = np.where(np.arange(n0) < n0 // 2, np.arange(n0), np.arange(n0) - n0)
    fine = np.where(s < 0, s + n_grid, s)
    dh = np.zeros((n_grid, n_grid, n_grid // 2 + 1), dtype=np.complex128)
    dh[np.ix_(fine, fine, np.arange(n0 // 2))] = (n_grid / n0) ** 3 * mock.dhat_true[:, :, : n0 // 2]
    pk = PowerSpectrum(omega_m=mock.omega_m, h=mock.h).table_n2(n_grid, mock.box)
    return dataclasses.replace(mock, n_grid=n_grid, pk_n2=pk, dhat_true=dh)


def batched_16_sizes():
    """(N, n) of the 16 independent chains of the batched workload: grids
    64^3, 128^3, 256^3 in turn, catalogues from 2000 to 30 000 points."""
    grids = (64, 128, 256)
    return [(grids[j % 3], 2000 + (28000 * j) // 15) for j in range(16)]


def batched_16():
    """16 mock problems of uneven size (box 500 Mpc/h, n ~ 1/r to 200 Mpc/h,
    20-25 % distance errors, one seed each)."""
    return [make_mock(ng, 500.0, n, 200.0, "inv_r", (0.20, 0.25), seed=config_seed(4) + j)
            for j, (ng, n) in enumerate(batched_16_sizes())]


def small_case(n_grid=16, box=200.0, n_gal=300, radius=80.0, seed=7):
    """A tiny problem for oracle-only pins."""
    return make_mock(n_grid, box, n_gal, radius, "sphere", (0.2, 0.2), seed=seed)
