"""Pins of the cosmological coordinates of the oracle (Section 6, item 3:
H0, sigma_8 and the growth rate estimated with the field): u8 = sigma_8 /
sigma_8,fid scales P(k) by u8^2, phi = f / f_fid scales the velocity field,
eta = h / h_fid sets the zero point of the distance moduli.

The prior with u8 must be the normalised Gaussian of variance u8^2 sigma_k^2
(checked against scipy's normal log-density, term for term); the velocity
field must be linear in the growth rate and obey linear continuity with the
scaled f; Psi at eta must equal Psi at the fiducial h with every observed
distance modulus moved by +5 log10 eta (the luminosity distance in Mpc is
d_L / h); the gradient in (u8, phi, eta) against central differences (Psi is
smooth in all three), the mode gradient away from the fiducial point against
exact central differences; the leapfrog with the new coordinates reversible.
"""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import hmc, model
from paper_2203_02369_amd import mocks


def _problem(n_grid=8, box=160.0, n_gal=60, **kw):
    m = mocks.make_mock(n_grid, box, n_gal, 60.0, "sphere", (0.2, 0.2), seed=3)
    args = m.problem_kwargs()
    args.update(sample_cosmology=True, **kw)
    return m, model.Problem(**args)


def test_sigma8_prior_is_the_normalised_gaussian():
    m, prob = _problem()
    n = prob.n_grid
    rng = np.random.default_rng(1)
    var = model.mode_variance(prob)
    dhat = hmc.symmetrise(n, np.sqrt(0.5 * var) * (rng.standard_normal(var.shape) + 1j * rng.standard_normal(var.shape)))
    x = hmc.pack_modes(n, dhat)                       # independent real coordinates
    v = hmc.pack_modes(n, (0.5 * var).astype(complex))
    v = np.concatenate([v[: len(v) // 2], v[: len(v) // 2]])   # variance of each real coordinate at u8 = 1
    ref1 = stats.norm.logpdf(x, scale=np.sqrt(v)).sum()
    for u8 in (0.6, 0.93, 1.4):
        refu = stats.norm.logpdf(x, scale=u8 * np.sqrt(v)).sum()
        got = model.prior_energy(prob, dhat, u8) - model.prior_energy(prob, dhat, 1.0)
        assert abs(got - (ref1 - refu)) <= 1e-9 * abs(ref1), (u8, got, ref1 - refu)


def test_growth_rate_scales_the_velocity_field():
    m, prob = _problem()
    n = prob.n_grid
    dhat = hmc.symmetrise(n, m.dhat_true)
    phi = 1.37
    v1 = model.velocity_grids(prob, dhat)
    vp = model.velocity_grids(prob, dhat, phi)
    assert np.abs(vp - phi * v1).max() <= 1e-13 * np.abs(v1).max() * phi
    # linear continuity with the scaled growth rate: -div v / H0 = phi f delta
    kf = 2 * math.pi / prob.box
    k = kf * np.fft.fftfreq(n, d=1.0 / n)
    div = sum(np.fft.ifftn(1j * kk * np.fft.fftn(vp[a])).real
              for a, kk in enumerate((k[:, None, None], k[None, :, None], k[None, None, :])))
    delta = model.density_grid(prob, dhat)
    assert np.allclose(-div / model.H0, phi * prob.f_growth * delta, atol=1e-9 * np.abs(delta).max())


def test_hubble_parameter_moves_the_distance_modulus_zero_point():
    m, prob = _problem()
    n = prob.n_grid
    dhat = hmc.symmetrise(n, m.dhat_true)
    d = m.d_true.copy()
    s = 1.3
    for eta in (0.93, 1.0, 1.08):
        got = model.logpost(prob, dhat, d, s, cosmo=np.array([1.0, 1.0, eta]))
        # the same universe measured with h = eta h_fid: d_L / h in Mpc, so
        # the predicted modulus drops by 5 log10 eta; equivalently every
        # observed modulus rises by as much at the fiducial h
        args = m.problem_kwargs()
        args.update(sample_cosmology=True, mu=np.asarray(prob.mu) + 5.0 * math.log10(eta))
        ref = model.logpost(model.Problem(**args), dhat, d, s, cosmo=np.array([1.0, 1.0, 1.0]))
        assert abs(got - ref) <= 1e-12 * abs(ref), (eta, got, ref)
    # a smaller h puts every point farther in Mpc: with the moduli of the mock
    # (drawn at h_fid) the fit is best near eta = 1
    psis = [model.logpost(prob, dhat, d, s, cosmo=np.array([1.0, 1.0, e])) for e in (0.8, 1.0, 1.25)]
    assert psis[1] < psis[0] and psis[1] < psis[2]


@pytest.mark.parametrize("cosmo", [(1.0, 1.0, 1.0), (0.9, 1.2, 0.95)])
def test_cosmology_gradient_central_differences(cosmo):
    m, prob = _problem()
    n = prob.n_grid
    dhat = hmc.symmetrise(n, m.dhat_true)
    rng = np.random.default_rng(4)
    d = m.d_true * (1.0 + 0.02 * rng.standard_normal(prob.n_gal))
    s = 1.3
    c = np.array(cosmo)
    psi, gm, gd, gs, gc = model.logpost_grad(prob, dhat, d, s, cosmo=c)
    assert psi == model.logpost(prob, dhat, d, s, cosmo=c)
    for a in range(3):
        h = 1e-5 * c[a]
        cp, cm = c.copy(), c.copy()
        cp[a] += h
        cm[a] -= h
        fd = (model.logpost(prob, dhat, d, s, cosmo=cp) - model.logpost(prob, dhat, d, s, cosmo=cm)) / (2 * h)
        assert abs(fd - gc[a]) <= 1e-6 * max(abs(gc[a]), 1.0), (a, fd, gc[a])
    # the mode gradient at this (u8, phi): Psi is quadratic in one mode
    # coordinate, so the central difference is exact up to rounding
    x = hmc.pack_modes(n, dhat)
    g_flat = hmc.pack_modes(n, gm)
    for j in rng.choice(len(x), 6, replace=False):
        h = 0.3 * abs(x[j]) + 1.0
        xp, xm = x.copy(), x.copy()
        xp[j] += h
        xm[j] -= h
        fd = (model.logpost(prob, hmc.unpack_modes(n, xp), d, s, cosmo=c)
              - model.logpost(prob, hmc.unpack_modes(n, xm), d, s, cosmo=c)) / (2 * h)
        assert abs(fd - g_flat[j]) <= 1e-6 * np.abs(g_flat).max(), (j, fd, g_flat[j])
    # outside (0, inf)^3 the posterior vanishes
    assert model.logpost(prob, dhat, d, s, cosmo=np.array([-0.1, 1.0, 1.0])) == math.inf
    assert model.logpost(prob, dhat, d, s, cosmo=np.array([1.0, 0.0, 1.0])) == math.inf
    assert model.logpost(prob, dhat, d, s, cosmo=np.array([1.0, 1.0, -0.5])) == math.inf


def test_leapfrog_with_cosmology_is_reversible():
    m, prob = _problem()
    n = prob.n_grid
    q0 = hmc.State(hmc.symmetrise(n, m.dhat_true), m.d_true.copy(), 1.2, np.array([1.05, 0.95, 1.02]))
    p0 = hmc.draw_momenta(prob, 9, 0)
    assert p0.cosmo is not None and p0.cosmo.shape == (3,)
    q1, p1, _ = hmc.leapfrog(prob, q0, p0, 0.05, 12)
    assert np.abs(q1.cosmo - q0.cosmo).max() > 1e-4          # the new coordinates moved
    back = hmc.State(p1.modes * -1, -p1.dist, -p1.s, -p1.cosmo)
    q2, p2, _ = hmc.leapfrog(prob, q1, back, 0.05, 12)
    assert np.abs(q2.cosmo - q0.cosmo).max() <= 1e-10
    assert np.abs(q2.modes - q0.modes).max() <= 1e-10 * np.abs(q0.modes).max()
    # the kinetic energy carries the new momenta with their masses
    kin = hmc.kinetic(prob, p0)
    p0c = p0.copy()
    p0c.cosmo = np.zeros(3)
    assert abs(kin - hmc.kinetic(prob, p0c) - 0.5 * float(np.sum(hmc.cosmo_inverse_mass(prob) * p0.cosmo ** 2))) \
        <= 1e-12 * kin
