"""Pins of the oracle posterior (Section 2) against closed forms and brute force."""
import math

import numpy as np
import pytest

from oracle import hmc, model
from paper_2203_02369_amd import mocks


def _problem(n_grid=8, box=200.0, n_gal=60, radius=80.0, seed=3, **kw):
    m = mocks.make_mock(n_grid, box, n_gal, radius, "sphere", (0.2, 0.2), seed=seed)
    kwargs = m.problem_kwargs()
    kwargs.update(kw)
    return m, model.Problem(**kwargs)


def _empty_problem(n_grid=8, box=200.0):
    m = mocks.make_mock(n_grid, box, 1, 50.0, seed=1)
    kw = m.problem_kwargs()
    for key in ("mu", "sigma_mu", "cz", "sigma_cz"):
        kw[key] = np.zeros(0)
    kw["rhat"] = np.zeros((0, 3))
    return model.Problem(**kw)


# ---------------------------------------------------------------- cosmology --

def test_zbar_solves_its_quadratic():
    # zbar(d) = (2/3Om)(1 - sqrt(1 - 3 Om H0 d / c)) is the root of
    # (3 Om / 4) z^2 - z + H0 d / c = 0 that vanishes at d = 0.
    for om in (0.3, 1.0):
        d = np.linspace(0.1, 0.99 * model.C_KMS / (3 * om * model.H0), 50)
        z = model.zbar(d, om)
        resid = 0.75 * om * z * z - z + model.H0 * d / model.C_KMS
        assert np.abs(resid).max() < 1e-14
    # low-distance limit: Hubble law
    z1 = model.H0 * 1e-3 / model.C_KMS
    assert abs(model.zbar(1e-3, 0.3) - z1) < 1e-6 * z1


def test_distance_modulus_of_ten_parsec_is_zero():
    h = 0.7
    # d (1 + zbar(d)) / h = 1e-5 Mpc  <=>  mu = 0; zbar is ~1e-9 there.
    d = 1e-5 * h
    for _ in range(5):
        d = 1e-5 * h / (1.0 + model.zbar(d, 0.3))
    assert abs(model.distance_modulus(d, 0.3, h)) < 1e-12
    # one decade in distance is 5 magnitudes (up to the (1 + zbar) factor,
    # here ~3e-9)
    d1, d2 = 1e-6, 1e-5
    dmu = model.distance_modulus(d2, 0.3, h) - model.distance_modulus(d1, 0.3, h)
    assert abs(dmu - 5.0) < 1e-7


def test_vobs_inverts_the_redshift_composition():
    # (1 + z) = (1 + zbar)(1 + v/c) is the relation eq:vrobs inverts.
    d = np.array([10.0, 100.0, 250.0])
    v = np.array([-300.0, 0.0, 750.0])
    zb = model.zbar(d, 0.3)
    cz = model.C_KMS * ((1.0 + zb) * (1.0 + v / model.C_KMS) - 1.0)
    assert np.abs(model.v_obs(cz, d, 0.3) - v).max() < 1e-9


@pytest.mark.parametrize("z", [0.001, 0.05, 0.2])
def test_redshift_distance_closed_forms(z):
    # Om = 1 (Einstein-de Sitter): d_z = (2c/H0)(1 - 1/sqrt(1+z)).
    eds = 2.0 * model.C_KMS / model.H0 * (1.0 - 1.0 / math.sqrt(1.0 + z))
    assert abs(model.redshift_distance(z, 1.0)[0] - eds) < 1e-9 * eds
    # Om = 0: the integrand is 1, d_z = c z / H0 exactly.
    assert abs(model.redshift_distance(z, 0.0)[0] - model.C_KMS * z / model.H0) < 1e-9


def test_histogram_is_a_density_with_pseudocounts():
    m, prob = _problem(n_gal=200)
    hist = prob.hist
    assert abs(np.sum(hist.density) * hist.width - 1.0) < 1e-12
    assert np.all(hist.density > 0)
    # zero outside the support: -ln N = +inf
    top = len(hist.density) * hist.width
    ld = hist.log_density(np.array([-1.0, 0.0, top - 1e-9, top, np.nan]))
    assert np.isinf(ld[0]) and np.isfinite(ld[1]) and np.isfinite(ld[2])
    assert np.isinf(ld[3]) and np.isinf(ld[4])


# ------------------------------------------------------------ mode bookkeeping

@pytest.mark.parametrize("n", [4, 8, 16])
def test_retained_degrees_of_freedom(n):
    # every mode without a Nyquist index, minus k = 0, counted in real d.o.f.
    assert 2 * int(hmc.canonical_mask(n).sum()) == (n - 1) ** 3 - 1
    w = model.pair_weight(n)
    assert int(w.sum()) == (n - 1) ** 3 - 1


def _pk_problem(n_grid, box, pk_of_n2):
    """An empty-catalogue problem whose P(k) table is pk_of_n2(j), j = |n|^2."""
    prob = _empty_problem(n_grid=n_grid, box=box)
    j = np.arange(3 * (n_grid // 2) ** 2 + 1, dtype=np.float64)
    prob.pk_n2 = pk_of_n2(j)
    return prob


@pytest.mark.parametrize("kvec", [(1, 0, 2), (3, -2, 1), (2, 1, 0), (0, -3, 0)])
def test_mode_variance_single_mode_closed_form(kvec):
    # eq:prior-k with P the variance of the complex mode (reading of the
    # normalisation): a field with the one mode pair +-k at amplitude
    # |dhat_k| = sigma_k is 2 sigma_k/N^3 cos(k.x) on the nodes, whose mean
    # square over the box is 2 sigma_k^2 / N^6.  The continuum gives the same
    # pair 2 P(|k|) / V (the variance of delta is V^-1 sum_k P(|k|)), so the
    # node mean of delta^2 must equal 2 P(|k|) / V exactly: this fixes the
    # powers of N and of the box in sigma_k^2 = N^6 P / V.
    n, box = 16, 300.0
    prob = _pk_problem(n, box, lambda j: 1e3 * (1.0 + j) ** -1.3)
    var = model.mode_variance(prob)
    kx, ky, kz = kvec
    dhat = np.zeros(model.half_shape(n), dtype=np.complex128)
    dhat[kx % n, ky % n, kz] = math.sqrt(var[kx % n, ky % n, kz])
    if kz == 0:
        # both members of the pair are stored on the kz = 0 plane (real value)
        dhat[-kx % n, -ky % n, 0] = dhat[kx % n, ky % n, 0]
    assert np.array_equal(hmc.symmetrise(n, dhat), dhat)
    delta = model.density_grid(prob, dhat)
    pk = prob.pk_n2[kx * kx + ky * ky + kz * kz]
    expect = 2.0 * pk / box ** 3
    assert abs(float(np.mean(delta ** 2)) - expect) <= 1e-12 * expect
    # the real-space amplitude of the cosine itself
    assert abs(float(np.abs(delta).max()) - 2.0 * math.sqrt(var[kx % n, ky % n, kz]) / n ** 3) <= 1e-12 * expect ** 0.5


@pytest.mark.parametrize("shape", ["flat", "bbks"])
def test_mode_variance_field_variance(shape):
    # Fields drawn with <|dhat_k|^2> = sigma_k^2 (complex Gaussian per
    # independent mode, Hermitian partners mirrored) must have
    # <delta(x)^2> = V^-1 sum_k P(|k|) over the retained modes of the whole
    # spectrum: the discrete form of the variance integral of P(k).  The node
    # and draw mean of delta^2 is compared with it; its relative standard
    # deviation is (sum_pairs sigma^4)^(1/2) / sum_pairs sigma^2 / sqrt(draws),
    # and the bound is 5 of those.
    n, box, draws = 16, 200.0, 40
    if shape == "flat":
        prob = _pk_problem(n, box, lambda j: np.full(j.shape, 2.5e3))
    else:
        m = mocks.make_mock(n, box, 1, 50.0, seed=1)
        prob = _pk_problem(n, box, lambda j: np.asarray(m.pk_n2, dtype=np.float64))
    var = model.mode_variance(prob)
    canon = hmc.canonical_mask(n)
    nx, ny, nz = model.mode_indices(n)
    n2 = nx * nx + ny * ny + nz * nz
    # every retained mode of the full N^3 spectrum is a stored canonical
    # entry or the partner -k of one: 2 per canonical entry
    expect = 2.0 * float(np.sum(prob.pk_n2[n2][canon])) / box ** 3
    rng = np.random.default_rng(2203)
    acc = 0.0
    for _ in range(draws):
        z = rng.standard_normal(var.shape) + 1j * rng.standard_normal(var.shape)
        dhat = hmc.symmetrise(n, np.sqrt(0.5 * var) * z)
        acc += float(np.mean(model.density_grid(prob, dhat) ** 2))
    got = acc / draws
    s2 = var[canon]
    rel_sd = math.sqrt(float(np.sum(s2 * s2))) / float(np.sum(s2)) / math.sqrt(draws)
    assert abs(got / expect - 1.0) <= 5.0 * rel_sd, (got, expect, rel_sd)
    # a factor of two in the normalisation (the variance of the real part read
    # as P, or N^3 for N^6 / V) lies far outside this bound
    assert 5.0 * rel_sd < 0.1


def test_pack_unpack_roundtrip_is_hermitian():
    n = 8
    rng = np.random.default_rng(2)
    ndof = (n - 1) ** 3 - 1
    v = rng.standard_normal(ndof)
    dhat = hmc.unpack_modes(n, v)
    assert np.allclose(hmc.pack_modes(n, dhat), v)
    full = model.full_spectrum(dhat)
    from oracle.fft import ifftn_unnormalised
    field = ifftn_unnormalised(full)
    assert np.abs(field.imag).max() < 1e-12 * np.abs(field.real).max()


# --------------------------------------------------------------- the field --

@pytest.mark.parametrize("kvec", [(1, 2, 3), (2, -1, 0), (0, 0, 1), (-3, 1, 2)])
def test_single_mode_velocity_closed_form(kvec):
    # delta(x) = A cos(k0 . x)  =>  v(x) = -H0 f A k0 sin(k0 . x) / k0^2.
    m, prob = _problem(n_grid=8)
    n, box, amp = prob.n_grid, prob.box, 0.7
    dhat = np.zeros(model.half_shape(n), dtype=np.complex128)
    nx, ny, nz = kvec
    dhat[nx % n, ny % n, nz] = amp * n ** 3 / 2.0
    if nz == 0:
        dhat[(-nx) % n, (-ny) % n, 0] = amp * n ** 3 / 2.0
    v = model.velocity_grids(prob, dhat)
    k0 = 2.0 * math.pi / box * np.array(kvec, dtype=np.float64)
    j = np.arange(n) * box / n
    X, Y, Z = np.meshgrid(j, j, j, indexing="ij")
    phase = k0[0] * X + k0[1] * Y + k0[2] * Z
    for c in range(3):
        exact = -model.H0 * prob.f_growth * amp * k0[c] / np.dot(k0, k0) * np.sin(phase)
        assert np.abs(v[c] - exact).max() < 1e-12 * model.H0 * amp * 100


def test_divergence_identity_per_mode():
    # i k . vhat = -H0 f dhat on every retained mode (linear continuity).
    m, prob = _problem(n_grid=8)
    mult = model.velocity_multiplier(prob)
    kf = 2 * math.pi / prob.box
    nx, ny, nz = model.mode_indices(prob.n_grid)
    kdotm = 1j * kf * (nx * mult[0] + ny * mult[1] + nz * mult[2])
    keep = model.retained_mask(prob.n_grid)
    assert np.allclose(kdotm[keep], -model.H0 * prob.f_growth)
    assert np.all(mult[:, ~keep] == 0)


def test_density_grid_is_the_direct_mode_sum():
    # delta(x_j) = N^-3 sum_k dhat_k e^{i k.x_j}, summed directly over all N^3
    # modes (the half spectrum's mirror entries conjugated) on an 8^3 grid
    m, prob = _problem(n_grid=8, box=80.0)
    n = prob.n_grid
    rng = np.random.default_rng(2)
    shape = model.half_shape(n)
    dhat = hmc.symmetrise(n, rng.standard_normal(shape) + 1j * rng.standard_normal(shape))
    got = model.density_grid(prob, dhat)
    s = model.signed_index(n)
    ref = np.zeros((n, n, n))
    j = np.arange(n)
    for a in range(n):
        for b in range(n):
            for c in range(n):
                # stored entry of (s_a, s_b, s_c) or the conjugate of (-k)'s
                if s[c] >= 0:
                    v = dhat[a, b, s[c]]
                else:
                    v = np.conj(dhat[(-s[a]) % n, (-s[b]) % n, -s[c]])
                ph = np.exp(2j * math.pi * (s[a] * j[:, None, None] + s[b] * j[None, :, None]
                                           + s[c] * j[None, None, :]) / n)
                ref += (v * ph).real
    ref /= n ** 3
    assert np.allclose(got, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    # and the linear continuity relation with the velocity grids: -div v / H0 = f delta,
    # the divergence taken spectrally from the oracle's own velocity field
    v = model.velocity_grids(prob, dhat)
    kf = 2 * math.pi / prob.box
    k = kf * np.fft.fftfreq(n, d=1.0 / n)
    div = sum(np.fft.ifftn(1j * kk * np.fft.fftn(v[a])).real
              for a, kk in enumerate((k[:, None, None], k[None, :, None], k[None, None, :])))
    # Nyquist components are excluded from the modes, so the relation is exact
    assert np.allclose(-div / model.H0, prob.f_growth * got, atol=1e-9 * np.abs(got).max() * prob.f_growth)


# ------------------------------------------------------------------ the CIC --

def test_cic_reproduces_constant_and_linear_fields():
    m, prob = _problem(n_grid=16, box=200.0, radius=60.0)
    n, box = prob.n_grid, prob.box
    j = np.arange(n) * box / n
    X, Y, Z = np.meshgrid(j, j, j, indexing="ij")
    const = np.array([120.0, -40.0, 75.0])
    grids = np.stack([np.full((n, n, n), c) for c in const])
    u, du = model.cic_gather(prob, grids, m.d_true)
    assert np.abs(u - prob.rhat @ const).max() < 1e-11
    assert np.abs(du).max() < 1e-12
    # linear field v_c = sum_a G_ca x_a (no cell of the 60 Mpc/h sphere
    # touches the periodic seam of the 200 Mpc/h box)
    G = np.array([[1.0, 2.0, -0.5], [0.3, -1.0, 0.7], [0.0, 0.4, 2.0]])
    grids = np.stack([G[c, 0] * X + G[c, 1] * Y + G[c, 2] * Z for c in range(3)])
    x = model.galaxy_positions(prob, m.d_true)
    u, du = model.cic_gather(prob, grids, m.d_true)
    exact_u = np.einsum("ic,ca,ia->i", prob.rhat, G, x)
    exact_du = np.einsum("ic,ca,ia->i", prob.rhat, G, prob.rhat)
    assert np.abs(u - exact_u).max() < 1e-9
    assert np.abs(du - exact_du).max() < 1e-9


def test_cic_matches_bruteforce_hat_functions():
    # Trilinear interpolation = sum over every node of the product of 1-D
    # hat functions max(0, 1 - |x - x_j|/Delta) with periodic images.
    m, prob = _problem(n_grid=4, box=40.0, n_gal=25, radius=30.0, seed=11)
    n, box = prob.n_grid, prob.box
    rng = np.random.default_rng(4)
    grids = rng.standard_normal((3, n, n, n))
    u, _ = model.cic_gather(prob, grids, m.d_true)
    x = model.galaxy_positions(prob, m.d_true)
    delta = box / n
    brute = np.zeros(len(u))
    for i in range(len(u)):
        vel = np.zeros(3)
        for a in range(n):
            for b in range(n):
                for c in range(n):
                    w = 1.0
                    for ax, node in enumerate((a, b, c)):
                        dist = (x[i, ax] - node * delta) % box
                        dist = min(dist, box - dist)
                        w *= max(0.0, 1.0 - dist / delta)
                    vel += w * grids[:, a, b, c]
        brute[i] = vel @ prob.rhat[i]
    assert np.abs(u - brute).max() < 1e-12


def test_scatter_is_the_adjoint_of_the_gather():
    m, prob = _problem(n_grid=8, n_gal=40)
    rng = np.random.default_rng(8)
    grids = rng.standard_normal((3, 8, 8, 8))
    g = rng.standard_normal(prob.n_gal)
    u, _ = model.cic_gather(prob, grids, m.d_true)
    G = model.cic_scatter(prob, m.d_true, g)
    assert abs(np.dot(u, g) - np.sum(G * grids)) < 1e-12 * np.abs(np.dot(u, g)) * 10
    # weights of each point sum to one: scatter of g = 1 with component c
    ones = model.cic_scatter(prob, m.d_true, np.ones(prob.n_gal))
    assert np.allclose(ones.reshape(3, -1).sum(axis=1), prob.rhat.sum(axis=0))


def test_mode_operator_adjoint_dot_product():
    # <A x, g> = <x, A^T g> for the modes -> u map in flat real coordinates.
    m, prob = _problem(n_grid=8, n_gal=50)
    n = prob.n_grid
    rng = np.random.default_rng(12)
    x = rng.standard_normal((n - 1) ** 3 - 1)
    g = rng.standard_normal(prob.n_gal)
    ax = model.project_gather(prob, hmc.unpack_modes(n, x), m.d_true)
    atg = hmc.pack_modes(n, model.modes_adjoint(prob, m.d_true, g))
    lhs, rhs = np.dot(ax, g), np.dot(x, atg)
    assert abs(lhs - rhs) <= 1e-13 * max(abs(lhs), np.abs(ax).max())


@pytest.mark.parametrize("n_grid", [8, 16])
def test_direct_adjoint_at_sampled_modes_equals_the_transform(n_grid):
    # The adjoint summed directly over the nodes the points reach, at every
    # stored entry, against the scatter-and-transform form (pinned above by
    # the dot-product test and the exact central differences below).
    m, prob = _problem(n_grid=n_grid, n_gal=70, box=40.0 * n_grid)
    n = prob.n_grid
    rng = np.random.default_rng(5)
    g = rng.standard_normal(prob.n_gal)
    full = model.modes_adjoint(prob, m.d_true, g)
    ix, iy, iz = np.meshgrid(np.arange(n), np.arange(n), np.arange(n // 2 + 1), indexing="ij")
    kidx = (ix.ravel(), iy.ravel(), iz.ravel())
    direct = model.modes_adjoint_at(prob, m.d_true, g, kidx)
    assert np.abs(direct - full.ravel()).max() <= 1e-12 * np.abs(full).max()
    # and the sampled evaluation agrees with the whole one where it is defined
    dhat = hmc.symmetrise(n, m.dhat_true)
    d = m.d_true * (1.0 + 0.01 * rng.standard_normal(prob.n_gal))
    ref = model.logpost_grad(prob, dhat, d, 1.3)
    pick = rng.choice(len(kidx[0]), 40, replace=False)
    sub = tuple(a[pick] for a in kidx)
    got = model.logpost_grad_sampled(prob, dhat, d, 1.3, sub)
    assert got[0] == ref[0] and got[3] == ref[3]
    assert np.array_equal(got[2], ref[2])
    assert np.abs(got[1] - ref[1][sub]).max() <= 1e-12 * np.abs(ref[1]).max()


# ---------------------------------------------------------- the gradient --

def _psi(prob, x_flat, d, s):
    return model.logpost(prob, hmc.unpack_modes(prob.n_grid, x_flat), d, s)


def test_gradient_modes_exact_central_difference():
    # Psi is a quadratic polynomial in any single mode coordinate, so the
    # central difference is exact up to rounding even for a large step.
    m, prob = _problem(n_grid=8, n_gal=60)
    n = prob.n_grid
    dhat = hmc.symmetrise(n, m.dhat_true)
    d, s = m.d_true.copy(), 1.3
    psi, gm, gd, gs = model.logpost_grad(prob, dhat, d, s)
    assert abs(psi - model.logpost(prob, dhat, d, s)) < 1e-12 * abs(psi)
    x0 = hmc.pack_modes(n, dhat)
    gflat = hmc.pack_modes(n, gm)
    hstep = 0.3 * math.sqrt(model.mode_variance(prob).max())
    rng = np.random.default_rng(1)
    # include kz = 0 plane coordinates explicitly
    plane = np.nonzero(hmc.pack_modes(n, (model.mode_indices(n)[2] == 0).astype(complex)))[0]
    picks = np.concatenate([rng.choice(len(x0), 24, replace=False), plane[:4]])
    for a in picks:
        xp, xm = x0.copy(), x0.copy()
        xp[a] += hstep
        xm[a] -= hstep
        fd = (_psi(prob, xp, d, s) - _psi(prob, xm, d, s)) / (2 * hstep)
        assert abs(fd - gflat[a]) < 1e-6 * (abs(gflat[a]) + 1.0)


def test_gradient_distances_and_sigma_nl_central_difference():
    m, prob = _problem(n_grid=8, n_gal=60)
    n = prob.n_grid
    dhat = hmc.symmetrise(n, m.dhat_true)
    d, s = m.d_true.copy(), 1.3
    _, _, gd, gs = model.logpost_grad(prob, dhat, d, s)
    x = model.galaxy_positions(prob, d) / prob.spacing
    frac = x - np.floor(x)
    hh = 1e-5
    # skip points within 4 steps of a cell face: the CIC derivative jumps there
    far = np.all((frac > 4 * hh / prob.spacing) & (frac < 1 - 4 * hh / prob.spacing), axis=1)
    checked = 0
    for i in np.nonzero(far)[0][:12]:
        dp, dm = d.copy(), d.copy()
        dp[i] += hh
        dm[i] -= hh
        fd = (model.logpost(prob, dhat, dp, s) - model.logpost(prob, dhat, dm, s)) / (2 * hh)
        assert abs(fd - gd[i]) < 1e-5 * (abs(gd[i]) + 1e-2)
        checked += 1
    assert checked >= 8
    fd = (model.logpost(prob, dhat, d, s + hh) - model.logpost(prob, dhat, d, s - hh)) / (2 * hh)
    assert abs(fd - gs) < 1e-6 * abs(gs)


def test_psi_is_even_in_s_and_inf_outside_domain():
    m, prob = _problem(n_grid=8, n_gal=30)
    dhat = hmc.symmetrise(8, m.dhat_true)
    d = m.d_true.copy()
    assert model.logpost(prob, dhat, d, 1.7) == model.logpost(prob, dhat, d, -1.7)
    for bad in (0.0, -5.0, model.C_KMS / (3 * prob.omega_m * model.H0), np.nan):
        dd = d.copy()
        dd[3] = bad
        assert model.logpost(prob, dhat, dd, 1.0) == math.inf
        assert model.logpost_grad(prob, dhat, dd, 1.0)[0] == math.inf


def test_prior_energy_matches_flat_sum():
    # (1/2) sum_k w_k |dhat|^2/sigma^2 = sum over independent real coords x_a^2/(2 S_a).
    m, prob = _problem(n_grid=8)
    n = prob.n_grid
    dhat = hmc.symmetrise(n, m.dhat_true)
    x = hmc.pack_modes(n, dhat)
    sv = hmc.pack_modes(n, model.mode_variance(prob).astype(complex))
    mm = len(x) // 2
    sdiag = 0.5 * np.concatenate([sv[:mm], sv[:mm]])
    assert abs(model.prior_energy(prob, dhat) - np.sum(x * x / (2 * sdiag))) < 1e-10


def test_empty_catalogue_is_prior_only():
    prob = _empty_problem()
    rng = np.random.default_rng(3)
    dhat = hmc.unpack_modes(8, rng.standard_normal(7 ** 3 - 1))
    psi, gm, gd, gs = model.logpost_grad(prob, dhat, np.zeros(0), 1.0)
    var = model.mode_variance(prob)
    assert abs(psi - model.prior_energy(prob, dhat)) < 1e-12 * psi
    assert np.allclose(gm, np.where(var > 0, 2 * dhat / np.where(var > 0, var, 1), 0))
    assert gs == 0.0 and gd.shape == (0,)
