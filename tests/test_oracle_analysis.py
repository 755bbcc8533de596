"""Pins of the oracle's sphere moments (Section 5, "Monopole and dipole")
against values fixed independently of its k-space sums: the field at the
observer node, quadrature of the band-limited field over the ball, the
window's own integral, and a single mode in closed form.  Pins of the radial
velocity and the field sums: the components along the axes and diagonals
through the observer, a single mode's radial field in closed form, and
linearity of the sums.  Pins of the shell statistics: brute force over the
nodes of a small grid, exact correlations of +-1, and the distance field's
shell means inside their shells."""
import math

import numpy as np
import pytest

from oracle import analysis, hmc, model
from paper_2203_02369_amd import mocks

from helpers import oracle_problem


def _problem(n, box, seed):
    m = mocks.make_mock(n, box, 20, 0.3 * box, "sphere", (0.2, 0.2), seed=seed)
    prob = oracle_problem(m)
    rng = np.random.default_rng(seed)
    shape = model.half_shape(n)
    dhat = hmc.symmetrise(n, rng.standard_normal(shape) + 1j * rng.standard_normal(shape))
    return prob, dhat


def test_window_is_the_ball_mean_of_a_plane_wave():
    # (3 / R^3) int_0^R j0(k r) r^2 dr by Gauss-Legendre, against W(kR)
    x, w = np.polynomial.legendre.leggauss(40)
    for kr in (1e-6, 5e-3, 0.02, 0.7, 3.0, 9.5, 21.0):
        r = 0.5 * (x + 1.0)                     # R = 1
        j0 = np.sin(kr * r) / (kr * r)
        quad = 3.0 * np.sum(0.5 * w * j0 * r * r)
        assert abs(analysis.tophat_window(kr) - quad) <= 1e-13, kr
    assert analysis.tophat_window(0.0) == 1.0


def test_vanishing_radius_gives_the_field_at_the_observer():
    n = 8
    prob, dhat = _problem(n, 100.0, 3)
    mono, dip = analysis.sphere_moments(prob, dhat, [1e-9])
    v = model.velocity_grids(prob, dhat)
    c = n // 2                                     # o = (L/2)(1,1,1) is node N/2
    assert np.allclose(dip[0], v[:, c, c, c], rtol=1e-12, atol=1e-12 * np.abs(v).max())
    delta = np.fft.ifftn(model.full_spectrum(dhat)).real   # N^-3 sum_k dhat e^{ik.x}
    assert abs(mono[0] - prob.f_growth * delta[c, c, c]) <= 1e-12 * np.abs(delta).max()


def _ball_quadrature(prob, full, mult, radius):
    """Ball means of N^-3 sum_k a_k e^{ik.x} by a product rule in (r, mu, phi)."""
    n = prob.n_grid
    s = model.signed_index(n)
    nx, ny, nz = np.meshgrid(s, s, s, indexing="ij")
    kf = 2.0 * math.pi / prob.box
    kx, ky, kz = (kf * a.reshape(-1) for a in (nx, ny, nz))
    xr, wr = np.polynomial.legendre.leggauss(24)
    r = 0.5 * radius * (xr + 1.0)
    wr = 0.5 * radius * wr * r * r
    mu, wmu = np.polynomial.legendre.leggauss(24)
    nphi = 48
    phi = 2.0 * math.pi * np.arange(nphi) / nphi
    R, MU, PHI = np.meshgrid(r, mu, phi, indexing="ij")
    W = (wr[:, None, None] * wmu[None, :, None] * np.full(nphi, 2.0 * math.pi / nphi)[None, None, :]).reshape(-1)
    st = np.sqrt(1.0 - MU * MU)
    o = 0.5 * prob.box
    px = (o + R * st * np.cos(PHI)).reshape(-1)
    py = (o + R * st * np.sin(PHI)).reshape(-1)
    pz = (o + R * MU).reshape(-1)
    vol = 4.0 / 3.0 * math.pi * radius ** 3
    out = []
    for a in mult:
        coef = (a * full).reshape(-1) / float(n) ** 3
        acc = 0.0
        for i0 in range(0, len(px), 4096):
            ph = np.exp(1j * (np.outer(px[i0:i0 + 4096], kx) + np.outer(py[i0:i0 + 4096], ky)
                              + np.outer(pz[i0:i0 + 4096], kz)))
            acc += np.sum(W[i0:i0 + 4096] * (ph @ coef).real)
        out.append(acc / vol)
    return np.array(out)


def test_ball_means_match_quadrature_of_the_band_limited_field():
    n = 8
    prob, dhat = _problem(n, 100.0, 5)
    full = model.full_spectrum(dhat)
    # m_c(k) on the full grid from the half-spectrum multiplier's own formula
    s = model.signed_index(n)
    nx, ny, nz = np.meshgrid(s, s, s, indexing="ij")
    kf = 2.0 * math.pi / prob.box
    k2 = (kf * kf) * (nx * nx + ny * ny + nz * nz)
    half = n // 2
    keep = ~((np.abs(nx) == half) | (np.abs(ny) == half) | (np.abs(nz) == half) | (k2 == 0))
    amp = model.H0 * prob.f_growth
    mult = [np.where(keep, 1j * amp * kf * a / np.where(keep, k2, 1.0), 0.0) for a in (nx, ny, nz)]
    radii = [6.0, 17.0, 33.0]
    mono, dip = analysis.sphere_moments(prob, dhat, radii)
    for j, r in enumerate(radii):
        qv = _ball_quadrature(prob, full, mult, r)
        qd = _ball_quadrature(prob, full, [np.ones_like(full)], r)[0]   # mean density contrast
        scale = np.abs(qv).max()
        assert np.abs(dip[j] - qv).max() <= 1e-10 * scale, (r, dip[j], qv)
        # -div v / H0 = f delta for the linear velocity field
        assert abs(mono[j] - prob.f_growth * qd) <= 1e-10 * max(abs(qd), 1e-3), (r, mono[j], qd)


@pytest.mark.parametrize("mode", [(1, 0, 0), (0, 0, 2)])
def test_single_mode_in_closed_form(mode):
    n = 16
    prob, _ = _problem(n, 200.0, 7)
    dhat = np.zeros(model.half_shape(n), dtype=np.complex128)
    a = 0.3 - 1.7j
    dhat[mode[0] % n, mode[1] % n, mode[2]] = a
    if mode[2] == 0:
        dhat[(-mode[0]) % n, (-mode[1]) % n, 0] = np.conj(a)
    kf = 2.0 * math.pi / prob.box
    kvec = kf * np.array(mode, dtype=float)
    k = np.linalg.norm(kvec)
    sign = (-1.0) ** sum(mode)                      # e^{i k.o}, o = (L/2)(1,1,1)
    radii = [5.0, 40.0]
    mono, dip = analysis.sphere_moments(prob, dhat, radii)
    for j, r in enumerate(radii):
        w = analysis.tophat_window(k * r)
        # the pair k, -k: N^-3 (a e^{ik.o} + conj(a) e^{-ik.o}) times each factor
        m_ref = 2.0 * sign * prob.f_growth * a.real * w / n ** 3
        d_ref = -2.0 * sign * model.H0 * prob.f_growth * a.imag * w * kvec / (k * k) / n ** 3
        assert abs(mono[j] - m_ref) <= 1e-13 * abs(m_ref)
        assert np.allclose(dip[j], d_ref, rtol=1e-13, atol=1e-13 * np.abs(d_ref).max())


def test_radial_velocity_on_lines_through_the_observer():
    n = 16
    prob, dhat = _problem(n, 160.0, 9)
    v = model.velocity_grids(prob, dhat)
    vr = analysis.radial_velocity_grid(prob, dhat)
    c = n // 2
    assert vr[c, c, c] == 0.0
    for d in (1, 3, c - 1):
        assert abs(vr[c + d, c, c] - v[0, c + d, c, c]) <= 1e-13 * np.abs(v).max()     # +x
        assert abs(vr[c, c - d, c] + v[1, c, c - d, c]) <= 1e-13 * np.abs(v).max()     # -y
        assert abs(vr[c, c, c + d] - v[2, c, c, c + d]) <= 1e-13 * np.abs(v).max()     # +z
        diag = (-v[0, c - d, c + d, c - d] + v[1, c - d, c + d, c - d] - v[2, c - d, c + d, c - d]) / math.sqrt(3.0)
        assert abs(vr[c - d, c + d, c - d] - diag) <= 1e-13 * np.abs(v).max()
    # the corner node sits at r = -(L/2)(1, 1, 1)
    assert abs(vr[0, 0, 0] + v[:, 0, 0, 0].sum() / math.sqrt(3.0)) <= 1e-13 * np.abs(v).max()


def test_radial_velocity_of_a_single_mode_in_closed_form():
    # one mode pair k = (1, 0, 0) kf with dhat = a: v(x) = -(2 H0 f / (N^3 kf))
    # * Im(a e^{i kf x}) along x only, so v_r = v_x (x - L/2) / |r|
    n = 16
    prob, _ = _problem(n, 160.0, 9)
    dhat = np.zeros(model.half_shape(n), dtype=np.complex128)
    a = 0.8 + 0.45j
    dhat[1, 0, 0] = a
    dhat[n - 1, 0, 0] = np.conj(a)
    kf = 2.0 * math.pi / prob.box
    h = prob.box / n
    xs = np.arange(n) * h
    vx = -2.0 * model.H0 * prob.f_growth / (n ** 3 * kf) * np.imag(a * np.exp(1j * kf * xs))
    pos = xs - 0.5 * prob.box
    rx, ry, rz = np.meshgrid(pos, pos, pos, indexing="ij")
    r = np.sqrt(rx * rx + ry * ry + rz * rz)
    ref = np.where(r > 0, vx[:, None, None] * rx / np.where(r > 0, r, 1.0), 0.0)
    got = analysis.radial_velocity_grid(prob, dhat)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


def test_field_sums_are_linear_in_the_states():
    n = 8
    prob, a = _problem(n, 100.0, 12)
    _, b = _problem(n, 100.0, 13)
    delta = model.density_grid(prob, a)
    vr = analysis.radial_velocity_grid(prob, a)
    one = analysis.field_sums(prob, [a])
    assert np.array_equal(one, np.stack([delta, delta * delta, vr, vr * vr]))
    # a state and its negative: the sums cancel, the squares double
    pm = analysis.field_sums(prob, [a, -a])
    assert np.abs(pm[0]).max() <= 1e-15 * np.abs(delta).max() and np.abs(pm[2]).max() <= 1e-15 * np.abs(vr).max()
    assert np.allclose(pm[1], 2 * delta * delta, rtol=1e-14, atol=0) and np.allclose(pm[3], 2 * vr * vr, rtol=1e-14, atol=0)
    # (a + b) / 2 and (a - b) / 2: the sums give a, the squares (A^2 + B^2) / 2
    two = analysis.field_sums(prob, [0.5 * (a + b), 0.5 * (a - b)])
    db = model.density_grid(prob, b)
    assert np.allclose(two[0], delta, rtol=0, atol=1e-14 * np.abs(delta).max())
    assert np.allclose(two[1], 0.5 * (delta * delta + db * db), rtol=0, atol=1e-13 * (delta * delta).max())


def _shell_problem(n, box):
    m = mocks.make_mock(n, box, 20, 0.3 * box, "sphere", (0.2, 0.2), seed=2)
    return oracle_problem(m)


def test_shell_stats_by_brute_force():
    # every node visited in plain loops on a 6^3 grid (observer at node 3)
    n, box, width = 6, 60.0, 7.0
    prob = _shell_problem(n, box)
    rng = np.random.default_rng(4)
    a = rng.standard_normal((n, n, n))
    b = 0.5 * a + rng.standard_normal((n, n, n))
    n_shells = 6
    members = [[] for _ in range(n_shells)]
    h = box / n
    for x in range(n):
        for y in range(n):
            for z in range(n):
                r = math.sqrt(((x - 3) * h) ** 2 + ((y - 3) * h) ** 2 + ((z - 3) * h) ** 2)
                s = int(r // width)
                if s < n_shells:
                    members[s].append((a[x, y, z], b[x, y, z]))
    got = analysis.shell_stats(prob, a, b, width, n_shells)
    for s, mem in enumerate(members):
        assert got[s, 0] == len(mem)
        if not mem:
            assert np.all(np.isnan(got[s, 1:]))
            continue
        xa = [p[0] for p in mem]
        xb = [p[1] for p in mem]
        k = len(mem)
        ma, mb = sum(xa) / k, sum(xb) / k
        sa = math.sqrt(sum((v - ma) ** 2 for v in xa) / k)
        sb = math.sqrt(sum((v - mb) ** 2 for v in xb) / k)
        assert abs(got[s, 1] - ma) <= 1e-14 and abs(got[s, 3] - mb) <= 1e-14
        assert abs(got[s, 2] - sa) <= 1e-14 and abs(got[s, 4] - sb) <= 1e-14
        if k > 1:
            cov = sum((u - ma) * (v - mb) for u, v in zip(xa, xb)) / k
            assert abs(got[s, 5] - cov / (sa * sb)) <= 1e-13
    # the observer's own node is alone in shell 0 here (the next node is 10 away)
    assert got[0, 0] == 1 and np.isnan(got[0, 5])


def test_shell_correlations_and_the_distance_field():
    n, box = 16, 160.0
    prob = _shell_problem(n, box)
    rng = np.random.default_rng(8)
    a = rng.standard_normal((n, n, n))
    width = 13.7
    st = analysis.shell_stats(prob, a, 2.0 * a + 3.0, width, 12)
    full = st[st[:, 0] > 1]
    assert np.allclose(full[:, 5], 1.0, atol=1e-13)
    assert np.allclose(full[:, 3], 2.0 * full[:, 1] + 3.0, atol=1e-13) and np.allclose(full[:, 4], 2.0 * full[:, 2], atol=1e-13)
    st = analysis.shell_stats(prob, a, -a, width, 12)
    assert np.allclose(st[st[:, 0] > 1][:, 5], -1.0, atol=1e-13)
    # the distance field: each shell's mean lies in its own shell, and the
    # counts add up to the nodes within the outer radius
    r = analysis.node_distances(prob)
    st = analysis.shell_stats(prob, r, None, width, 12)
    for s in range(12):
        if st[s, 0] > 0:
            assert s * width <= st[s, 1] < (s + 1) * width and st[s, 2] <= width / 2
    assert st[:, 0].sum() == np.count_nonzero(r < 12 * width)
    occupied = st[:, 0] > 0
    assert np.all(st[occupied, 3] == 0.0) and np.all(st[occupied, 4] == 0.0)
    # beyond the box corner the shells are empty
    far = analysis.shell_stats(prob, a, a, 30.0, 12)
    assert far[-1, 0] == 0 and np.all(np.isnan(far[-1, 1:]))
