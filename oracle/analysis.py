"""Oracle of the chain's field statistics of Section 5: the monopole and
dipole moments of the velocity field in spheres about the observer
("Monopole and dipole"), the maps of the mean and the scatter along the
chain of the density contrast and of the radial velocity, and statistics of
fields in spherical shells ("Correlation Coefficients").

TEST INFRASTRUCTURE ONLY.  Plain FP64 numpy written from the definitions;
only the test suite, the smoke check and the CPU baseline leg of the
benchmark may import it.

For a sphere of radius R centred on the observer o = (L/2)(1, 1, 1):
  * the monopole M(R) is the volume mean of -div v / H0 over the ball
    (the paper scales by H0 so that it follows the mean linear overdensity:
    with the velocity operator of model.velocity_multiplier, -div v / H0 is
    f delta);
  * the dipole D(R) is the volume mean of v over the ball: the bulk velocity
    of the sphere, in km/s.

Readings (also in the design notes):
  * The field between grid nodes is the band-limited (trigonometric)
    interpolant of the retained modes, v_c(x) = N^-3 sum_k m_c(k) dhat_k
    exp(i k.x) over all N^3 modes; on the nodes it is model.velocity_grids.
    The paper averages over grid cells; the continuous mean of the
    interpolant is the limit of that average for fine cells and has no
    dependence on how cells straddle the sphere.
  * The ball mean of a plane wave exp(i k.x) is exp(i k.o) W(|k| R) with the
    top-hat window W(y) = 3 (sin y - y cos y) / y^3, W(0) = 1.  Hence
        M(R)   = N^-3 sum_k (-i k.m(k) / H0) dhat_k exp(i k.o) W(|k| R),
        D_c(R) = N^-3 sum_k m_c(k) dhat_k exp(i k.o) W(|k| R),
    summed over the full spectrum (model.full_spectrum), real by Hermitian
    symmetry.
"""
import math

import numpy as np

from . import model


def tophat_window(y):
    """W(y) = 3 (sin y - y cos y) / y^3.  Below |y| = 1/2, where the closed
    form cancels, its Taylor series sum_m (-1)^m 3 (2m + 2) y^(2m) / (2m + 3)!
    to m = 7 (next term below 1e-17)."""
    y = np.asarray(y, dtype=np.float64)
    small = np.abs(y) < 0.5
    ys = np.where(small, 1.0, y)
    exact = 3.0 * (np.sin(ys) - ys * np.cos(ys)) / ys ** 3
    y2 = y * y
    series = np.zeros_like(y)
    for m in range(7, -1, -1):
        series = series * y2 + (-1) ** m * 3.0 * (2 * m + 2) / math.factorial(2 * m + 3)
    return np.where(small, series, exact)


def _full_grid_modes(prob):
    """Signed wave vectors and the retained mask over all N^3 modes."""
    n = prob.n_grid
    s = model.signed_index(n)
    nx, ny, nz = np.meshgrid(s, s, s, indexing="ij")
    half = n // 2
    keep = ~((np.abs(nx) == half) | (np.abs(ny) == half) | (np.abs(nz) == half) | ((nx == 0) & (ny == 0) & (nz == 0)))
    kf = 2.0 * math.pi / prob.box
    return (kf * nx, kf * ny, kf * nz), keep


def sphere_moments(prob, dhat, radii):
    """(M, D) for each radius: arrays (n_R,) and (n_R, 3).

    dhat: half spectrum (N, N, N/2 + 1) complex, as everywhere in the oracle.
    """
    n = prob.n_grid
    kvec, keep = _full_grid_modes(prob)
    k2 = kvec[0] ** 2 + kvec[1] ** 2 + kvec[2] ** 2
    safe = np.where(keep, k2, 1.0)
    amp = model.H0 * prob.f_growth
    m = [np.where(keep, 1j * amp * kc / safe, 0.0) for kc in kvec]       # m_c(k), eq:vel-field
    div = -1j * (kvec[0] * m[0] + kvec[1] * m[1] + kvec[2] * m[2]) / model.H0
    full = model.full_spectrum(dhat)
    o = 0.5 * prob.box
    phase = np.exp(1j * (kvec[0] * o + kvec[1] * o + kvec[2] * o))
    kmag = np.sqrt(k2)
    norm = 1.0 / float(n) ** 3
    mono, dip = [], []
    for r in radii:
        w = tophat_window(kmag * r)
        base = full * phase * w
        mono.append(norm * np.sum(div * base).real)
        dip.append([norm * np.sum(mc * base).real for mc in m])
    return np.array(mono), np.array(dip)


def sphere_moments_abs(prob, dhat, radii):
    """Sum of the absolute values of the terms of sphere_moments, per
    quantity: the scale of its rounding error (shape (n_R, 4))."""
    n = prob.n_grid
    kvec, keep = _full_grid_modes(prob)
    k2 = kvec[0] ** 2 + kvec[1] ** 2 + kvec[2] ** 2
    safe = np.where(keep, k2, 1.0)
    amp = model.H0 * prob.f_growth
    m = [np.where(keep, amp * np.abs(kc) / safe, 0.0) for kc in kvec]
    full = np.abs(model.full_spectrum(dhat))
    kmag = np.sqrt(k2)
    norm = 1.0 / float(n) ** 3
    out = []
    for r in radii:
        w = np.abs(tophat_window(kmag * r))
        out.append([norm * np.sum(prob.f_growth * keep * full * w)] + [norm * np.sum(mc * full * w) for mc in m])
    return np.array(out)


def radial_velocity_grid(prob, dhat):
    """v_r(x_j) = v(x_j) . (x_j - o) / |x_j - o| on every node x_j = j L / N,
    the observer at o = (L/2)(1, 1, 1); 0 at the observer itself.  Shape
    (N, N, N)."""
    n = prob.n_grid
    v = model.velocity_grids(prob, dhat)
    pos = np.arange(n) * (prob.box / n) - 0.5 * prob.box
    rx, ry, rz = np.meshgrid(pos, pos, pos, indexing="ij")
    r = np.sqrt(rx * rx + ry * ry + rz * rz)
    dot = v[0] * rx + v[1] * ry + v[2] * rz
    return np.where(r > 0, dot / np.where(r > 0, r, 1.0), 0.0)


def field_sums(prob, states):
    """Running sums over a chain's states of the density contrast and the
    radial velocity on the grid and of their squares:
    array (4, N, N, N) = [sum delta, sum delta^2, sum v_r, sum v_r^2].  With
    n states, the mean map is S1 / n and the scatter map Sigma^2 is
    S2 / n - (S1 / n)^2."""
    n = prob.n_grid
    out = np.zeros((4, n, n, n))
    for dhat in states:
        delta = model.density_grid(prob, dhat)
        vr = radial_velocity_grid(prob, dhat)
        out[0] += delta
        out[1] += delta * delta
        out[2] += vr
        out[3] += vr * vr
    return out


def node_distances(prob):
    """|x_j - o| (Mpc/h) of every node x_j = j L / N from the observer
    o = (L/2)(1, 1, 1); shape (N, N, N)."""
    n = prob.n_grid
    pos = np.arange(n) * (prob.box / n) - 0.5 * prob.box
    rx, ry, rz = np.meshgrid(pos, pos, pos, indexing="ij")
    return np.sqrt(rx * rx + ry * ry + rz * rz)


def shell_stats(prob, a, b, width, n_shells):
    """Per shell s (the nodes at distance in [s width, (s + 1) width)): node
    count, mean and scatter (population standard deviation) of a and of b,
    and the Pearson correlation coefficient of a and b over those nodes;
    NaN where undefined.  b None counts as zero.  Shape (n_shells, 6)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.zeros_like(a) if b is None else np.asarray(b, dtype=np.float64)
    shell = np.floor(node_distances(prob) / width).astype(np.int64)
    out = np.full((n_shells, 6), np.nan)
    for s in range(n_shells):
        sel = shell == s
        cnt = int(np.count_nonzero(sel))
        out[s, 0] = cnt
        if cnt == 0:
            continue
        xa, xb = a[sel], b[sel]
        ma, mb = xa.mean(), xb.mean()
        da, db = xa - ma, xb - mb
        va, vb = np.mean(da * da), np.mean(db * db)
        out[s, 1:5] = [ma, math.sqrt(va), mb, math.sqrt(vb)]
        if va > 0 and vb > 0:
            out[s, 5] = np.mean(da * db) / math.sqrt(va * vb)
    return out
