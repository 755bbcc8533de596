"""Pins of the oracle sampler (Section 3): RNG, leapfrog, MH, dual averaging."""
import math
import os

import numpy as np
import pytest

from oracle import hmc, model, philox
from paper_2203_02369_amd import mocks

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _problem(n_grid=8, box=200.0, n_gal=60, radius=80.0, seed=3, **kw):
    m = mocks.make_mock(n_grid, box, n_gal, radius, "sphere", (0.2, 0.2), seed=seed)
    kwargs = m.problem_kwargs()
    kwargs.update(kw)
    return m, model.Problem(**kwargs)


def _prior_only(n_grid=8, box=200.0):
    m = mocks.make_mock(n_grid, box, 1, 50.0, seed=1)
    kw = m.problem_kwargs()
    for key in ("mu", "sigma_mu", "cz", "sigma_cz"):
        kw[key] = np.zeros(0)
    kw["rhat"] = np.zeros((0, 3))
    return m, model.Problem(**kw)


# ------------------------------------------------------------------- Philox --

def test_philox_known_answers():
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(t, 16) for t in r]
        out = philox.philox4x32_10(np.array(v[:4]), (v[4], v[5]))
        assert [int(o) for o in out] == v[6:10]


def test_uniforms_and_normals():
    w = philox.draw_words(123, 0, philox.PURPOSE_MODES, np.arange(200000))
    u = philox.uniform53(w[:, 0], w[:, 1])
    assert u.min() > 0.0 and u.max() <= 1.0
    assert abs(u.mean() - 0.5) < 0.003
    z0, z1 = philox.normal_pair(w)
    z = np.concatenate([z0, z1])
    assert abs(z.mean()) < 0.01 and abs(z.var() - 1.0) < 0.01
    assert abs(np.mean(z0 * z1)) < 0.01
    # different stream coordinates give different words
    w2 = philox.draw_words(123, 1, philox.PURPOSE_MODES, np.arange(4))
    assert not np.array_equal(w[:4], w2)


# ---------------------------------------------------------------- momenta --

def test_momenta_respect_layout_and_mass():
    m, prob = _problem(n_grid=16, n_gal=50)
    n = prob.n_grid
    p = hmc.draw_momenta(prob, seed=5, iteration=2)
    # mirrors hold the conjugate of their canonical partner, excluded modes 0
    assert np.array_equal(hmc.symmetrise(n, p.modes), p.modes)
    assert np.all(p.modes[~model.retained_mask(n)] == 0)
    # p ~ N(0, M): sigma_k^2 |p|^2 / 2 has mean 2 (two real parts, each chi^2_1)
    var = model.mode_variance(prob)
    keep = hmc.canonical_mask(n)
    stat = var[keep] * np.abs(p.modes[keep]) ** 2 / 2.0
    assert abs(stat.mean() - 2.0) < 0.1
    # distances: variance H0^2 / sigma_v^2
    assert p.dist.shape == (50,)
    # E[K] = D/2 with D the number of momentum coordinates
    dof = (n - 1) ** 3 - 1 + 50 + 1
    k = hmc.kinetic(prob, p)
    assert abs(k - dof / 2.0) < 4.0 * math.sqrt(dof / 2.0)


# --------------------------------------------------------------- leapfrog --

def test_prior_only_leapfrog_closed_form():
    # Prior only: each real coordinate is a unit-frequency oscillator in
    # q~ = q / sqrt(S), p~ = sqrt(S) p (S = sigma_k^2 / 2 = M^-1), and one
    # kick-drift-kick step is the exact linear map
    #   [[1 - e^2/2, e], [-e (1 - e^2/4), 1 - e^2/2]].
    m, prob = _prior_only(n_grid=8)
    n = prob.n_grid
    rng = np.random.default_rng(0)
    var = model.mode_variance(prob)
    sv = hmc.pack_modes(n, var.astype(complex))
    mm = len(sv) // 2
    S = 0.5 * np.concatenate([sv[:mm], sv[:mm]])
    x0 = rng.standard_normal(len(S)) * np.sqrt(S)
    q0 = hmc.State(hmc.unpack_modes(n, x0), np.zeros(0), 1.0)
    p0 = hmc.draw_momenta(prob, 9, 0)
    eps, steps = 0.37, 7
    q1, p1, _ = hmc.leapfrog(prob, q0, p0, eps, steps)
    a = 1.0 - eps * eps / 2.0
    step = np.array([[a, eps], [-eps * (1.0 - eps * eps / 4.0), a]])
    mat = np.linalg.matrix_power(step, steps)
    qt = x0 / np.sqrt(S)
    pt = hmc.pack_modes(n, p0.modes) * np.sqrt(S)
    q_exp = (mat[0, 0] * qt + mat[0, 1] * pt) * np.sqrt(S)
    p_exp = (mat[1, 0] * qt + mat[1, 1] * pt) / np.sqrt(S)
    assert np.abs(hmc.pack_modes(n, q1.modes) - q_exp).max() < 1e-12 * np.abs(q_exp).max()
    assert np.abs(hmc.pack_modes(n, p1.modes) - p_exp).max() < 1e-12 * np.abs(p_exp).max()
    # the shadow energy (1 - e^2/4) q~^2 + p~^2 is conserved per coordinate
    q1t = hmc.pack_modes(n, q1.modes) / np.sqrt(S)
    p1t = hmc.pack_modes(n, p1.modes) * np.sqrt(S)
    e0 = (1 - eps ** 2 / 4) * qt ** 2 + pt ** 2
    e1 = (1 - eps ** 2 / 4) * q1t ** 2 + p1t ** 2
    assert np.abs(e1 - e0).max() < 1e-11 * e0.max()


def test_leapfrog_is_reversible():
    m, prob = _problem(n_grid=8, n_gal=60)
    n = prob.n_grid
    q0 = hmc.State(hmc.symmetrise(n, 0.5 * m.dhat_true), m.d_true.copy(), 1.2)
    p0 = hmc.draw_momenta(prob, 4, 0)
    q1, p1, _ = hmc.leapfrog(prob, q0, p0, 0.05, 50)
    p1n = hmc.State(-p1.modes, -p1.dist, -p1.s)
    q2, p2, _ = hmc.leapfrog(prob, q1, p1n, 0.05, 50)
    assert np.abs(q2.modes - q0.modes).max() <= 1e-10 * np.abs(q0.modes).max()
    assert np.abs(q2.dist - q0.dist).max() <= 1e-10 * np.abs(q0.dist).max()
    assert abs(q2.s - q0.s) <= 1e-10
    assert np.abs(p2.modes + p0.modes).max() <= 1e-9 * np.abs(p0.modes).max()
    # and it moved
    assert np.abs(q1.dist - q0.dist).max() > 1e-3


def test_energy_error_scales_as_eps_squared():
    # Distances held fixed: with them free, Psi jumps where d crosses a bin
    # of the distance histogram (eq:D is piecewise constant) and the CIC
    # derivative jumps at cell faces, which adds an O(1) energy error that
    # does not scale with the step.
    m, prob = _problem(n_grid=8, n_gal=60, sample_distances=False)
    n = prob.n_grid
    q0 = hmc.State(hmc.symmetrise(n, 0.5 * m.dhat_true), m.d_true.copy(), 1.2)
    cached = hmc.gradient(prob, q0)
    # steps well inside the stability limit of the stiffest (data-bound) mode
    T = 0.4
    errs = []
    eps_list = [0.04, 0.02, 0.01]
    for eps in eps_list:
        e = []
        for seed in range(3):
            p0 = hmc.draw_momenta(prob, 100 + seed, 0)
            h0 = hmc.kinetic(prob, p0) + cached[0]
            q1, p1, c1 = hmc.leapfrog(prob, q0, p0, eps, int(round(T / eps)), cached)
            e.append(abs(hmc.kinetic(prob, p1) + c1[0] - h0))
        errs.append(np.mean(e))
    slope = np.polyfit(np.log(eps_list), np.log(errs), 1)[0]
    assert 1.8 <= slope <= 2.2, (errs, slope)


# ------------------------------------------------------------------- chains --

def test_rejection_keeps_the_state():
    m, prob = _problem(n_grid=8, n_gal=40)
    n = prob.n_grid
    q0 = hmc.State(hmc.symmetrise(n, m.dhat_true), m.d_true.copy(), 1.0)
    res = hmc.hmc_run(prob, q0, n_iter=4, n_leapfrog=3, eps0=5.0, seed=1)
    assert res.accepted.sum() == 0
    assert np.array_equal(res.state.modes, q0.modes)
    assert np.array_equal(res.state.dist, q0.dist)
    assert np.allclose(res.mode_sum, 4 * q0.modes)
    assert np.all(res.dh > 0)


def test_accept_rule_uses_the_uniform_stream():
    m, prob = _problem(n_grid=8, n_gal=40)
    n = prob.n_grid
    q0 = hmc.State(hmc.symmetrise(n, m.dhat_true), m.d_true.copy(), 1.0)
    res = hmc.hmc_run(prob, q0, n_iter=12, n_leapfrog=4, eps0=0.1, seed=77)
    for it in range(12):
        w = philox.draw_words(77, it, philox.PURPOSE_ACCEPT, [0])
        u = float(philox.uniform53(w[0, 0], w[0, 1]))
        assert bool(res.accepted[it]) == (math.log(u) < -res.dh[it])


@pytest.mark.slow
def test_prior_only_chain_recovers_mode_variance():
    m, prob = _prior_only(n_grid=8)
    n = prob.n_grid
    # start from a prior draw (from dhat = 0 every trajectory gains energy)
    var = model.mode_variance(prob)
    rng = np.random.default_rng(0)
    x0 = hmc.pack_modes(n, np.sqrt(var / 2) * (rng.standard_normal(var.shape)
                                               + 1j * rng.standard_normal(var.shape)))
    q0 = hmc.State(hmc.unpack_modes(n, x0), np.zeros(0), 1.0)
    samples = []
    res = hmc.hmc_run(prob, q0, n_iter=400, n_leapfrog=5, eps0=0.3, seed=3, jitter=True,
                      callback=lambda it, q, dh, acc, e: samples.append(q.modes.copy()))
    keep = hmc.canonical_mask(n)
    ratio = np.array([np.abs(s[keep]) ** 2 / var[keep] for s in samples[50:]])
    # <|dhat|^2> / sigma_k^2 = 1 for every mode; averaged over modes and states
    assert abs(ratio.mean() - 1.0) < 0.05
    assert res.accepted.mean() > 0.75


@pytest.mark.slow
def test_dual_averaging_reaches_the_target_acceptance():
    m, prob = _problem(n_grid=8, n_gal=40)
    n = prob.n_grid
    q0 = hmc.State(hmc.symmetrise(n, m.dhat_true), m.d_true.copy(), 1.3)
    res = hmc.hmc_run(prob, q0, n_iter=400, n_leapfrog=5, eps0=0.5, seed=11, warmup=200)
    post = np.array([hmc.accept_probability(x) for x in res.dh[200:]])
    assert 0.5 < post.mean() < 0.8, post.mean()
    assert res.eps > 0
