"""Pins of the oracle No-U-Turn sampler (Section 3.3; Hoffman & Gelman's
efficient NUTS with dual averaging).

The sampler leaves its target distribution invariant: on Gaussian targets
(one and two dimensions, a correlated pair with a non-unit mass matrix) the
chain must reproduce the known mean and covariance; on the posterior of
Section 2 it must reproduce the prior's mode variance when there are no data
and the closed-form Wiener filter on linear Gaussian data.  A plausible
mistake in the tree (always moving to the new subtree, a missing subtree
test, a wrong merge probability) biases these moments.  The tree's
bookkeeping is checked against its definition: leaves per doubling, the
sampled leaf inside the trajectory, the draws that decide it.
"""
import math

import numpy as np
import pytest

from oracle import hmc, model, nuts, philox, wiener
from paper_2203_02369_amd import mocks

from test_oracle_wiener import integrated_autocorrelation_time


def _moments_ok(samples, cov, zmax=4.5):
    """Sample mean and covariance against the exact ones, in units of their
    standard errors (autocorrelation taken into account)."""
    x = np.asarray(samples)
    tau = integrated_autocorrelation_time(x)
    n_eff = len(x) / tau
    sd = np.sqrt(np.diag(cov))
    z_mean = x.mean(axis=0) / (sd / np.sqrt(n_eff))
    var = x.var(axis=0)
    # the variance of a Gaussian sample variance is 2 sigma^4 / n
    z_var = (var - np.diag(cov)) / (np.diag(cov) * np.sqrt(2.0 / n_eff))
    assert np.all(np.abs(z_mean) < zmax), z_mean
    assert np.all(np.abs(z_var) < zmax), z_var
    return x


@pytest.mark.parametrize("case", ["1d", "2d_correlated_mass"])
def test_nuts_samples_gaussian_targets(case):
    if case == "1d":
        cov, minv, eps = np.array([[1.0]]), np.array([1.0]), 0.4
    else:
        # correlation 0.9, scales 1 and 3, a mass matrix that does not match
        cov = np.array([[1.0, 2.7], [2.7, 9.0]])
        minv, eps = np.array([2.0, 0.5]), 0.3
    t = nuts.GaussianTarget(cov, minv)
    samples = []
    res = nuts.nuts_run(t, nuts.VecState(np.zeros(len(minv))), 3000, eps, 17,
                        callback=lambda it, q, st: samples.append(q.x.copy()))
    x = _moments_ok(samples[100:], cov)
    if case != "1d":
        r = np.corrcoef(x.T)[0, 1]
        assert abs(r - 0.9) < 0.02, r
    # the trees do grow: several doublings per iteration on these targets
    assert res.depth.mean() > 1.5


def test_a_biased_merge_is_detected():
    # The moment pin above detects a plausible slip in the tree: merging two
    # halves by always keeping the second half's sample (instead of with
    # probability n''/(n' + n'')) drives the chain towards the trajectory
    # ends and overstates the correlated target's variances (by ~1.8x here).
    cov, minv = np.array([[1.0, 2.7], [2.7, 9.0]]), np.array([2.0, 0.5])
    t = nuts.GaussianTarget(cov, minv)
    orig = nuts.uniform

    def biased(seed, it, purpose, index):
        return 0.0 if purpose == philox.PURPOSE_NUTS_MERGE else orig(seed, it, purpose, index)
    samples = []
    nuts.uniform = biased
    try:
        nuts.nuts_run(t, nuts.VecState(np.zeros(2)), 3000, 0.3, 17,
                      callback=lambda it, q, st: samples.append(q.x.copy()))
    finally:
        nuts.uniform = orig
    with pytest.raises(AssertionError):
        _moments_ok(samples[100:], cov)


def test_tree_bookkeeping():
    t = nuts.GaussianTarget(np.diag([1.0, 4.0]), np.ones(2))
    steps = []
    nuts.nuts_run(t, nuts.VecState(np.array([0.3, -1.0])), 300, 0.25, 5, max_depth=6,
                  callback=lambda it, q, st: steps.append(st))
    for it, st in enumerate(steps):
        assert 1 <= st.depth <= 6
        # every doubling but the last is complete: 2^j leaves each
        full = 2 ** (st.depth - 1) - 1
        assert full < st.leaves <= 2 ** st.depth - 1
        j, pos = st.where
        if j >= 0:
            # the sample is a leaf of a doubling that completed
            assert j < st.depth and 0 <= pos < 2 ** j
            assert j < st.depth - 1 or st.leaves == 2 ** st.depth - 1
        assert 0.0 <= st.alpha <= 1.0
    # the depth cap holds
    capped = []
    nuts.nuts_run(t, nuts.VecState(np.array([0.3, -1.0])), 20, 0.01, 5, max_depth=3,
                  callback=lambda it, q, st: capped.append(st))
    assert all(st.depth == 3 and st.leaves == 7 for st in capped)


def test_direction_and_slice_draws():
    # the direction of doubling j is -1 iff its uniform is <= 1/2, and the
    # slice variable is ln U - H0 with U the accept-purpose uniform
    t = nuts.GaussianTarget(np.array([[1.0]]), np.array([1.0]))
    q = nuts.VecState(np.array([0.7]))
    c = t.gradient(q)
    step = nuts.nuts_iteration(t, q, c, 0.5, 42, 3, max_depth=1)
    r0 = t.momenta(42, 3)
    assert abs(step.h0 - (c[0] + t.kinetic(r0))) < 1e-15
    v = -1 if nuts.uniform(42, 3, philox.PURPOSE_NUTS_DIR, 0) <= 0.5 else 1
    q1, p1, c1 = t.leapfrog(q, r0, v * 0.5, c)
    h1 = c1[0] + t.kinetic(p1)
    ln_u = math.log(nuts.uniform(42, 3, philox.PURPOSE_ACCEPT, 0)) - step.h0
    moved = step.where == (0, 0)
    # one doubling of one leaf: the chain moves to it iff it is in the slice
    # (n' = 1 = n, so the move has probability one)
    assert moved == (ln_u <= -h1)
    assert abs(step.alpha - min(1.0, math.exp(step.h0 - h1))) < 1e-15


def _prior_only(n_grid=8, box=200.0):
    m = mocks.make_mock(n_grid, box, 1, 50.0, seed=1)
    kw = m.problem_kwargs()
    for key in ("mu", "sigma_mu", "cz", "sigma_cz"):
        kw[key] = np.zeros(0)
    kw["rhat"] = np.zeros((0, 3))
    kw["sample_sigma_nl"] = False
    return m, model.Problem(**kw)


@pytest.mark.slow
def test_nuts_prior_only_recovers_mode_variance():
    m, prob = _prior_only(n_grid=8)
    n = prob.n_grid
    var = model.mode_variance(prob)
    rng = np.random.default_rng(0)
    x0 = hmc.pack_modes(n, np.sqrt(var / 2) * (rng.standard_normal(var.shape) + 1j * rng.standard_normal(var.shape)))
    q0 = hmc.State(hmc.unpack_modes(n, x0), np.zeros(0), 1.0)
    samples = []
    res = nuts.nuts_run(nuts.PosteriorTarget(prob), q0, 200, 0.4, 3,
                        callback=lambda it, q, st: samples.append(q.modes.copy()))
    keep = hmc.canonical_mask(n)
    ratio = np.array([np.abs(s[keep]) ** 2 / var[keep] for s in samples[20:]])
    assert abs(ratio.mean() - 1.0) < 0.05, ratio.mean()
    assert res.depth.mean() >= 2


@pytest.mark.slow
def test_nuts_chain_mean_converges_to_wiener_filter():
    m = mocks.make_mock(16, 200.0, 300, 80.0, "sphere", (0.2, 0.2), seed=21)
    kw = m.problem_kwargs()
    kw.update(sample_distances=False, sample_sigma_nl=False)
    prob = model.Problem(**kw)
    n, s = 16, 1.5
    x_wf, cdiag, _, _ = wiener.wiener_filter(prob, m.d_true, s)
    rng = np.random.default_rng(5)
    x0 = x_wf + np.sqrt(cdiag) * rng.standard_normal(len(cdiag))
    q0 = hmc.State(hmc.unpack_modes(n, x0), m.d_true.copy(), s)
    samples = []
    # eps below the leapfrog's stability limit 2 / omega_max (omega_max ~ 9.4
    # in whitened units)
    res = nuts.nuts_run(nuts.PosteriorTarget(prob), q0, 300, 0.15, 8,
                        callback=lambda it, q, st: samples.append(hmc.pack_modes(n, q.modes)))
    x = np.array(samples)
    # NUTS samples of this Gaussian are antithetic (tau < 1)
    tau = integrated_autocorrelation_time(x, floor=0.05)
    z = (x.mean(axis=0) - x_wf) / np.sqrt(cdiag * tau / len(x))
    assert 0.75 <= np.mean(z * z) <= 1.3, np.mean(z * z)
    assert np.abs(z).max() < 5.5
    # and the posterior covariance: the whitened variance of every mode is 1
    white = ((x - x_wf) ** 2 / cdiag).mean()
    assert abs(white - 1.0) < 0.03, white
    assert np.array_equal(res.state.dist, m.d_true) and res.state.s == s


@pytest.mark.slow
def test_nuts_dual_averaging_reaches_the_target():
    # modes and sigma_NL sampled (distances frozen: with them the adapted step
    # is tiny and every tree reaches the depth cap, see the design notes)
    m = mocks.make_mock(8, 200.0, 40, 80.0, "sphere", (0.2, 0.2), seed=3)
    kw = m.problem_kwargs()
    kw.update(sample_distances=False)
    prob = model.Problem(**kw)
    q0 = hmc.State(hmc.symmetrise(8, m.dhat_true), m.d_true.copy(), 1.3)
    res = nuts.nuts_run(nuts.PosteriorTarget(prob), q0, 160, 0.5, 11, warmup=80, max_depth=7)
    assert 0.5 < res.alpha[80:].mean() < 0.85, res.alpha[80:].mean()
    assert res.eps > 0
