"""The oracle chain on linear Gaussian data converges to the Wiener filter.

With distances and sigma_NL frozen the posterior of Section 2 is Gaussian and
its mean is the closed-form Wiener filter; the HMC Monte-Carlo mean
(eq:int_mc) must converge to it with error ~ n_S^-1/2.  16^3 grid, 300 points.
"""
import numpy as np
import pytest

from oracle import hmc, model, wiener
from paper_2203_02369_amd import mocks


def integrated_autocorrelation_time(x, floor=1.0):
    """Geyer's initial monotone sequence estimator, per column of x (n_s, m),
    at least `floor` (below 1 for antithetic chains such as NUTS often gives)."""
    n = x.shape[0]
    xc = x - x.mean(axis=0)
    f = np.fft.rfft(xc, n=2 * n, axis=0)
    ac = np.fft.irfft(f * np.conj(f), axis=0)[:n] / n
    rho = ac / ac[0]
    out = np.empty(x.shape[1])
    for j in range(x.shape[1]):
        pairs = rho[0:n - 1:2, j] + rho[1:n:2, j]
        tau, prev = -1.0, np.inf
        for g in pairs:
            if g <= 0:
                break
            g = min(g, prev)
            prev = g
            tau += 2.0 * g
        out[j] = max(tau, floor)
    return out


@pytest.mark.slow
def test_chain_mean_converges_to_wiener_filter():
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
    # eps below 2/omega_max (omega_max ~ 9.4 in whitened units), eps*L ~ pi/2
    res = hmc.hmc_run(prob, q0, n_iter=800, n_leapfrog=10, eps0=0.15, seed=8, jitter=True,
                      callback=lambda it, q, dh, acc, e: samples.append(hmc.pack_modes(n, q.modes)))
    assert 0.5 < res.accepted.mean() < 0.95
    x = np.array(samples)
    tau = integrated_autocorrelation_time(x)
    z = (x.mean(axis=0) - x_wf) / np.sqrt(cdiag * tau / len(x))
    assert 0.8 <= np.mean(z * z) <= 1.25, np.mean(z * z)
    assert np.abs(z).max() < 5.5
    # the error falls as n_S^-1/2
    err = [np.sqrt(np.mean((x[:k].mean(axis=0) - x_wf) ** 2 / cdiag)) for k in (200, 800)]
    assert 1.5 < err[0] / err[1] < 2.7, err
    # the distances and sigma_NL never moved
    assert np.array_equal(res.state.dist, m.d_true) and res.state.s == s
