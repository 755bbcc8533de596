"""Shared test helpers: layout conversion between the oracle and the library.

The oracle stores the half spectrum with kz in [0, N/2]; the library drops
the kz = N/2 plane (it holds only excluded Nyquist modes, always zero).
"""
import math

import numpy as np

from oracle import hmc, model


def to_lib_layout(dhat):
    n = dhat.shape[0]
    return np.ascontiguousarray(dhat[:, :, : n // 2])


def from_lib_layout(arr):
    n = arr.shape[0]
    out = np.zeros((n, n, n // 2 + 1), dtype=np.complex128)
    out[:, :, : n // 2] = arr
    return out


def oracle_problem(mock, **kw):
    args = mock.problem_kwargs()
    args.update(kw)
    return model.Problem(**args)


def start_modes(mock, scale=1.0):
    """A valid start state: the mock field, Hermitian on kz = 0, excluded zeroed."""
    return hmc.symmetrise(mock.n_grid, scale * mock.dhat_true)


def rel_inf(x, ref):
    x = np.asarray(x)
    ref = np.asarray(ref)
    den = np.abs(ref).max()
    return float(np.abs(x - ref).max() / (den if den > 0 else 1.0))


# FP64 tolerance (relative, max-norm per array) of the GPU path against the oracle
TOL64 = 1e-12


def path_length(states):
    """Sum over consecutive states of the max-norm move, relative to the
    last state's largest entry: how far a chain travelled, per array."""
    states = [np.asarray(x) for x in states]
    moved = sum(float(np.abs(b - a).max()) for a, b in zip(states[:-1], states[1:]))
    den = float(np.abs(states[-1]).max())
    return moved / (den if den > 0 else 1.0)


# a trajectory whose energy error exceeds this is rejected whatever its
# rounding (acceptance below e^-10)
DECISIVE_DH = 10.0


def check_adapted_chain(res, warmup, eps_gpu, dh_gpu, states, h_scale):
    """The tolerances of an HMC chain whose step is adapted (dual averaging).

    Accept decisions are compared exactly by the caller.  dH is held to
    TOL64 of the Hamiltonian where it can decide (|dH| <= 10); beyond, the
    trajectory ran past the leapfrog's stability limit, where rounding grows
    exponentially, and it is rejected on both sides.  The adapted step is a
    function of the acceptance statistics alpha = min(1, exp(-dH)): with
    gamma = 0.05, h-bar a weighted mean of the alphas and log eps_bar a
    weighted mean of mu - sqrt(m)/gamma h-bar_m, |d ln eps| <= (sqrt(W) /
    gamma) max |d alpha| over the W adaptation iterations, plus the rounding
    of exp and log.  A chain's state depends on the step through every
    trajectory, each of which moves it by an amount proportional to the
    step: the states carry at most (d eps / eps) times the path the chain
    travelled (`states` maps a name to (gpu, oracle, path length relative to
    the oracle's array)); they are compared within TOL64 plus twice that."""
    fin = np.isfinite(res.dh)
    assert np.array_equal(fin, np.isfinite(dh_gpu))

    def alpha(dh):
        return np.where(np.isfinite(dh), np.minimum(1.0, np.exp(-np.where(np.isfinite(dh), dh, 0.0))), 0.0)
    a_err = float(np.abs(alpha(dh_gpu[:warmup]) - alpha(res.dh[:warmup])).max()) if warmup else 0.0
    eps_err = abs(eps_gpu - res.eps) / res.eps
    dec = fin & (np.abs(np.where(fin, res.dh, 0.0)) <= DECISIVE_DH)
    dh_err = float(np.abs(dh_gpu[dec] - res.dh[dec]).max()) if dec.any() else 0.0
    errs = {"dh": dh_err / h_scale, "eps": eps_err}
    # dH moves with the step as well: |d dH| <= 2 |dH| d ln eps near the
    # leapfrog's eps^2 scaling
    tols = {"dh": TOL64 + 2.0 * DECISIVE_DH * eps_err / h_scale, "eps": TOL64 + math.sqrt(warmup) / 0.05 * a_err}
    for name, (got, ref, path) in states.items():
        errs[name] = rel_inf(got, ref)
        tols[name] = TOL64 + 2.0 * eps_err * path
    print("adapted chain errors", errs, "tolerances", tols, flush=True)
    for k in errs:
        assert errs[k] <= tols[k], (k, errs[k], tols[k])
