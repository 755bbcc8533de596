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


def check_adapted_chain(res, warmup, eps_gpu, dh_gpu, states, h_scale):
    """The tolerances of a chain whose step is adapted (dual averaging).

    dH is held to TOL64 of the Hamiltonian.  The adapted step is a function of
    the dH sequence: with gamma = 0.05, h-bar a weighted mean of the
    acceptance statistics alpha = min(1, exp(-dH)) and log eps_bar a weighted
    mean of mu - sqrt(m)/gamma h-bar_m, |d ln eps| <= (sqrt(W) / gamma)
    max |d dH| over the W adaptation iterations (|d alpha| <= |d dH|), plus
    the rounding of exp and log.  A state after adaptation moved by eps times
    its trajectories, so it carries (d eps / eps) of its displacement from the
    start; each state is compared within TOL64 plus twice that."""
    fin = np.isfinite(res.dh)
    assert np.array_equal(fin, np.isfinite(dh_gpu))
    dh_err = float(np.abs(dh_gpu[fin] - res.dh[fin]).max()) if fin.any() else 0.0
    eps_err = abs(eps_gpu - res.eps) / res.eps
    eps_tol = TOL64 + math.sqrt(warmup) / 0.05 * dh_err
    errs = {"dh": dh_err / h_scale, "eps": eps_err}
    tols = {"dh": TOL64, "eps": eps_tol}
    for name, (got, ref, start) in states.items():
        errs[name] = rel_inf(got, ref)
        tols[name] = TOL64 + 2.0 * eps_err * rel_inf(ref, start) if start is not None else TOL64 + 2.0 * eps_err
    print("adapted chain errors", errs, "tolerances", tols, flush=True)
    for k in errs:
        assert errs[k] <= tols[k], (k, errs[k], tols[k])
