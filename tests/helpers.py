"""Shared test helpers: layout conversion between the oracle and the library.

The oracle stores the half spectrum with kz in [0, N/2]; the library drops
the kz = N/2 plane (it holds only excluded Nyquist modes, always zero).
"""
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
