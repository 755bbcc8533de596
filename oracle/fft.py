"""Oracle discrete Fourier transforms (test infrastructure only).

The velocity field of eq:vel-field is an inverse Fourier transform of the
Fourier modes; the gradient of the posterior needs the transposed operator
(Section 4 states that only the gradient of the inverse transform had to be
written by hand).  This module is the oracle's own transform: a plain radix-2
Cooley-Tukey FFT in self-sorting (Stockham) order, vectorised over every
axis but the one being transformed, written for readability rather than speed.

Conventions (fixed for the whole oracle):
  forward   X[k] = sum_n x[n] exp(-2 pi i k n / N)            (unnormalised)
  backward  x[n] = sum_k X[k] exp(+2 pi i k n / N)            (unnormalised)
so backward(forward(x)) = N x.  The 3-D field transform of the oracle divides
the backward sum by N^3 where it defines delta(x) from its modes.

Pinned in tests against a brute-force direct DFT on 4^3, 8^3 and 16^3 grids,
against Parseval's identity and against numpy.fft (a library routine).
"""
import numpy as np


def _fft_last_axis(x, sign):
    """Radix-2 transform of length N = 2^m along the last axis.

    Stockham (self-sorting) form of the Cooley-Tukey recursion: after the
    stage that builds sub-transforms of length 2L from pairs of length-L
    sub-transforms E (even samples) and O (odd samples),
        X[k]     = E[k] + w^k O[k]
        X[k + L] = E[k] - w^k O[k],   w = exp(sign 2 pi i / (2L)),  0 <= k < L,
    the results are already in natural order, so no bit reversal is needed.
    """
    y = np.ascontiguousarray(x, dtype=np.complex128)
    n = y.shape[-1]
    if n < 1 or n & (n - 1):
        raise ValueError("oracle FFT length must be a power of two, got %d" % n)
    batch = y.shape[:-1]
    half = 1
    while half < n:
        groups = n // (2 * half)
        # The array holds 2*groups finished sub-transforms of length `half`;
        # the two that combine into output group g sit n/2 apart, at
        # offsets g*half and g*half + n/2.
        a = y.reshape(batch + (2, groups, half))
        w = np.exp(sign * 2j * np.pi * np.arange(half) / (2 * half))
        even = a[..., 0, :, :]
        odd = a[..., 1, :, :] * w
        out = np.empty(batch + (groups, 2, half), dtype=np.complex128)
        np.add(even, odd, out=out[..., 0, :])
        np.subtract(even, odd, out=out[..., 1, :])
        y = out.reshape(batch + (n,))
        half *= 2
    return y


def fft_axis(x, axis, sign=-1):
    """Unnormalised transform along one axis; sign=-1 forward, +1 backward."""
    x = np.moveaxis(np.asarray(x, dtype=np.complex128), axis, -1)
    return np.moveaxis(_fft_last_axis(x, sign), -1, axis)


def fftn(x):
    """Forward unnormalised 3-D transform (all three axes)."""
    y = np.asarray(x, dtype=np.complex128)
    for ax in range(y.ndim):
        y = fft_axis(y, ax, -1)
    return y


def ifftn_unnormalised(x):
    """Backward unnormalised 3-D transform: sum_k X[k] exp(+i k.x)."""
    y = np.asarray(x, dtype=np.complex128)
    for ax in range(y.ndim):
        y = fft_axis(y, ax, +1)
    return y


def direct_dft(x, sign=-1):
    """Brute-force N^d-term DFT over every axis, by explicit DFT matrices.

    Used only to pin the FFT above on small grids.
    """
    y = np.asarray(x, dtype=np.complex128)
    for ax in range(y.ndim):
        n = y.shape[ax]
        j = np.arange(n)
        mat = np.exp(sign * 2j * np.pi * np.outer(j, j) / n)
        y = np.moveaxis(np.tensordot(mat, np.moveaxis(y, ax, 0), axes=(1, 0)), 0, ax)
    return y
