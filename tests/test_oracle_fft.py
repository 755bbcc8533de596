"""Pins of the oracle's own FFT (the transform of eq:vel-field and its adjoint)."""
import numpy as np
import pytest

from oracle import fft


@pytest.mark.parametrize("n", [1, 2, 4, 8, 16])
def test_fft_matches_direct_dft(n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal((n, n, n)) + 1j * rng.standard_normal((n, n, n))
    ref_f = fft.direct_dft(x, -1)
    ref_b = fft.direct_dft(x, +1)
    scale = np.abs(ref_f).max()
    assert np.abs(fft.fftn(x) - ref_f).max() <= 1e-13 * scale * max(1, n)
    assert np.abs(fft.ifftn_unnormalised(x) - ref_b).max() <= 1e-13 * scale * max(1, n)


def test_direct_dft_is_the_textbook_sum():
    # The brute-force reference itself, one coefficient at a time on 4^3.
    rng = np.random.default_rng(0)
    n = 4
    x = rng.standard_normal((n, n, n)) + 1j * rng.standard_normal((n, n, n))
    ref = fft.direct_dft(x, -1)
    j = np.arange(n)
    for k in [(0, 0, 0), (1, 2, 3), (3, 0, 1), (2, 2, 2)]:
        phase = np.exp(-2j * np.pi * (k[0] * j[:, None, None] + k[1] * j[None, :, None]
                                      + k[2] * j[None, None, :]) / n)
        assert abs(ref[k] - np.sum(x * phase)) < 1e-12


def test_fft_matches_library_routine():
    rng = np.random.default_rng(5)
    x = rng.standard_normal((32, 16, 8)) + 1j * rng.standard_normal((32, 16, 8))
    ref = np.fft.fftn(x)
    assert np.abs(fft.fftn(x) - ref).max() <= 1e-12 * np.abs(ref).max()
    refb = np.fft.ifftn(x) * x.size
    assert np.abs(fft.ifftn_unnormalised(x) - refb).max() <= 1e-12 * np.abs(refb).max()


def test_parseval_and_inverse():
    rng = np.random.default_rng(9)
    x = rng.standard_normal((16, 16, 16))
    xk = fft.fftn(x)
    assert abs(np.sum(x ** 2) - np.sum(np.abs(xk) ** 2) / x.size) < 1e-10 * np.sum(x ** 2)
    back = fft.ifftn_unnormalised(xk) / x.size
    assert np.abs(back - x).max() < 1e-13


def test_rejects_non_power_of_two():
    with pytest.raises(ValueError):
        fft.fftn(np.zeros((6, 6, 6)))
