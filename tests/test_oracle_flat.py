"""The oracle's flat parameter vector (Section 3.1, eq:q) against a hand
enumeration, the paper's degree-of-freedom count, and round trips."""
import os

import numpy as np

from oracle import hmc
from oracle.model import mode_indices

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "flat_order_n4.txt")


def test_flat_order_matches_hand_enumeration_n4():
    want = np.loadtxt(GOLDEN, dtype=np.int64)
    n = 4
    nx, ny, nz = mode_indices(n)
    # tag each stored entry with its signed wave vector, pack, and read the order back
    tag = nx * 100 + ny * 10 + nz + 1j * (nx * 100 + ny * 10 + nz)
    flat = hmc.pack_modes(n, hmc.symmetrise(n, tag))
    m = len(want)
    assert flat.size == 2 * m
    got = flat[:m].astype(np.int64)
    assert np.array_equal(got, want[:, 0] * 100 + want[:, 1] * 10 + want[:, 2])
    assert np.array_equal(flat[m:], flat[:m])


def test_degrees_of_freedom():
    # (N-1)^3 - 1 real coordinates; about 2 x 10^6 at 128^3 (Section 4)
    for n in (4, 8, 16, 32):
        assert hmc.canonical_mask(n).sum() * 2 == (n - 1) ** 3 - 1
    assert abs(((128 - 1) ** 3 - 1) / 2e6 - 1) < 0.03


def test_state_round_trip():
    n, n_gal = 8, 5
    rng = np.random.default_rng(3)
    modes = hmc.symmetrise(n, rng.standard_normal((n, n, n // 2 + 1)) + 1j * rng.standard_normal((n, n, n // 2 + 1)))
    dist = rng.uniform(10, 100, n_gal)
    vec = hmc.pack_state(n, modes, dist, 1.7)
    assert vec.size == (n - 1) ** 3 - 1 + n_gal + 1
    m2, d2, s2 = hmc.unpack_state(n, vec, n_gal)
    assert np.array_equal(m2, modes) and np.array_equal(d2, dist) and s2 == 1.7
    f = rng.standard_normal(vec.size)
    assert np.array_equal(hmc.pack_state(n, *hmc.unpack_state(n, f, n_gal)), f)
