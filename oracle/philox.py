"""Oracle counter-based random numbers (test infrastructure only).

HMC draws fresh momenta for every trajectory and a uniform number for the
Metropolis-Hastings test (Section 3.2).  For the oracle and the GPU path to
make the same draws, each implements the same published counter-based
generator on its own: Philox4x32-10 (Salmon, Moraes, Dror & Shaw, "Parallel
random numbers: as easy as 1, 2, 3", SC'11).

Round function on the counter (c0, c1, c2, c3) with key (k0, k1):
    (hi0, lo0) = 0xD2511F53 * c0,   (hi1, lo1) = 0xCD9E8D57 * c2   (64-bit products)
    c <- (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0)
and the key is bumped by the Weyl constants (0x9E3779B9, 0xBB67AE85) between
rounds; ten rounds in all.  Pinned by the published known-answer vectors.

Stream layout shared with the GPU path (a reading: the paper states none):
    key     = (seed & 0xffffffff, seed >> 32)
    counter = (index & 0xffffffff, index >> 32, iteration, purpose)
    index of a mode: (kx N + ky) N/2 + kz; of a distance: its catalogue
    position; of sigma_NL and of the accept/jitter draws: 0; of a NUTS
    direction or new-subtree draw: the doubling j; of a NUTS merge: the node
    ((j * 16 + height) << 32) | position.
Uniforms: u = ((x >> 11) + 1) * 2^-53 in (0, 1], x = (w1 << 32) | w0 built
from two 32-bit output words.  Normals: Box-Muller on two such uniforms.
"""
import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK32 = np.uint64(0xFFFFFFFF)

PURPOSE_MODES = 0
PURPOSE_DIST = 1
PURPOSE_SNL = 2
PURPOSE_ACCEPT = 3
PURPOSE_JITTER = 4
# the No-U-Turn sampler's draws: direction of each doubling (index: the
# doubling), the merge of the two halves of a subtree (index: doubling,
# height and position of the node) and the move to a new subtree's sample
# (index: the doubling)
PURPOSE_NUTS_DIR = 5
PURPOSE_NUTS_MERGE = 6
PURPOSE_NUTS_TOP = 7
# momenta of the cosmological coordinates (index 0: the pair (u8, phi);
# index 1: eta from the first of its pair)
PURPOSE_COSMO = 8


def philox4x32_10(counter, key):
    """Vectorised Philox4x32-10.

    counter: uint array (..., 4); key: two ints.  Returns uint32 array (..., 4).
    """
    c = np.asarray(counter, dtype=np.uint64) & MASK32
    c0, c1, c2, c3 = c[..., 0], c[..., 1], c[..., 2], c[..., 3]
    k0, k1 = int(key[0]) & 0xFFFFFFFF, int(key[1]) & 0xFFFFFFFF
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + W0) & 0xFFFFFFFF
            k1 = (k1 + W1) & 0xFFFFFFFF
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0), lo1,
                          hi0 ^ c3 ^ np.uint64(k1), lo0)
    return np.stack([c0, c1, c2, c3], axis=-1).astype(np.uint32)


def draw_words(seed, iteration, purpose, index):
    """Philox output words for the given stream coordinates.

    index: integer array of element indices.  Returns uint32 (len(index), 4).
    """
    index = np.asarray(index, dtype=np.uint64)
    ctr = np.zeros(index.shape + (4,), dtype=np.uint64)
    ctr[..., 0] = index & MASK32
    ctr[..., 1] = index >> np.uint64(32)
    ctr[..., 2] = np.uint64(iteration)
    ctr[..., 3] = np.uint64(purpose)
    seed = int(seed)
    return philox4x32_10(ctr, (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF))


def uniform53(w_lo, w_hi):
    """((x >> 11) + 1) * 2^-53 with x = (w_hi << 32) | w_lo; result in (0, 1]."""
    x = (np.asarray(w_hi, dtype=np.uint64) << np.uint64(32)) | np.asarray(w_lo, dtype=np.uint64)
    return ((x >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0 ** -53


def normal_pair(words):
    """Two standard normals per Philox output (Box-Muller on words 0-1, 2-3)."""
    u1 = uniform53(words[..., 0], words[..., 1])
    u2 = uniform53(words[..., 2], words[..., 3])
    rad = np.sqrt(-2.0 * np.log(u1))
    ang = 2.0 * np.pi * u2
    return rad * np.cos(ang), rad * np.sin(ang)
