"""Philox4x32-10, written from its published definition (test infrastructure only).

Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as easy as 1, 2, 3" (SC'11),
Sec. 3.2: a counter of four 32-bit words and a key of two 32-bit words go through ten
rounds. Each round multiplies counter words 0 and 2 by fixed odd constants into 64-bit
products, and builds the next counter from the high halves XORed with the other two words
and the round key, and the low halves. The key is advanced by the Weyl constants
(golden ratio and sqrt(3) - 1, scaled to 2^32) between rounds.

All arithmetic is on NumPy ``uint64`` arrays holding 32-bit values, so products of two
32-bit words are exact.
"""
import numpy as np

_MASK = np.uint64(0xFFFFFFFF)
_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint64(0x9E3779B9)
_W1 = np.uint64(0xBB67AE85)
_S32 = np.uint64(32)


def philox4x32_10(ctr, key):
    """Apply Philox4x32-10 to counters ``ctr`` = (c0, c1, c2, c3) under ``key`` = (k0, k1).

    Each of the six inputs is an integer or an integer array (broadcast together); every
    value must lie in [0, 2^32). Returns four ``uint64`` arrays (x0, x1, x2, x3), each word
    in [0, 2^32).
    """
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) for c in ctr)
    k0, k1 = (np.asarray(k, dtype=np.uint64) for k in key)
    c0, c1, c2, c3, k0, k1 = np.broadcast_arrays(c0, c1, c2, c3, k0, k1)
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        p0 = _M0 * c0
        p1 = _M1 * c2
        hi0, lo0 = p0 >> _S32, p0 & _MASK
        hi1, lo1 = p1 >> _S32, p1 & _MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def seed_key(seed):
    """Split a 64-bit seed into the Philox key words (low word first)."""
    seed = int(seed)
    if not 0 <= seed < 2**64:
        raise ValueError("seed must be in [0, 2^64)")
    return seed & 0xFFFFFFFF, seed >> 32


def mode_words(seed, ix, iy, iz, stream=0):
    """The two 32-bit words that drive the normal pair of half-grid mode (ix, iy, iz).

    Counter = (iz >> 1, iy, ix, stream), key = the seed's two words. One Philox call serves
    the two neighbouring modes iz = 2q and 2q + 1: the even one takes words (x0, x1), the
    odd one (x2, x3). The first word feeds the Box-Muller radius, the second its angle.
    The fourth counter word separates the streams of the box kinds: 0 for the cubic box,
    1 for the layers of the 2-D (hybrid) method, 2 for the flat N x N x M box.
    """
    ix = np.asarray(ix, dtype=np.uint64)
    iy = np.asarray(iy, dtype=np.uint64)
    iz = np.asarray(iz, dtype=np.uint64)
    k0, k1 = seed_key(seed)
    x0, x1, x2, x3 = philox4x32_10((iz >> np.uint64(1), iy, ix, np.uint64(stream)), (k0, k1))
    odd = (iz & np.uint64(1)) == np.uint64(1)
    a = np.where(odd, x2, x0)
    b = np.where(odd, x3, x1)
    return a, b
