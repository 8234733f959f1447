"""Philox4x32-10 counter-based generator, written from its published definition.

Oracle module (test infrastructure only; the product path never imports it).

Definition followed: J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11 -- the Philox-4x32 bijection
with 10 rounds.  Each round multiplies counter words 0 and 2 by the two
multipliers, forms the new counter from the high/low halves xor-ed with the
other two words and the round key, and the key is bumped by the two Weyl
constants between rounds.

The paper being reproduced does not say how its random numbers are drawn; the
reading used on both sides (oracle and device) is: key = (low 32 bits of the
seed, high 32 bits of the seed + grain index), counter = (stream tag, species |
purpose << 8, particle slot, draw block).  A uniform u32 ``u`` becomes the double
``(u + 0.5) * 2**-32`` in the open interval (0, 1).
"""
import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint32(0x9E3779B9)
W1 = np.uint32(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10.  All inputs are broadcast to uint32 arrays.

    Returns four uint32 arrays (the output block)."""
    c0, c1, c2, c3 = (np.asarray(v, dtype=np.uint64) & _MASK for v in (c0, c1, c2, c3))
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    k0 = np.asarray(k0, dtype=np.uint64) & _MASK
    k1 = np.asarray(k1, dtype=np.uint64) & _MASK
    for rnd in range(10):
        p0 = M0 * c0            # < 2**64, exact in uint64
        p1 = M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
        if rnd < 9:
            k0 = (k0 + np.uint64(W0)) & _MASK
            k1 = (k1 + np.uint64(W1)) & _MASK
    return tuple(np.asarray(v, dtype=np.uint32) for v in (c0, c1, c2, c3))


def to_unit(u):
    """uint32 -> double in (0, 1): (u + 0.5) * 2**-32."""
    return (np.asarray(u, dtype=np.float64) + 0.5) * (1.0 / 4294967296.0)


def key_for(seed, grain):
    """Key words for a (seed, grain) pair: (lo32(seed), hi32(seed) + grain)."""
    seed = int(seed)
    return seed & 0xFFFFFFFF, ((seed >> 32) + int(grain)) & 0xFFFFFFFF
