"""Counter-based random numbers of the oracle (written independently of the
device library; both follow the published definitions).

* Philox4x32-10: Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
  easy as 1, 2, 3", SC'11 (2011). Ten rounds; multipliers 0xD2511F53,
  0xCD9E8D57; Weyl key increments 0x9E3779B9, 0xBB67AE85.
* SplitMix64 finaliser: Steele, Lea, Flood, "Fast splittable pseudorandom
  number generators", OOPSLA 2014.
* Box-Muller: Box & Muller, Ann. Math. Statist. 29 (1958) 610.

The Gaussian sketch Omega of the randomized SVD (Sec. 4: a matrix of
Gaussian random numbers; Halko et al. 2011, Example 1.6) is drawn from these.
"""
from __future__ import annotations

import numpy as np

M0, M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK32 = np.uint64(0xFFFFFFFF)
GOLDEN = 0x9E3779B97F4A7C15
U64 = (1 << 64) - 1


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10. Counters are uint32-valued arrays (any int
    dtype), keys python ints. Returns four uint64 arrays holding uint32 words."""
    c0 = np.asarray(c0, dtype=np.uint64) & MASK32
    c1 = np.asarray(c1, dtype=np.uint64) & MASK32
    c2 = np.asarray(c2, dtype=np.uint64) & MASK32
    c3 = np.asarray(c3, dtype=np.uint64) & MASK32
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    k0, k1 = int(k0) & 0xFFFFFFFF, int(k1) & 0xFFFFFFFF
    for r in range(10):
        if r > 0:
            k0 = (k0 + W0) & 0xFFFFFFFF
            k1 = (k1 + W1) & 0xFFFFFFFF
        p0 = M0 * c0            # < 2^64: exact in uint64
        p1 = M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0), lo1, hi0 ^ c3 ^ np.uint64(k1), lo0)
    return c0, c1, c2, c3


def splitmix64_mix(z):
    """SplitMix64 output function on a python int (mod 2^64)."""
    z &= U64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & U64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & U64
    return z ^ (z >> 31)


def hash_words(seed, words):
    """Fold a sequence of integers into one 64-bit value:
    h <- mix(h + GOLDEN + w) for each word w (taken mod 2^64)."""
    h = int(seed) & U64
    for w in words:
        h = splitmix64_mix((h + GOLDEN + (int(w) & U64)) & U64)
    return h


def unit_from_hash(h):
    """Top 53 bits as a double in [0, 1)."""
    return (int(h) >> 11) * (1.0 / 9007199254740992.0)


def gaussian_block(seed, c1, c2, c3, nelem):
    """``nelem`` N(0,1) draws for element indices 0..nelem-1 of one stream.

    Element e uses counter (e >> 1, c1, c2, c3) with key (seed lo, seed hi);
    the four words give u1 = (w0>>5 * 2^26 + w1>>6) 2^-53 and u2 likewise
    from (w2, w3); r = sqrt(-2 ln(1 - u1)); even e takes r cos(2 pi u2),
    odd e takes r sin(2 pi u2)."""
    if nelem == 0:
        return np.zeros(0)
    seed = int(seed) & U64
    k0, k1 = seed & 0xFFFFFFFF, seed >> 32
    npair = (nelem + 1) // 2
    pair = np.arange(npair, dtype=np.uint64)
    r0, r1, r2, r3 = philox4x32_10(pair, c1, c2, c3, k0, k1)
    sc = 1.0 / 9007199254740992.0
    u1 = ((r0 >> np.uint64(5)).astype(np.float64) * 67108864.0
          + (r1 >> np.uint64(6)).astype(np.float64)) * sc
    u2 = ((r2 >> np.uint64(5)).astype(np.float64) * 67108864.0
          + (r3 >> np.uint64(6)).astype(np.float64)) * sc
    rad = np.sqrt(-2.0 * np.log(1.0 - u1))
    ang = 2.0 * np.pi * u2
    out = np.empty(2 * npair)
    out[0::2] = rad * np.cos(ang)
    out[1::2] = rad * np.sin(ang)
    return out[:nelem]


def gaussian_matrix(seed, c1, c2, c3, n, k):
    """n x k row-major Gaussian matrix, element (r, c) at index r*k + c."""
    return gaussian_block(seed, c1, c2, c3, n * k).reshape(n, k)
