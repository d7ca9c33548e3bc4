"""Philox counter-based generator, written generically in the word width.

Test infrastructure only (see ``oracle/__init__.py``).

The paper does not say how random numbers are drawn for its Monte-Carlo
collisions (Section 2, "Methodology"; Section 2a).  This oracle fixes a
counter-based contract so that collisions are reproducible and independent of
particle order: every draw is one Philox block keyed by the particle id and
counted by (step, tag, seed).  Philox is the generator of Salmon et al.,
"Parallel random numbers: as easy as 1, 2, 3" (SC'11): ``R`` rounds of a
multiply-hi/lo S-box plus a Weyl-sequence key schedule.

The same code path serves two instances:

* 4x64-10, which numpy ships as ``numpy.random.Philox``; the tests pin this
  generic implementation bit-for-bit against numpy (numpy advances its counter
  by one before producing its first block);
* 4x32-10, the instance the particle kernels use (32-bit words map onto the
  GPU's 32x32->64 multiply), with the multipliers and Weyl constants of the
  SC'11 paper.
"""
from __future__ import annotations

import numpy as np

# Multipliers and Weyl increments of the SC'11 paper.
PHILOX4x32 = dict(bits=32, M0=0xD2511F53, M1=0xCD9E8D57, W0=0x9E3779B9, W1=0xBB67AE85)
PHILOX4x64 = dict(bits=64, M0=0xD2E7470EE14C6C93, M1=0xCA5A826395121157,
                  W0=0x9E3779B97F4A7C15, W1=0xBB67AE8584CAA73B)


def philox_scalar(ctr, key, params=PHILOX4x32, rounds=10):
    """One Philox block on Python ints (any width).  ``ctr`` has 4 words, ``key`` 2."""
    bits = params["bits"]
    mask = (1 << bits) - 1
    c0, c1, c2, c3 = (int(v) & mask for v in ctr)
    k0, k1 = (int(v) & mask for v in key)
    for _ in range(rounds):
        p0 = params["M0"] * c0
        p1 = params["M1"] * c2
        hi0, lo0 = p0 >> bits, p0 & mask
        hi1, lo1 = p1 >> bits, p1 & mask
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        k0 = (k0 + params["W0"]) & mask
        k1 = (k1 + params["W1"]) & mask
    return c0, c1, c2, c3


def philox4x32(ctr0, ctr1, ctr2, ctr3, key0, key1, rounds=10):
    """Vectorised Philox4x32 on numpy arrays (broadcasting).

    All inputs are reduced to 32 bits; products are formed in uint64, which is
    exact for 32x32-bit operands.  Returns four uint32 arrays.
    """
    m32 = np.uint64(0xFFFFFFFF)
    c0 = np.asarray(ctr0, dtype=np.uint64) & m32
    c1 = np.asarray(ctr1, dtype=np.uint64) & m32
    c2 = np.asarray(ctr2, dtype=np.uint64) & m32
    c3 = np.asarray(ctr3, dtype=np.uint64) & m32
    k0 = np.asarray(key0, dtype=np.uint64) & m32
    k1 = np.asarray(key1, dtype=np.uint64) & m32
    c0, c1, c2, c3, k0, k1 = np.broadcast_arrays(c0, c1, c2, c3, k0, k1)
    M0 = np.uint64(PHILOX4x32["M0"])
    M1 = np.uint64(PHILOX4x32["M1"])
    W0 = np.uint64(PHILOX4x32["W0"])
    W1 = np.uint64(PHILOX4x32["W1"])
    s32 = np.uint64(32)
    for _ in range(rounds):
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> s32, p0 & m32
        hi1, lo1 = p1 >> s32, p1 & m32
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        k0 = (k0 + W0) & m32
        k1 = (k1 + W1) & m32
    return (c0.astype(np.uint32), c1.astype(np.uint32),
            c2.astype(np.uint32), c3.astype(np.uint32))


# ---------------------------------------------------------------------------
# Uniform variates from raw words (the contract both implementations follow).
# ---------------------------------------------------------------------------
TWO_M32 = 2.0 ** -32
TWO_M52 = 2.0 ** -52


def u32(r):
    """(r + 1/2) 2^-32: a double in (0, 1), exact for every 32-bit word."""
    return (np.asarray(r, dtype=np.float64) + 0.5) * TWO_M32


def u52(ra, rb):
    """52-bit uniform in (0, 1) from two words: (((ra << 20) | (rb >> 12)) + 1/2) 2^-52.

    With 52 bits the sum m + 1/2 still fits a double's 53-bit significand, so
    the value is exact and never reaches 0 or 1.
    """
    a = np.asarray(ra, dtype=np.uint64)
    b = np.asarray(rb, dtype=np.uint64)
    m = (a << np.uint64(20)) | (b >> np.uint64(12))
    return (m.astype(np.float64) + 0.5) * TWO_M52
