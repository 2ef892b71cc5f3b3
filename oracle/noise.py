"""Seeded white noise for the initial conditions (FP64).

Test infrastructure only (see the package docstring).

The paper states only that runs sharing a seed share their initial Gaussian field, which
cancels cosmic variance between them (Sec. 2.3).  For the oracle and the GPU path to
evolve the *same* realization, both draw the noise from one counter-based generator:

  * Philox4x64 with 10 rounds (Salmon, Moraes, Dror & Shaw 2011, "Parallel random
    numbers: as easy as 1, 2, 3"), key = (seed, 0), counter = (cell index, 0, 0, 0);
  * from the first two 64-bit outputs r0, r1 of a block, the top 24 bits give two
    uniforms that are exact in both float32 and float64:
        u1 = (floor(r0 / 2^40) + 1) / 2^24   in (0, 1]
        u2 =  floor(r1 / 2^40)      / 2^24   in [0, 1)
  * Box-Muller: w = sqrt(-2 ln u1) cos(2 pi u2), unit-variance Gaussian.

The cell index is the linear Lagrangian index (i * N + j) * N + l, z fastest.
"""

import numpy as np

_MASK32 = np.uint64(0xFFFFFFFF)
_SH32 = np.uint64(32)
PHILOX_M0 = np.uint64(0xD2E7470EE14C6C93)
PHILOX_M1 = np.uint64(0xCA5A826395121157)
PHILOX_W0 = np.uint64(0x9E3779B97F4A7C15)
PHILOX_W1 = np.uint64(0xBB67AE8584CAA73B)


def _mulhilo64(a, b):
    """Full 64x64 -> 128-bit product of uint64 arrays, returned as (hi, lo)."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    a0, a1 = a & _MASK32, a >> _SH32
    b0, b1 = b & _MASK32, b >> _SH32
    t = a0 * b0
    u = a1 * b0 + (t >> _SH32)
    v = a0 * b1 + (u & _MASK32)
    hi = a1 * b1 + (u >> _SH32) + (v >> _SH32)
    lo = a * b
    return hi, lo


def philox4x64(counter, key, rounds=10):
    """Philox4x64-R block function on arrays of counters.

    counter: tuple of 4 uint64 arrays (broadcastable); key: tuple of 2 uint64 scalars.
    Returns the 4 output words.
    """
    with np.errstate(over="ignore"):
        c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) for c in counter)
        k0, k1 = np.uint64(key[0]), np.uint64(key[1])
        for _ in range(rounds):
            hi0, lo0 = _mulhilo64(PHILOX_M0, c0)
            hi1, lo1 = _mulhilo64(PHILOX_M1, c2)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
            k0 = k0 + PHILOX_W0
            k1 = k1 + PHILOX_W1
    return c0, c1, c2, c3


def uniforms(index, seed):
    """The two 24-bit uniforms (u1 in (0,1], u2 in [0,1)) of each cell index."""
    index = np.asarray(index, dtype=np.uint64)
    zero = np.zeros_like(index)
    r0, r1, _, _ = philox4x64((index, zero, zero, zero), (seed, 0))
    u1 = ((r0 >> np.uint64(40)).astype(np.float64) + 1.0) * 2.0 ** -24
    u2 = (r1 >> np.uint64(40)).astype(np.float64) * 2.0 ** -24
    return u1, u2


def white_noise(n, seed):
    """Unit-variance Gaussian white noise on an n^3 Lagrangian grid, shape (n, n, n)."""
    index = np.arange(n ** 3, dtype=np.uint64)
    u1, u2 = uniforms(index, seed)
    w = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    return w.reshape(n, n, n)
