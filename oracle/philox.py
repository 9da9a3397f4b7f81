"""Philox4x32-10 counter-based generator and Box-Muller normals (oracle side).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The HIP library draws the random vectors that the method itself needs (the
restart vectors after a Lanczos breakdown, and the start vector / sketch when
the caller passes none) from this generator, so the oracle implements the same
published definition independently: Salmon, Moraes, Dror, Shaw, "Parallel
random numbers: as easy as 1, 2, 3", SC'11 (Philox-4x32, 10 rounds,
multipliers 0xD2511F53 / 0xCD9E8D57, Weyl increments 0x9E3779B9 / 0xBB67AE85).

Stream layout (shared definition): the normal number with index e of stream
``stream`` under 64-bit ``seed`` comes from the block counter
(low and high 32 bits of e // 2, stream, 0) with key (seed & 0xffffffff, seed >> 32). The block's
output words w0..w3 give two 53-bit uniforms
u_a = ((w0 >> 5) * 2^26 + (w1 >> 6)) * 2^-53, u_b likewise from (w2, w3);
with r = sqrt(-2 ln(1 - u_a)) and t = 2 pi u_b the pair is
(r cos t, r sin t); index e takes the first member when e is even.
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """Philox4x32-10 on arrays of counters.

    ctr: uint32-valued array of shape (..., 4); key: 2 ints. Returns uint32
    words (..., 4).
    """
    c = np.asarray(ctr, dtype=np.uint64) & MASK
    c0, c1, c2, c3 = c[..., 0], c[..., 1], c[..., 2], c[..., 3]
    k0, k1 = int(key[0]) & 0xFFFFFFFF, int(key[1]) & 0xFFFFFFFF
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + W0) & 0xFFFFFFFF
            k1 = (k1 + W1) & 0xFFFFFFFF
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0)), lo1, (hi0 ^ c3 ^ np.uint64(k1)), lo0
    return np.stack([c0, c1, c2, c3], axis=-1).astype(np.uint32)


def normals(count: int, seed: int, stream: int) -> np.ndarray:
    """``count`` standard normals of (seed, stream) per the layout above."""
    nblk = (count + 1) // 2
    b = np.arange(nblk, dtype=np.uint64)
    ctr = np.zeros((nblk, 4), dtype=np.uint64)
    ctr[:, 0] = b & MASK
    ctr[:, 1] = b >> np.uint64(32)
    ctr[:, 2] = stream & 0xFFFFFFFF
    ctr[:, 3] = 0
    w = philox4x32_10(ctr, (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)).astype(np.uint64)
    two53 = 2.0 ** -53
    ua = ((w[:, 0] >> np.uint64(5)).astype(np.float64) * 67108864.0
          + (w[:, 1] >> np.uint64(6)).astype(np.float64)) * two53
    ub = ((w[:, 2] >> np.uint64(5)).astype(np.float64) * 67108864.0
          + (w[:, 3] >> np.uint64(6)).astype(np.float64)) * two53
    rr = np.sqrt(-2.0 * np.log(1.0 - ua))
    t = 2.0 * np.pi * ub
    out = np.empty(2 * nblk)
    out[0::2] = rr * np.cos(t)
    out[1::2] = rr * np.sin(t)
    return out[:count]
