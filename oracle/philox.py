"""Counter-based Philox4x32-10 generator and Box-Muller normals (reference form).

Written from the published definition (Salmon, Moraes, Dror & Shaw, "Parallel
random numbers: as easy as 1, 2, 3", SC 2011): ten rounds of the 4x32 Philox
S-box with multipliers 0xD2511F53 / 0xCD9E8D57 and Weyl key increments
0x9E3779B9 / 0xBB67AE85. Pure Python integers; slow and only for tests.

Probe draws: the pair index j of a column-major n x m block (entries 2j and
2j+1) uses counter (j_lo, j_hi, stream_lo, stream_hi) and key (seed_lo,
seed_hi). The four output words give two 53-bit uniforms
u = ((hi << 32 | lo) >> 11 + 0.5) * 2^-53 in (0, 1), and Box-Muller turns
them into N(0, 1) values r cos(2 pi u2), r sin(2 pi u2) with
r = sqrt(-2 ln u1).
"""

from __future__ import annotations

import math

import numpy as np

_M0 = 0xD2511F53
_M1 = 0xCD9E8D57
_W0 = 0x9E3779B9
_W1 = 0xBB67AE85
_MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """Return the four 32-bit output words for counter ctr (4 words), key (2 words)."""
    c0, c1, c2, c3 = (int(v) & _MASK for v in ctr)
    k0, k1 = (int(v) & _MASK for v in key)
    for r in range(10):
        if r:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        p0 = _M0 * c0
        p1 = _M1 * c2
        hi0, lo0 = p0 >> 32, p0 & _MASK
        hi1, lo1 = p1 >> 32, p1 & _MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
    return c0, c1, c2, c3


def _u53(lo: int, hi: int) -> float:
    v = ((hi << 32) | lo) >> 11
    return (v + 0.5) * 2.0 ** -53


def normal_pair(j: int, seed: int, stream: int):
    """The two N(0,1) values of pair index j."""
    x0, x1, x2, x3 = philox4x32_10(
        (j & _MASK, (j >> 32) & _MASK, stream & _MASK, (stream >> 32) & _MASK),
        (seed & _MASK, (seed >> 32) & _MASK))
    u1 = _u53(x0, x1)
    u2 = _u53(x2, x3)
    r = math.sqrt(-2.0 * math.log(u1))
    t = 2.0 * math.pi * u2
    return r * math.cos(t), r * math.sin(t)


def normal_block(n: int, m: int, seed: int, stream: int = 0) -> np.ndarray:
    """Column-major n x m block of N(0,1) draws (entry e = col * n + row)."""
    total = n * m
    flat = np.empty(total + (total & 1))
    for j in range((total + 1) // 2):
        flat[2 * j], flat[2 * j + 1] = normal_pair(j, seed, stream)
    return flat[:total].reshape((m, n)).T.copy(order="F")


def philox4x32_10_vec(c0, c1, c2, c3, k0, k1):
    """Vectorised philox4x32_10 over uint64 arrays holding 32-bit words (same definition)."""
    M = np.uint64(_MASK)
    c0, c1, c2, c3 = (np.asarray(v, dtype=np.uint64) & M for v in (c0, c1, c2, c3))
    k0 = np.uint64(int(k0) & _MASK)
    k1 = np.uint64(int(k1) & _MASK)
    for r in range(10):
        if r:
            k0 = (k0 + np.uint64(_W0)) & M
            k1 = (k1 + np.uint64(_W1)) & M
        p0 = np.uint64(_M0) * c0
        p1 = np.uint64(_M1) * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & M
        hi1, lo1 = p1 >> np.uint64(32), p1 & M
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
    return c0, c1, c2, c3


def normal_columns(n: int, cols, seed: int, stream: int = 0) -> np.ndarray:
    """Selected columns of the column-major N(0,1) block of normal_block (vectorised)."""
    cols = np.asarray(cols, dtype=np.int64)
    e = (cols[None, :] * n + np.arange(n)[:, None]).ravel(order="F")
    j = (e // 2).astype(np.uint64)
    x0, x1, x2, x3 = philox4x32_10_vec(j & np.uint64(_MASK), j >> np.uint64(32),
                                      np.full_like(j, stream & _MASK),
                                      np.full_like(j, (stream >> 32) & _MASK),
                                      seed & _MASK, (seed >> 32) & _MASK)
    u1 = (((x1 << np.uint64(32)) | x0) >> np.uint64(11)).astype(np.float64)
    u2 = (((x3 << np.uint64(32)) | x2) >> np.uint64(11)).astype(np.float64)
    u1 = (u1 + 0.5) * 2.0 ** -53
    u2 = (u2 + 0.5) * 2.0 ** -53
    r = np.sqrt(-2.0 * np.log(u1))
    t = 2.0 * np.pi * u2
    z = np.where(e % 2 == 0, r * np.cos(t), r * np.sin(t))
    return z.reshape((n, cols.size), order="F")
