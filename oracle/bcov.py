"""Background-error covariance square root L (B = L L^T) for periodic 1-D grids.

Section 2.1 / eq. (3): the inner loop works in the control variable dz with
dx = L dz and B = L L^T. The paper asks for Gaussian correlations but does not
say how the square root is built. Reading used here: L is the symmetric
circulant whose row is the truncated kernel l_d = c exp(-d^2 / ell^2),
|d| <= w = ceil(6.25 ell), with c fixed so that sum_d l_d^2 = sigma_b^2; then
B := L L^T = L^2 has, on an unbounded grid, the Gaussian correlation
exp(-d^2 / (2 ell^2)). On a periodic grid taps that wrap onto the same offset
are summed.
"""

from __future__ import annotations

import math

import numpy as np


def gaussian_taps(ell: float, sigma_b: float) -> np.ndarray:
    """Half-kernel taps l_0..l_w of the Gaussian square root (see module doc)."""
    w = int(math.ceil(6.25 * ell))
    d = np.arange(-w, w + 1, dtype=np.float64)
    k = np.exp(-(d * d) / (ell * ell))
    c = sigma_b / math.sqrt(float(np.sum(k * k)))
    return (c * k)[w:].copy()


def dense_L(n: int, taps: np.ndarray) -> np.ndarray:
    """Dense n x n matrix of the symmetric circulant with half-kernel ``taps``."""
    w = taps.size - 1
    L = np.zeros((n, n))
    for i in range(n):
        for d in range(-w, w + 1):
            L[i, (i + d) % n] += taps[abs(d)]
    return L


def apply_L(x: np.ndarray, taps: np.ndarray) -> np.ndarray:
    """L x for 1-D x (n,) or column block (n, m), as an explicit tap loop."""
    w = taps.size - 1
    out = taps[0] * x
    for d in range(1, w + 1):
        out = out + taps[d] * (np.roll(x, -d, axis=0) + np.roll(x, d, axis=0))
    return out
