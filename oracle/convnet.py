"""Sketch-proposal network and its training loss (test oracle, plain NumPy FP64).

Test infrastructure only: nothing in the product path imports this module.

A 1-D periodic convolutional network maps a background state x (n,) to k basis vectors
N (n, k) that are used as RIOT probes in place of Gaussian ones. Input h_0: each of the C0
input rows (e.g. states along the window) minus its mean, over its standard deviation.
Layers l = 1..L:
  z_l[c, i] = b_l[c] + sum_{c', j} W_l[c, c', j] h_{l-1}[c', (i + j - r) mod n],
  h_l = relu(z_l) for l < L, h_L = z_L,
width 2 r + 1. Output head with S segments (S = 1: N[:, c] = h_L[c, :]): column c S + q of
N is channel c of h_L on the q-th block of n / S consecutive grid points and zero elsewhere,
so that span(N) can hold structures at different places independently.

Loss (subspace capture of the leading Hessian eigenvectors V (n, k) with weights w):
  loss(N) = - sum_i w_i v_i^T P v_i / sum_i w_i,   P = N (N^T N)^{-1} N^T,
whose gradient is  d loss / d N = -(2 / sum w) (I - P) M N (N^T N)^{-1},  M = V diag(w) V^T.
"""

from __future__ import annotations

import numpy as np


def conv1d(x: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """z[c, i] = b[c] + sum_{c', j} W[c, c', j] x[c', (i + j - r) mod n] (x: (cin, n))."""
    cout, cin, width = W.shape
    r = width // 2
    n = x.shape[1]
    z = np.repeat(b[:, None], n, axis=1).astype(np.float64)
    for j in range(width):
        shifted = np.roll(x, -(j - r), axis=1)  # shifted[c', i] = x[c', (i + j - r) mod n]
        z += W[:, :, j] @ shifted
    return z


def conv1d_backward(x: np.ndarray, W: np.ndarray, gz: np.ndarray):
    """Gradients (gx, gW, gb) of sum(gz * conv1d(x, W, b))."""
    cout, cin, width = W.shape
    r = width // 2
    gW = np.zeros_like(W, dtype=np.float64)
    gx = np.zeros_like(x, dtype=np.float64)
    for j in range(width):
        shifted = np.roll(x, -(j - r), axis=1)
        gW[:, :, j] = gz @ shifted.T
        gx += np.roll(W[:, :, j].T @ gz, j - r, axis=1)
    return gx, gW, gz.sum(axis=1)


def standardize(x: np.ndarray) -> np.ndarray:
    """The network's input: each row of x (C0, n) minus its mean over the grid, divided by
    its standard deviation; a single state (n,) is one row."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    return (x - x.mean(axis=1, keepdims=True)) / x.std(axis=1, keepdims=True)


def localize(z: np.ndarray, segments: int) -> np.ndarray:
    """Output head: N[i, c S + q] = z[c, i] for grid points i in segment q (the q-th block
    of n / S consecutive points), zero elsewhere. S = 1 gives N = z^T."""
    kch, n = z.shape
    seg = np.arange(n) // (n // segments)
    N = np.zeros((n, kch * segments))
    for c in range(kch):
        for q in range(segments):
            on = seg == q
            N[on, c * segments + q] = z[c, on]
    return N


def forward(params, x: np.ndarray, segments: int = 1):
    """Network output N (n, k) for the standardized input, and the per-layer activations."""
    h = standardize(x)
    acts = [h]
    for li, (W, b) in enumerate(params):
        z = conv1d(h, W, b)
        h = np.maximum(z, 0.0) if li < len(params) - 1 else z
        acts.append(h)
    return localize(h, segments), acts


def backward(params, acts, gN: np.ndarray, segments: int = 1):
    """Parameter gradients [(gW, gb)] of sum(gN * N)."""
    n = gN.shape[0]
    seg = np.arange(n) // (n // segments)
    kch = gN.shape[1] // segments
    g = np.zeros((kch, n))
    for c in range(kch):   # transpose of localize
        for q in range(segments):
            on = seg == q
            g[c, on] = gN[on, c * segments + q]
    grads = [None] * len(params)
    for li in range(len(params) - 1, -1, -1):
        W, b = params[li]
        if li < len(params) - 1:
            g = g * (acts[li + 1] > 0.0)  # relu'
        gx, gW, gb = conv1d_backward(acts[li], W, g)
        grads[li] = (gW, gb)
        g = gx
    return grads


def capture_loss(N: np.ndarray, V: np.ndarray, w: np.ndarray):
    """(loss, d loss / d N) of the weighted subspace capture (module doc)."""
    G = N.T @ N
    Gi = np.linalg.inv(G)
    A = V.T @ N                      # a_i = N^T v_i
    sw = float(np.sum(w))
    loss = -float(np.sum(w * np.einsum("ij,jk,ik->i", A, Gi, A))) / sw
    MN = V @ (w[:, None] * A)        # M N
    X = MN @ Gi
    PX = N @ (Gi @ (N.T @ X))
    return loss, -(2.0 / sw) * (X - PX)


def adam(p: np.ndarray, g: np.ndarray, m: np.ndarray, v: np.ndarray, t: int, lr: float,
         beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam step (Kingma and Ba, 2015) at step t >= 1 with bias-corrected moments:
    m <- b1 m + (1 - b1) g, v <- b2 v + (1 - b2) g^2, p <- p - lr m_hat / (sqrt(v_hat) + eps),
    m_hat = m / (1 - b1^t), v_hat = v / (1 - b2^t). Returns (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
