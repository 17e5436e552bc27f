"""Pins of the sketch-proposal network oracle (oracle/convnet.py)."""

import numpy as np
import pytest

from oracle import convnet
from synthetic import net_init


def test_conv1d_is_a_circulant_matrix_product():
    """One input and one output channel: the layer is x -> C x with C circulant."""
    rng = np.random.default_rng(0)
    n, width = 11, 5
    r = width // 2
    W = rng.standard_normal((1, 1, width))
    x = rng.standard_normal((1, n))
    C = np.zeros((n, n))
    for i in range(n):
        for j in range(width):
            C[i, (i + j - r) % n] += W[0, 0, j]
    z = convnet.conv1d(x, W, np.array([0.3]))
    assert np.max(np.abs(z[0] - (C @ x[0] + 0.3))) < 1e-14


def _fd_check(f, x, g, rng, eps=1e-6):
    d = rng.standard_normal(x.shape)
    fd = (f(x + eps * d) - f(x - eps * d)) / (2 * eps)
    an = float(np.sum(g * d))
    return abs(fd - an) / max(abs(an), 1e-12)


def test_localized_head_partitions_the_channels():
    """Columns c S + q, q = 0..S-1, have disjoint supports (blocks of n / S points) and
    sum to channel c."""
    z = np.random.default_rng(6).standard_normal((3, 24))
    N = convnet.localize(z, 4)
    assert N.shape == (24, 12)
    for c in range(3):
        cols = N[:, c * 4: c * 4 + 4]
        assert np.array_equal(cols.sum(axis=1), z[c])
        assert np.all(np.count_nonzero(cols, axis=1) <= 1)
        for q in range(4):
            assert np.all(cols[:q * 6, q] == 0) and np.all(cols[q * 6 + 6:, q] == 0)
    assert np.array_equal(convnet.localize(z, 1), z.T)


@pytest.mark.parametrize("segments", [1, 2])
def test_network_gradients_match_central_differences(segments):
    rng = np.random.default_rng(1)
    n = 16
    params = net_init(7, [(3, 1, 5), (3, 3, 5), (2, 3, 5)])
    x = rng.standard_normal(n)
    gN = rng.standard_normal((n, 2 * segments))
    N, acts = convnet.forward(params, x, segments)
    grads = convnet.backward(params, acts, gN, segments)
    for li in range(len(params)):
        W, b = params[li]

        def fW(Wp, li=li):
            p = [(Wp if i == li else params[i][0], params[i][1]) for i in range(len(params))]
            return float(np.sum(gN * convnet.forward(p, x, segments)[0]))

        def fb(bp, li=li):
            p = [(params[i][0], bp if i == li else params[i][1]) for i in range(len(params))]
            return float(np.sum(gN * convnet.forward(p, x, segments)[0]))

        assert _fd_check(fW, W, grads[li][0], rng) < 1e-7
        assert _fd_check(fb, b, grads[li][1], rng) < 1e-7


def test_capture_loss_invariances_and_gradient():
    rng = np.random.default_rng(2)
    n, k = 30, 4
    V = np.linalg.qr(rng.standard_normal((n, k)))[0]
    w = rng.uniform(0.2, 1.0, k)
    # a basis containing span(V) captures everything: loss = -1
    N = np.hstack([V @ rng.standard_normal((k, k)), rng.standard_normal((n, 2))])
    assert abs(convnet.capture_loss(N, V, w)[0] + 1.0) < 1e-12
    # a basis orthogonal to span(V) captures nothing
    Q = np.linalg.qr(np.hstack([V, rng.standard_normal((n, 3))]))[0][:, k:]
    assert abs(convnet.capture_loss(Q, V, w)[0]) < 1e-12
    # invariant to a change of basis of span(N)
    N = rng.standard_normal((n, 5))
    R = rng.standard_normal((5, 5)) + 3 * np.eye(5)
    assert abs(convnet.capture_loss(N, V, w)[0] - convnet.capture_loss(N @ R, V, w)[0]) < 1e-12
    loss, g = convnet.capture_loss(N, V, w)
    assert _fd_check(lambda Np: convnet.capture_loss(Np, V, w)[0], N, g, rng) < 1e-7


def test_network_is_shift_equivariant_and_scale_invariant():
    """Periodic convolutions commute with cyclic shifts of the grid, and the standardized
    input makes the output independent of an affine change a x + c (a > 0) of the state."""
    params = net_init(8, [(4, 1, 5), (4, 4, 5), (3, 4, 5)])
    x = np.random.default_rng(3).standard_normal(32)
    N, _ = convnet.forward(params, x)
    Ns, _ = convnet.forward(params, np.roll(x, 5))
    assert np.max(np.abs(Ns - np.roll(N, 5, axis=0))) < 1e-12
    Na, _ = convnet.forward(params, 3.0 * x + 7.0)
    assert np.max(np.abs(Na - N)) < 1e-12
    # several input rows: each row is standardized on its own
    p2 = net_init(9, [(4, 2, 5), (3, 4, 5)])
    X2 = np.random.default_rng(4).standard_normal((2, 32))
    N2, _ = convnet.forward(p2, X2)
    N2a, _ = convnet.forward(p2, np.stack([0.5 * X2[0] - 1.0, 4.0 * X2[1] + 2.0]))
    assert np.max(np.abs(N2a - N2)) < 1e-12


def test_adam_first_step_and_fixed_point():
    """Bias correction makes the first step lr g / (|g| + eps) (about lr sign(g)); a zero
    gradient with zero moments leaves the parameters unchanged; on f = 1/2 ||p||^2 the
    iteration approaches the minimiser."""
    rng = np.random.default_rng(4)
    p = rng.standard_normal(50)
    g = rng.standard_normal(50)
    z = np.zeros(50)
    p1, m1, v1 = convnet.adam(p, g, z, z, 1, 0.01)
    assert np.max(np.abs((p - p1) - 0.01 * g / (np.abs(g) + 1e-8))) < 1e-15
    p2, _, _ = convnet.adam(p, z, z, z, 1, 0.01)
    assert np.array_equal(p2, p)
    q, m, v = p.copy(), z.copy(), z.copy()
    for t in range(1, 3001):
        q, m, v = convnet.adam(q, q, m, v, t, 0.01)
    assert np.max(np.abs(q)) < 1e-2 * np.max(np.abs(p))
