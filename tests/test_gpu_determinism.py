"""Run-to-run reproducibility on the GPU: the same call twice on the same inputs.

Every reduction of the path sums in a fixed order (split-K GEMM partials, the Gram's
partial norms, the Cholesky's and triangular solve's tiles, the grid tridiagonalisation's
per-workgroup shares, the eigenvector and cluster steps), and the TL/AD kernels have no
atomics, so these calls must agree bit for bit:
* the Hessian-probe product (both TL/AD kernels: the LDS-ring kernel of the benchmarked shape
  and the register kernel of other shapes);
* the sketch's eigen-solve where m is past the register-tile tridiagonalisation (m = 300:
  grid tridiagonalisation, and at m = 400 the multi-workgroup Cholesky as well).

The register-tile tridiagonalisation (3 <= m <= 279) accumulates p = S v, |x|^2 and v^T S v
with LDS atomics, whose order of additions varies between runs, so there the Ritz values
must agree to rounding (1e-13 of the largest) and the Ritz vectors up to the same level.
"""

import numpy as np
import pytest

from tests._problems import oracle_problem, riot_for, to_np

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _spd(n, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = 1e3 * 10.0 ** (-6.0 * np.arange(n) / max(n - 1, 1))
    return (Q * lam) @ Q.T


def _twice(fn):
    a = fn()
    torch.cuda.synchronize()
    b = fn()
    torch.cuda.synchronize()
    return a, b


@pytest.mark.parametrize("name,m", [("l96_n40", 30), ("l96_n4096", 272)])
def test_hvp_bitwise_reproducible(name, m):
    """n = 40 (register kernel) and n = 4096 with 272 columns (LDS-ring kernel)."""
    from synthetic import probe_block
    w, p = oracle_problem(name, 0)
    r = riot_for(p, m_max=m)
    r.linearize(p.xb)
    W = probe_block(5, 0, p.n, m)
    a, b = _twice(lambda: to_np(r.hess_apply(W)))
    assert np.array_equal(a, b)


@pytest.mark.parametrize("m", [300, 400])
def test_sketch_eig_bitwise_reproducible_beyond_register_tiles(m):
    from paper_1906_01413_amd import Sketch
    n = m + 16
    A = _spd(n, 300 + m)
    Om = np.random.default_rng(400 + m).standard_normal((n, m))
    Y = A @ Om
    sk = Sketch(n, m)
    (l1, V1, _), (l2, V2, _) = _twice(lambda: sk.eig(Om, Y))
    assert np.array_equal(to_np(l1), to_np(l2))
    assert np.array_equal(to_np(V1), to_np(V2))


def test_sketch_eig_register_tiles_reproducible_to_rounding():
    from paper_1906_01413_amd import Sketch
    m = 272
    n = m + 16
    A = _spd(n, 999)
    Om = np.random.default_rng(998).standard_normal((n, m))
    Y = A @ Om
    sk = Sketch(n, m)
    (l1, V1, _), (l2, V2, _) = _twice(lambda: sk.eig(Om, Y))
    l1, l2, V1, V2 = to_np(l1), to_np(l2), to_np(V1), to_np(V2)
    assert np.max(np.abs(l1 - l2)) <= 1e-13 * abs(l1[0])
    # basis independent inside clusters: compare the rank-m reconstruction
    R1, R2 = (V1 * l1) @ V1.T, (V2 * l2) @ V2.T
    assert np.linalg.norm(R1 - R2) <= 1e-12 * np.linalg.norm(R1)
