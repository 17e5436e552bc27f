"""Run-to-run reproducibility on the GPU: the same call twice on the same inputs.

Every reduction of the path sums in a fixed order: split-K GEMM partials, the Gram's partial
norms, the Cholesky's and triangular solve's tiles, both tridiagonalisations (per-tile slots
in the register-tile kernel, per-workgroup shares in the grid kernel), the eigenvector and
cluster steps. The TL/AD kernels have no atomics. So these calls must agree bit for bit:
* the Hessian-probe product (both TL/AD kernels: the LDS-ring kernel of the benchmarked shape
  and the register kernel of other shapes);
* the sketch's eigen-solve at m = 272 (register-tile tridiagonalisation, one-workgroup
  Cholesky), m = 300 (grid tridiagonalisation) and m = 400 (also the multi-workgroup
  Cholesky).
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


@pytest.mark.parametrize("m", [272, 300, 400])
def test_sketch_eig_bitwise_reproducible(m):
    from paper_1906_01413_amd import Sketch
    n = m + 16
    A = _spd(n, 300 + m)
    Om = np.random.default_rng(400 + m).standard_normal((n, m))
    Y = A @ Om
    sk = Sketch(n, m)
    (l1, V1, _), (l2, V2, _) = _twice(lambda: sk.eig(Om, Y))
    assert np.array_equal(to_np(l1), to_np(l2))
    assert np.array_equal(to_np(V1), to_np(V2))
