"""Eigen-solve of the RSVD's small matrix (Alg. 3: K = Z Lambda Z^T, Ritz vectors Q Z) across the
sizes where the device path changes kernels: the register-tile tridiagonalisation (3 <= m <= 279)
or the grid one (other m), the one-workgroup Cholesky (m <= 352) or the one with a workgroup per
32-column block (m = 353, 512, 1088), and the blocked WY back-transformation (m <= 288) or the
per-column one (larger m). m below 16 is also where the blocked back-transformation's factors
need more scratch than the per-column kernels.

Each case is a seeded symmetric positive definite A (n = m + 16) with eigenvalues spread over six
decades; Y = A Omega is formed once on the host and handed to both sides, so the device RSVD
(sketch handle) and the oracle's RSVD see the same sketch. The Ritz values must agree to 1e-10 of
the largest, the rank-m approximation V diag(lam) V^T (basis independent inside clusters) to
1e-10, and V must be orthonormal.
"""

import numpy as np
import pytest

from oracle import fourdvar
from tests._problems import rel, to_np

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SIZES = [2, 3, 5, 8, 15, 16, 17, 33, 64, 279, 280, 288, 289, 300, 353, 512, 1088]


def _spd(n, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = 1e3 * 10.0 ** (-6.0 * np.arange(n) / max(n - 1, 1))
    return (Q * lam) @ Q.T


@pytest.mark.parametrize("m", SIZES)
def test_eig_sizes_match_oracle(m):
    from paper_1906_01413_amd import Sketch
    n = m + 16
    A = _spd(n, 100 + m)
    Om = np.random.default_rng(200 + m).standard_normal((n, m))
    Y = A @ Om
    ro = fourdvar.rsvd(lambda X: A @ X, Om, q=0)
    sk = Sketch(n, m)
    lam, V, info = sk.eig(Om, Y)
    lam, V = to_np(lam), to_np(V)
    assert info.orth_err < 1e-11
    assert np.all(np.diff(lam) <= 0.0)  # descending
    assert np.max(np.abs(lam - ro.lam)) <= 1e-10 * ro.lam[0]
    assert rel((V * lam) @ V.T, (ro.V * ro.lam) @ ro.V.T) < 1e-10
    assert np.max(np.abs(V.T @ V - np.eye(m))) < 1e-11


@pytest.mark.parametrize("m,c", [(100, 60), (300, 60), (400, 120)])
def test_eig_large_cluster_matches_oracle(m, c):
    """A cluster of c eigenvalues within a relative gap of 1e-5, more than the 48 one cluster
    step takes, so it is cut into a chain of two or three clusters whose vectors are
    orthogonalised against the whole chain; on the register-tile (m = 100) and grid
    (m = 300, 400) tridiagonalisations: the rank-m approximation (basis independent inside
    the cluster) and the orthonormality of V against the oracle."""
    from paper_1906_01413_amd import Sketch
    n = m + 16
    rng = np.random.default_rng(500 + m)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = 1e3 * 10.0 ** (-4.0 * np.arange(n) / (n - 1))
    lam[10:10 + c] = 50.0 * (1.0 + 1e-5 * np.arange(c) / c)
    A = (Q * lam) @ Q.T
    Om = rng.standard_normal((n, m))
    Y = A @ Om
    ro = fourdvar.rsvd(lambda X: A @ X, Om, q=0)
    lamg, V, info = Sketch(n, m).eig(Om, Y)
    lamg, V = to_np(lamg), to_np(V)
    e_lam = float(np.max(np.abs(lamg - ro.lam)) / ro.lam[0])
    e_rec = rel((V * lamg) @ V.T, (ro.V * ro.lam) @ ro.V.T)
    e_orth = float(np.max(np.abs(V.T @ V - np.eye(m))))
    print(f"m={m}, cluster of {c}: Ritz values {e_lam:.1e} of lam1, rank-m {e_rec:.1e}, "
          f"orthonormality {e_orth:.1e}")
    assert e_lam <= 1e-10 and e_rec < 1e-10 and e_orth < 1e-11
