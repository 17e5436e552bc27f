"""CholeskyQR on the GPU (riot_orth) against the oracle's Householder QR.

For a full-rank X the thin QR with a positive diagonal in R is unique, so Q is compared
element by element with oracle.fourdvar.orth. The blocks are near-orthonormal (an
orthonormal block plus a small perturbation) or graded, so that the passes take each
branch: the shifted first pass, full factorizations, and the first-order factor that a
pass takes when its Gram matrix is within sqrt(u) of the identity in the Frobenius norm.
m = 272 factors in one workgroup, m = 400 in one workgroup per 32-column block.
"""

import numpy as np
import pytest

from oracle import fourdvar
from tests._problems import oracle_problem, riot_for, to_np

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _block(n, m, seed, kind):
    rng = np.random.default_rng(seed)
    Q0, _ = np.linalg.qr(rng.standard_normal((n, m)))
    if kind == "near_orthonormal":
        return Q0 + 1e-11 * rng.standard_normal((n, m))
    # graded columns over ten decades, mixed by a random orthogonal matrix
    s = 10.0 ** (-10.0 * np.arange(m) / (m - 1))
    Vt, _ = np.linalg.qr(rng.standard_normal((m, m)))
    return (Q0 * s) @ Vt


@pytest.mark.parametrize("m", [272, 400])
@pytest.mark.parametrize("kind", ["near_orthonormal", "graded"])
def test_orth_matches_householder_qr(m, kind):
    w, p = oracle_problem("l96_n4096", 0)
    r = riot_for(p, m_max=m)
    X = _block(p.n, m, 900 + m, kind)
    Q = to_np(r.orth(torch.tensor(X, device="cuda")))
    Qo = fourdvar.orth(X)
    e_orth = float(np.max(np.abs(Q.T @ Q - np.eye(m))))
    e_q = float(np.max(np.abs(Q - Qo)))
    # Q is determined to about kappa(X) u (kappa 1 or 1e10 here)
    bound = 1e-13 if kind == "near_orthonormal" else 1e-5
    print(f"m={m} {kind}: orthonormality {e_orth:.1e}, |Q - Q_oracle|_max {e_q:.1e}")
    assert e_orth < 1e-14 * m
    assert e_q < bound


@pytest.mark.parametrize("kind", ["near_orthonormal", "graded"])
def test_pass_control_modes_agree(kind):
    """Passes launched on the host's reading of each decision, or all launched and
    predicated on the device: the same passes run, so Q is the same bit for bit."""
    w, p = oracle_problem("l96_n4096", 0)
    r = riot_for(p, m_max=272)
    X = torch.tensor(_block(p.n, 272, 77, kind), device="cuda")
    out = []
    for on in (True, False, True):
        r.set_pass_sync(on)
        out.append(to_np(r.orth(X)))
    print(f"{kind}: host-read vs predicated max diff {np.max(np.abs(out[0] - out[1])):.1e}")
    assert np.array_equal(out[0], out[1]) and np.array_equal(out[0], out[2])


def test_pass_control_rsvd_agrees():
    """The whole randomized eigendecomposition (two CholeskyQR sequences) in both modes."""
    w, p = oracle_problem("l96_n4096", 0)
    r = riot_for(p, m_max=272)
    r.linearize(p.xb)
    res = []
    for on in (True, False):
        r.set_pass_sync(on)
        lam, V, info = r.rsvd(256, 16, q=0, seed=5)
        res.append((to_np(lam), to_np(V), info.qr_passes))
    assert res[0][2] == res[1][2]
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])
