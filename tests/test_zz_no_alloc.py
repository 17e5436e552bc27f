"""riot_sketch_eig_noalloc: the steps of Alg. 3 after the Hessian-probe products (orthonormal
basis, K from K Q^T Omega = Q^T Y, eigendecomposition, Ritz vectors) with no handle and no
workspace, on the library's static device scratch.

Two calls in a row on one device, each checked against riot_sketch_eig (the same stages on a
caller-allocated workspace) on the same sketch:
  1. the benchmarked Lorenz-96 problem (n = 4096, T = 100, 20480 observations), m = 272
     Philox probes, Y = A Omega from the C ABI's Hessian-probe product;
  2. a smaller seeded SPD operator (n = 300, m = 64, eigenvalues over six decades), which
     reuses the scratch the first call left behind.
Ritz values must agree to 1e-12 of the largest, and the basis-independent rank-m forms
V diag(lam) V^T and V V^T (applied to a seeded block) to 1e-10: the tridiagonalisation's
accumulation order may differ between two runs, so bitwise equality is not expected.
"""

import os

import numpy as np
import pytest

from oracle import fourdvar
from tests._problems import rel, to_np

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

REF = os.path.join(os.path.dirname(__file__), "golden", "ref_l96_n4096_s0.npz")


def _compare(lam_a, V_a, lam_b, V_b, seed):
    lam_a, V_a, lam_b, V_b = to_np(lam_a), to_np(V_a), to_np(lam_b), to_np(V_b)
    Z = np.random.default_rng(seed).standard_normal((V_a.shape[0], 8))
    err_lam = float(np.max(np.abs(lam_a - lam_b)) / abs(lam_b[0]))
    err_op = rel(V_a @ (lam_a[:, None] * (V_a.T @ Z)), V_b @ (lam_b[:, None] * (V_b.T @ Z)))
    err_proj = rel(V_a @ (V_a.T @ Z), V_b @ (V_b.T @ Z))
    print(f"noalloc vs workspace: lambda {err_lam:.2e}, V diag(lam) V^T {err_op:.2e}, "
          f"V V^T {err_proj:.2e}", flush=True)
    assert err_lam <= 1e-12
    assert err_op <= 1e-10
    assert err_proj <= 1e-10


def _spd(n, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = 1e3 * 10.0 ** (-6.0 * np.arange(n) / (n - 1))
    return (Q * lam) @ Q.T


def test_noalloc_matches_workspace_entry_point_twice():
    from paper_1906_01413_amd import Riot, Sketch
    from paper_1906_01413_amd.riot import RiotError, sketch_eig_noalloc

    if not os.path.exists(REF):
        pytest.skip("reference problem not generated")
    z = dict(np.load(REF, allow_pickle=False))
    p = fourdvar.Problem(int(z["n"]), int(z["nsteps"]), float(z["dt"]), float(z["forcing"]),
                         z["obs_step"], z["obs_idx"], z["y"], z["rinv"], z["xb"], z["taps"])
    m = 272
    r = Riot(p.n, p.nsteps, p.h, p.F, p.obs_step, p.obs_idx, p.y, p.rinv, p.taps, m_max=m)
    r.linearize(p.xb)
    Om = r.philox_normal(p.n, m, seed=77)
    Y = r.hess_apply(Om)

    # call 1: full size
    lam_s, V_s, info_s = Sketch(p.n, m).eig(Om, Y)
    lam_n, V_n, info_n = sketch_eig_noalloc(Om, Y)
    torch.cuda.synchronize()
    assert info_n.orth_err < 1e-10 and info_s.orth_err < 1e-10
    _compare(lam_n, V_n, lam_s, V_s, 1)

    # call 2: a smaller problem in the same scratch
    n2, m2 = 300, 64
    A = _spd(n2, 5)
    Om2 = np.random.default_rng(6).standard_normal((n2, m2))
    Y2 = A @ Om2
    lam_s2, V_s2, _ = Sketch(n2, m2).eig(Om2, Y2)
    lam_n2, V_n2, info2 = sketch_eig_noalloc(Om2, Y2)
    torch.cuda.synchronize()
    assert info2.orth_err < 1e-11
    _compare(lam_n2, V_n2, lam_s2, V_s2, 2)
    ro = fourdvar.rsvd(lambda X: A @ X, Om2, q=0)
    assert np.max(np.abs(to_np(lam_n2) - ro.lam)) <= 1e-10 * ro.lam[0]

    # sizes beyond the static scratch are refused before any work is enqueued
    with pytest.raises(RiotError) as ei:
        sketch_eig_noalloc(torch.zeros((4096, 400), dtype=torch.float64, device="cuda").t()
                           .contiguous().t(),
                           torch.zeros((4096, 400), dtype=torch.float64, device="cuda").t()
                           .contiguous().t(), want_info=False)
    assert ei.value.status == -9
