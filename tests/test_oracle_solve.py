"""Pins of the oracle's inner-loop solvers: exact solve, RSVD, increments, covariance, CG.

Each pin is a mathematical fact independent of the oracle's own code paths:
primal/dual (Woodbury) equality, exactness at full rank, exactness for exact
low-rank operators, the Halko et al. range-finder bound, Krylov minimisation
of CG, and published Philox test vectors.
"""

import math
import os

import numpy as np
import pytest

from oracle import bcov, fourdvar, philox
from synthetic import l96_draws, probe_block, workload

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def c1():
    w = workload("l96_n40")
    p, _ = fourdvar.realize_l96(w, l96_draws(w, 0))
    lin = fourdvar.linearize(p, p.xb)
    A = fourdvar.dense_A(p, lin)
    return w, p, lin, A


def test_primal_equals_dual(c1):
    # Woodbury: L (I + A)^{-1} L G^T R^{-1} d = B G^T (G B G^T + R)^{-1} d  (dual form of eq. 3)
    _, p, lin, A = c1
    G = fourdvar.obs_jacobian(p, lin)
    Lm = bcov.dense_L(p.n, p.taps)
    B = Lm @ Lm.T
    R = np.diag(1.0 / p.rinv)
    dual = B @ G.T @ np.linalg.solve(G @ B @ G.T + R, lin.d)
    ex = fourdvar.exact_solve(p, A, lin.g)
    assert np.linalg.norm(ex.dx - dual) <= 1e-9 * np.linalg.norm(dual)
    # and A itself is L^T G^T R^{-1} G L built from the explicit Jacobian
    A2 = Lm.T @ G.T @ (p.rinv[:, None] * G) @ Lm
    assert np.linalg.norm(A - A2) <= 1e-11 * np.linalg.norm(A2)


def test_rsvd_exact_at_full_rank(c1):
    _, p, lin, A = c1
    Om = probe_block(0, 0, p.n, p.n)
    r = fourdvar.rsvd(lambda W: A @ W, Om, q=0)
    ex = fourdvar.exact_solve(p, A, lin.g)
    assert np.allclose(r.lam, ex.lam, rtol=0, atol=1e-9 * ex.lam[0])
    for mode in ("lra", "lru"):
        dz, dx, dofs, _ = fourdvar.increment(p, r.lam, r.V, lin.g, mode=mode)
        assert np.linalg.norm(dz - ex.dz) <= 1e-7 * np.linalg.norm(ex.dz)
    assert abs(dofs - np.trace(A @ np.linalg.inv(np.eye(p.n) + A))) < 1e-8


def test_rsvd_exact_for_exact_low_rank():
    rng = np.random.default_rng(11)
    n, r, m = 60, 10, 15
    U, _ = np.linalg.qr(rng.standard_normal((n, r)))
    s = np.logspace(3, -1, r)
    A = (U * s) @ U.T
    res = fourdvar.rsvd(lambda W: A @ W, rng.standard_normal((n, m)), q=0)
    assert np.allclose(res.lam[:r], s, rtol=1e-10)
    assert np.all(np.abs(res.lam[r:]) < 1e-10 * s[0])
    P = res.V[:, :r] @ res.V[:, :r].T
    assert np.linalg.norm(P - U @ U.T) < 1e-10


def test_range_finder_within_halko_bound():
    # Halko, Martinsson & Tropp (2011) Thm 10.6: E||(I - QQ^T) A|| <=
    # (1 + sqrt(k/(p-1))) s_{k+1} + e sqrt(k+p)/p (sum_{j>k} s_j^2)^{1/2}
    rng = np.random.default_rng(12)
    n, k, p_os = 80, 10, 5
    U, _ = np.linalg.qr(rng.standard_normal((n, n)))
    s = 1.0 / (1.0 + np.arange(n)) ** 1.5
    A = (U * s) @ U.T
    bound = (1 + math.sqrt(k / (p_os - 1))) * s[k] + math.e * math.sqrt(k + p_os) / p_os * math.sqrt(np.sum(s[k:] ** 2))
    errs = []
    for seed in range(20):
        res = fourdvar.rsvd(lambda W: A @ W, np.random.default_rng(seed).standard_normal((n, k + p_os)))
        errs.append(np.linalg.norm(A - res.Q @ (res.Q.T @ A), 2))
    assert np.median(errs) <= bound
    assert np.median(errs) >= s[k + p_os] * 0.99  # cannot beat the optimal rank-(k+p) error


def test_rsvd_power_iteration_improves(c1):
    _, p, lin, A = c1
    ex = fourdvar.exact_solve(p, A, lin.g)
    Om = probe_block(1, 0, p.n, 30)
    e = []
    for q in (0, 1):
        r = fourdvar.rsvd(lambda W: A @ W, Om, q=q)
        dz, *_ = fourdvar.increment(p, r.lam, r.V, lin.g)
        e.append(np.linalg.norm(dz - ex.dz) / np.linalg.norm(ex.dz))
    assert e[1] < e[0]
    assert e[1] < 1e-5


def test_posterior_cov_exact_at_full_rank(c1):
    _, p, lin, A = c1
    ex = fourdvar.exact_solve(p, A, lin.g)
    _, Px = fourdvar.exact_posterior(p, A)
    for mode in ("lra", "lru"):
        W, coef, diag, P, _ = fourdvar.posterior_cov(p, ex.lam, ex.V, mode=mode, dense=True)
        assert np.linalg.norm(P - Px) <= 1e-9 * np.linalg.norm(Px)
        assert np.allclose(diag, np.diag(Px), atol=1e-10)


def test_lru_better_than_lra_when_truncated_low(c1):
    # With the last kept eigenvalue below 1 (eq. 11's LRU branch) the full-rank LRU
    # keeps the prior in unresolved directions and beats LRA's rank-k truncation.
    _, p, lin, A = c1
    ex = fourdvar.exact_solve(p, A, lin.g)
    k = int(np.sum(ex.lam >= 1.0)) + 5
    e = {}
    for mode in ("lra", "lru"):
        dz, *_ = fourdvar.increment(p, ex.lam, ex.V, lin.g, k=k, mode=mode)
        e[mode] = np.linalg.norm(dz - ex.dz)
    assert e["lru"] < e["lra"]
    assert fourdvar.choose_update(1.0) == "lra" and fourdvar.choose_update(0.999) == "lru"


def test_cg_iterates_are_krylov_minimisers(c1):
    _, p, lin, A = c1
    its = fourdvar.cg(lambda x: x + A @ x, lin.g, 6)
    for q in (1, 3, 6):
        kq = fourdvar.krylov_minimizer(lambda x: A @ x, lin.g, q)
        assert np.linalg.norm(its[:, q - 1] - kq) <= 1e-8 * np.linalg.norm(kq)


def test_cg_and_lanczos_reach_exact_solution():
    # well-conditioned small problem: both Krylov methods terminate at the exact minimiser
    w = workload("l96_n40", n=16, nsteps=6, var_stride=2, step_stride=2)
    p, _ = fourdvar.realize_l96(w, l96_draws(w, 3))
    lin = fourdvar.linearize(p, p.xb)
    A = fourdvar.dense_A(p, lin)
    ex = fourdvar.exact_solve(p, A, lin.g)
    its = fourdvar.cg(lambda x: x + A @ x, lin.g, p.n)
    assert np.linalg.norm(its[:, -1] - ex.dz) <= 1e-8 * np.linalg.norm(ex.dz)
    dz, lam, _ = fourdvar.lanczos_varcg(lambda x: A @ x, lin.g, p.n)
    assert np.linalg.norm(dz - ex.dz) <= 1e-8 * np.linalg.norm(ex.dz)


def test_outer_loops_decrease_cost(c1):
    w, p, _, _ = c1
    def solver(k, lin):
        A = fourdvar.dense_A(p, lin)
        return fourdvar.exact_solve(p, A, lin.g).dz
    hist = fourdvar.outer_loop(p, 3, solver)
    J = [h["J"] for h in hist]
    assert J[1] < J[0] and J[3] <= J[2] * (1 + 1e-9)


def test_philox_known_answers():
    with open(os.path.join(GOLDEN, "philox_kat.txt")) as f:
        rows = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        assert philox.philox4x32_10(v[0:4], v[4:6]) == tuple(v[6:10])


def test_philox_normals_moments():
    z = philox.normal_block(200, 50, seed=1234, stream=3)
    assert z.shape == (200, 50)
    assert abs(z.mean()) < 0.03 and abs(z.std() - 1.0) < 0.03


def test_proj_residual_closed_form():
    """A = diag-like symmetric with eigenpairs (l1, v1), (l2, v2); Q = cos t v1 + sin t v2:
    A Q - Q Q^T A Q has norm |l1 - l2| |sin t cos t| and ||A Q||^2 = l1^2 cos^2 + l2^2 sin^2.
    An invariant subspace gives zero."""
    rng = np.random.default_rng(5)
    n = 12
    U = np.linalg.qr(rng.standard_normal((n, n)))[0]
    lam = np.linspace(9.0, 0.5, n)
    A = (U * lam) @ U.T
    t = 0.37
    q = np.cos(t) * U[:, 0] + np.sin(t) * U[:, 1]
    Q = q[:, None]
    want = abs(lam[0] - lam[1]) * abs(np.sin(t) * np.cos(t)) / np.sqrt(
        lam[0] ** 2 * np.cos(t) ** 2 + lam[1] ** 2 * np.sin(t) ** 2)
    assert abs(fourdvar.proj_residual(Q, A @ Q) - want) < 1e-14
    V = U[:, [2, 5, 7]]
    assert fourdvar.proj_residual(V, A @ V) < 1e-14


def test_increment_select_two_nonlinear_runs():
    """Deterministic LRA/LRU choice (Sec. 3.2.1): both candidates' non-quadratic costs equal
    eq. 2 at v + dz and are consistent to first order with the gradient along each
    candidate; the lower one is kept; at full rank the two updates coincide."""
    from oracle import bcov
    w = workload("l96_n40", nsteps=4, step_stride=1)
    p, _ = fourdvar.realize_l96(w, l96_draws(w, 2))
    v = 0.05 * np.random.default_rng(4).standard_normal(p.n)
    lin = fourdvar.linearize(p, p.xb + bcov.apply_L(v, p.taps), v)
    A = fourdvar.dense_A(p, lin)
    A = 0.5 * (A + A.T)
    lam, V = np.linalg.eigh(A)
    lam, V = lam[::-1], V[:, ::-1]
    for k in (3, 8, 20):
        dz, dx, mode, Ja, Ju = fourdvar.increment_select(p, lam, V, lin.g, v, k=k)
        dza, _, _, _ = fourdvar.increment(p, lam, V, lin.g, k, "lra")
        dzu, _, _, _ = fourdvar.increment(p, lam, V, lin.g, k, "lru")
        assert Ja == fourdvar.cost(p, v + dza) and Ju == fourdvar.cost(p, v + dzu)
        for dzc in (dza, dzu):
            # J(v + t dz) - J - t g^T dz = O(t^2) (the candidate lives in the gradient's
            # control variables): halving t divides the gap by about 4. The quadratic
            # model's I + A is the Gauss-Newton Hessian, which leaves out the model's second
            # derivative times the innovation, so J - q is itself second order.
            def gap(t, dzc=dzc):
                return fourdvar.cost(p, v + t * dzc) - lin.J - t * (lin.g @ dzc)
            r = gap(0.02) / gap(0.01)
            assert 3.6 < r < 4.4, r
        assert mode == ("lra" if Ja <= Ju else "lru")
        assert np.array_equal(dz, dza if mode == "lra" else dzu)
        assert np.allclose(dx, bcov.apply_L(dz, p.taps), rtol=0, atol=1e-14 * np.abs(dx).max())
    # both outcomes occur on this problem: truncated at 3 pairs (lambda_3 >> 1) the LRU step
    # along the unresolved directions overshoots; with 20 pairs LRU is the better one
    modes = {fourdvar.increment_select(p, lam, V, lin.g, v, k=k)[2] for k in (3, 20)}
    print("selected modes at k = 3, 20:", modes)
    # full rank: both updates are the exact minimiser of the quadratic model
    _, _, _, Jaf, Juf = fourdvar.increment_select(p, lam, V, lin.g, v, k=p.n)
    assert abs(Jaf - Juf) <= 1e-10 * abs(Jaf)


def test_psas_dual_matches_primal():
    """RIOT-PSAS (Appendix): A_hat = R^{-1/2} G B G^T R^{-1/2} has the nonzero spectrum of the
    primal A = L G^T R^{-1} G L (both are products of the same factor and its transpose); at
    full rank the dual increment is the primal Gauss-Newton step (Woodbury), at the first
    outer loop and at a later one (x != x_b, where the reading x_new = x_b + B G^T dw holds);
    with fewer probes the dual sketch gives the primal exact answer only approximately."""
    from oracle import bcov
    w = workload("l96_n40", nsteps=12, var_stride=4, step_stride=4)
    p, _ = fourdvar.realize_l96(w, l96_draws(w, 3))
    assert p.nobs < p.n  # 10 variables x 3 steps = 30 observations, 40 controls
    for v in (np.zeros(p.n), 0.1 * np.random.default_rng(8).standard_normal(p.n)):
        x = p.xb + bcov.apply_L(v, p.taps)
        lin = fourdvar.linearize(p, x, v)
        A = fourdvar.dense_A(p, lin)
        A = 0.5 * (A + A.T)
        Ah = fourdvar.psas_hvp(p, lin, np.eye(p.nobs))
        assert np.max(np.abs(Ah - Ah.T)) <= 1e-12 * np.max(np.abs(Ah))
        lp = np.sort(np.linalg.eigvalsh(A))[::-1][:p.nobs]
        ld = np.sort(np.linalg.eigvalsh(0.5 * (Ah + Ah.T)))[::-1]
        assert np.allclose(lp, ld, rtol=1e-9, atol=1e-11 * lp[0])
        # primal Gauss-Newton step: x + L dz*, dz* = -(I + A)^{-1} g
        dz = -np.linalg.solve(np.eye(p.n) + A, lin.g)
        x_primal = x + bcov.apply_L(dz, p.taps)
        Om = probe_block(5, 0, p.nobs, p.nobs)
        ro = fourdvar.rsvd(lambda X: fourdvar.psas_hvp(p, lin, X), Om, q=0)
        rhs = fourdvar.psas_rhs(p, lin, x)
        for mode in ("lra", "lru"):
            _, dx, x_new, _ = fourdvar.psas_increment(p, lin, ro.lam, ro.V, rhs, x, mode=mode)
            assert np.linalg.norm(x_new - x_primal) <= 1e-9 * np.linalg.norm(x_primal - x)
        # truncated: approximate only
        ro8 = fourdvar.rsvd(lambda X: fourdvar.psas_hvp(p, lin, X), Om[:, :8], q=0)
        _, _, x8, _ = fourdvar.psas_increment(p, lin, ro8.lam, ro8.V, rhs, x)
        e8 = np.linalg.norm(x8 - x_primal) / np.linalg.norm(x_primal - x)
        assert 1e-6 < e8 < 1.0


def _small():
    w = workload("l96_n40", nsteps=16, step_stride=4)
    p, _ = fourdvar.realize_l96(w, l96_draws(w, 5))
    return w, p


def test_spectral_preconditioner_and_rotation():
    """Alg. 3's precond / rotation branches (eqs. 6-7): P^{-1} P = I; with the exact leading
    eigenpairs of A as the first level, P^T (I + A) P has eigenvalue 1 on the resolved
    directions and the rest of 1 + lambda unchanged; rotated probes mapped by P are orthogonal
    to the resolved directions; at full rank the preconditioned step P dw is the
    unpreconditioned exact step; three outer loops with precond (with and without rotation)
    decrease J like the plain loops and approach the Gauss-Newton limit."""
    w, p = _small()
    lin = fourdvar.linearize(p, p.xb)
    A = fourdvar.dense_A(p, lin)
    A = 0.5 * (A + A.T)
    lam, V = np.linalg.eigh(A)
    lam, V = lam[::-1], V[:, ::-1]
    m = 12
    levels = [(V[:, :m], 1.0 + lam[:m])]
    X = np.random.default_rng(1).standard_normal((p.n, 4))
    assert np.allclose(fourdvar.precond_apply(levels, fourdvar.precond_apply(levels, X, "P"),
                                              "Pinv"), X, atol=1e-12)
    Pm = fourdvar.precond_apply(levels, np.eye(p.n), "P")
    M = Pm.T @ (np.eye(p.n) + A) @ Pm
    ev = np.sort(np.linalg.eigvalsh(0.5 * (M + M.T)))[::-1]
    expect = np.sort(np.concatenate([np.ones(m), 1.0 + lam[m:]]))[::-1]
    assert np.allclose(ev, expect, rtol=1e-9, atol=1e-9)
    # the operator form agrees with the matrix form
    Hw = fourdvar.precond_hvp(p, lin, levels, X)
    assert np.allclose(Hw, (M - np.eye(p.n)) @ X, rtol=0, atol=1e-8 * np.abs(Hw).max())
    # rotation: P omega_rot lies in the complement of span(resolved)
    Om = probe_block(4, 0, p.n, 6)
    resolved = [V[:, :m]]  # P_1 = I at the first loop
    Omr = fourdvar.rotate_probes(levels, resolved, Om)
    assert np.max(np.abs(V[:, :m].T @ fourdvar.precond_apply(levels, Omr, "P"))) < 1e-12
    # full rank: P dw* = dz*
    b = fourdvar.precond_apply(levels, lin.g, "PT")
    dw = -np.linalg.solve(M, b)
    dz = -np.linalg.solve(np.eye(p.n) + A, lin.g)
    assert np.allclose(fourdvar.precond_apply(levels, dw, "P"), dz, rtol=0,
                       atol=1e-9 * np.abs(dz).max())
    # three outer loops
    probes = [probe_block(30 + k, 0, p.n, 12) for k in range(3)]  # 2 x 12 resolved < n = 40
    runs = {}
    for key, pc, rot in (("plain", False, False), ("precond", True, False), ("rotation", True, True)):
        hist, v, x, J = fourdvar.riot_outer_loops(p, probes, 3, pc, rot)
        runs[key] = [h["J"] for h in hist] + [J]
        assert runs[key][-1] < runs[key][0]
    print("J per outer loop:", {k: [f"{j:.3f}" for j in r] for k, r in runs.items()})


def test_block_lanczos_varbl():
    """VarBL (Alg. 2): with one gradient (l = 1) it is Alg. 1's Lanczos; T is Q^T A Q; the
    increment is the Galerkin solution -Q (Q^T (I + A) Q)^{-1} Q^T g on the block Krylov space;
    with a full space it is exact; the gradient samples are linearisations at the moved state
    with moved observations (zero draws: the gradient itself)."""
    from oracle import bcov
    w, p = _small()
    v = 0.05 * np.random.default_rng(2).standard_normal(p.n)
    x = p.xb + bcov.apply_L(v, p.taps)
    lin = fourdvar.linearize(p, x, v)
    A = fourdvar.dense_A(p, lin)
    A = 0.5 * (A + A.T)
    ap = lambda X: A @ X  # noqa: E731
    # l = 1 against Alg. 1
    dv1, lam1, _, _, _ = fourdvar.block_lanczos(ap, lin.g[:, None], 8, lin.g)
    dzl, laml, _ = fourdvar.lanczos_varcg(ap, lin.g, 8)
    assert np.allclose(lam1, laml, rtol=1e-10, atol=1e-10 * laml[0])
    assert np.linalg.norm(dv1 - dzl) <= 1e-9 * np.linalg.norm(dzl)
    # gradient samples
    rng = np.random.default_rng(6)
    l = 4
    eb = rng.standard_normal((p.n, l))
    eo = rng.standard_normal((p.nobs, l))
    assert np.allclose(fourdvar.gradient_sample(p, x, v, None, np.zeros(p.nobs)), lin.g, atol=1e-13)
    Bg = np.stack([fourdvar.gradient_sample(p, x, v, None if j == 0 else eb[:, j], eo[:, j])
                   for j in range(l)], axis=1)
    pj = fourdvar.Problem(p.n, p.nsteps, p.h, p.F, p.obs_step, p.obs_idx,
                          p.y - eo[:, 2] / np.sqrt(p.rinv), p.rinv, p.xb, p.taps)
    g2 = fourdvar.linearize(pj, x + bcov.apply_L(eb[:, 2], p.taps), v + eb[:, 2]).g
    assert np.array_equal(Bg[:, 2], g2)
    # block Krylov space: T = Q^T A Q, Galerkin increment
    dv, lam, U, Q, T = fourdvar.block_lanczos(ap, Bg, 5, lin.g)
    assert np.max(np.abs(Q.T @ Q - np.eye(Q.shape[1]))) < 1e-12
    assert np.max(np.abs(Q.T @ A @ Q - T)) <= 1e-10 * np.max(np.abs(T))
    gal = -Q @ np.linalg.solve(Q.T @ (Q + A @ Q), Q.T @ lin.g)
    assert np.linalg.norm(dv - gal) <= 1e-10 * np.linalg.norm(gal)
    # full space (10 x 4 = n): exact
    dvf, _, _, _, _ = fourdvar.block_lanczos(ap, Bg, 10, lin.g)
    dz = -np.linalg.solve(np.eye(p.n) + A, lin.g)
    assert np.linalg.norm(dvf - dz) <= 1e-8 * np.linalg.norm(dz)
