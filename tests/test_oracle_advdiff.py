"""Pins of the source-inversion oracle (oracle/advdiff.py) against closed forms and
identities that do not reuse its own formulas."""

import dataclasses

import numpy as np

from oracle import advdiff
from synthetic import advdiff_draws


def _small(N=12, T=8, **over):
    g = advdiff.Grid(N=N, T=T, dt=0.1, u0=5.0, u1=2.0, v=1.0, K=0.1, block=4, ntb=2)
    return dataclasses.replace(g, **over)


def test_stencil_conserves_mass_and_is_monotone():
    g = _small()
    rng = np.random.default_rng(0)
    c = rng.standard_normal((g.N, g.N))
    assert abs(advdiff.step_A(g, c).sum() - c.sum()) < 1e-12 * np.abs(c).sum()
    a0, aW, aS, aE, aN = g.coeffs()
    assert np.all(a0 > 0) and np.all(aW > 0) and aS > 0 and aE > 0  # Courant number <= 1
    cpos = np.abs(c)
    assert np.all(advdiff.step_A(g, cpos) >= 0)


def test_pure_advection_is_a_shift():
    """K = 0, u = 1, v = 0, dt = 1: one cell to the right per step, exactly."""
    g = _small(K=0.0, u0=1.0, u1=0.0, v=0.0, dt=1.0)
    c = np.random.default_rng(1).standard_normal((g.N, g.N))
    assert np.array_equal(advdiff.step_A(g, c), np.roll(c, 1, axis=1))


def test_adjoint_stencil_is_the_transpose():
    g = _small(N=6)
    n = g.N * g.N
    A = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        A[:, k] = advdiff.step_A(g, e.reshape(g.N, g.N)).ravel()
    lam = np.random.default_rng(2).standard_normal((g.N, g.N))
    assert np.max(np.abs(advdiff.step_AT(g, lam).ravel() - A.T @ lam.ravel())) < 1e-14


def test_up_down_are_transposes():
    g = _small()
    rng = np.random.default_rng(3)
    S = rng.standard_normal((g.Nb, g.Nb))
    F = rng.standard_normal((g.N, g.N))
    assert abs(np.sum(advdiff.up(g, S) * F) - np.sum(S * advdiff.down(g, F))) < 1e-12


def _problem():
    return advdiff.realize(advdiff_draws("ad2_n64", 0))


def test_budget_emitted_mass_accumulates():
    """Mass conservation of the transport: total mass at T is dt times all emissions."""
    p = _problem()
    g = p.grid
    s = p.s_true
    S = s.reshape(g.ntb, g.Nb, g.Nb)
    emitted = sum(g.dt * np.sum(p.E * np.exp(advdiff.up(g, S[g.tau(t)]))) for t in range(g.T))
    _, cT = advdiff.forward(g, p.E, s, p.obs)
    assert abs(cT.sum() - emitted) < 1e-11 * emitted


def test_linear_in_emissions():
    p = _problem()
    a, _ = advdiff.forward(p.grid, p.E, p.s_true, p.obs)
    b, _ = advdiff.forward(p.grid, 2.5 * p.E, p.s_true, p.obs)
    assert np.max(np.abs(b - 2.5 * a)) < 1e-13 * np.max(np.abs(a))


def test_tangent_matches_central_differences():
    p = _problem()
    g = p.grid
    rng = np.random.default_rng(4)
    s0 = 0.3 * rng.standard_normal(g.ncontrol)
    ds = rng.standard_normal(g.ncontrol)
    Gd = advdiff.tangent(g, p.E, s0, p.obs, ds)
    errs = []
    for eps in (1e-2, 5e-3):
        fp, _ = advdiff.forward(g, p.E, s0 + eps * ds, p.obs)
        fm, _ = advdiff.forward(g, p.E, s0 - eps * ds, p.obs)
        errs.append(np.linalg.norm((fp - fm) / (2 * eps) - Gd))
    assert 3.0 < errs[0] / errs[1] < 5.0  # second order


def test_adjoint_dot_product():
    p = _problem()
    g = p.grid
    rng = np.random.default_rng(5)
    s0 = 0.3 * rng.standard_normal(g.ncontrol)
    ds = rng.standard_normal(g.ncontrol)
    f = rng.standard_normal(p.obs.t.size)
    lhs = np.dot(advdiff.tangent(g, p.E, s0, p.obs, ds), f)
    rhs = np.dot(ds, advdiff.adjoint(g, p.E, s0, p.obs, f))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_square_root_of_the_prior():
    """L1 symmetric, L1^2 = C1 (all eigenvalues of the periodic exponential kernel are
    positive here), so L L applied to a unit vector is the sigma^2-scaled correlation."""
    n, ell = 16, 3.0
    L1 = advdiff.sqrt_corr_1d(n, ell)
    i = np.arange(n)
    d = np.minimum(np.abs(i[:, None] - i), n - np.abs(i[:, None] - i))
    C1 = np.exp(-d / ell)
    assert np.min(np.linalg.eigvalsh(C1)) > 0
    assert np.max(np.abs(L1 - L1.T)) < 1e-14
    assert np.max(np.abs(L1 @ L1 - C1)) < 1e-13
    g = _small(N=64, T=8)  # Nb = 16
    e = np.zeros(g.ncontrol)
    e[0] = 1.0
    LLe = advdiff.apply_L(g, L1, 0.5, advdiff.apply_L(g, L1, 0.5, e))
    row = 0.25 * np.outer(C1[0], C1[0]).ravel()
    assert np.max(np.abs(LLe[: g.Nb * g.Nb] - row)) < 1e-13
    assert np.max(np.abs(LLe[g.Nb * g.Nb:])) == 0.0
