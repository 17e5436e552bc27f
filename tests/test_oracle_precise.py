"""Pins of the oracle's precision certificates (oracle/precise.py) and of the cost J.

* The refined solve of (I + A) dz = -g recovers the exact answer of an integer system whose
  solution is known exactly, far beyond the plain FP64 Cholesky solve, and its certified
  bound holds and is tight.
* The Dot2 residual agrees with exact rational arithmetic within its stated bound.
* The extended-precision Hessian-probe product reproduces the closed-form Fourier multipliers
  at the Lorenz-96 rest state (every variable observed, R = r I) more accurately than FP64.
* ||L||_2 is the largest singular value of the dense circulant.
* The cost of eq. 2 in control variables and the gradient g = v - L^T G^T R^{-1} d agree by
  central differences at v != 0 (a dropped 1/2 on either term of J, or on g, fails).
"""

from fractions import Fraction

import numpy as np
import pytest

from oracle import bcov, fourdvar, precise
from synthetic import l96_draws, workload

EXT = np.longdouble


def _integer_system(n, seed, scale_bits):
    """A = M^T M with M an integer matrix whose rows are scaled by powers of two: every
    entry of A and of g = -(I + A) z is an integer below 2^53, so FP64 holds them exactly."""
    rng = np.random.default_rng(seed)
    B = rng.integers(-3, 4, size=(n, n)).astype(np.float64)
    D = 2.0 ** rng.integers(0, scale_bits, size=n)
    M = D[:, None] * B
    A = M.T @ M
    z = rng.integers(-5, 6, size=n).astype(np.float64)
    g = -(z + A @ z)
    assert np.max(np.abs(A)) < 2.0 ** 52 and np.max(np.abs(g)) < 2.0 ** 52
    return A, g, z


@pytest.mark.parametrize("n,seed,bits", [(64, 1, 12), (256, 3, 16), (512, 4, 15)])
def test_refined_solve_known_answer(n, seed, bits):
    A, g, z = _integer_system(n, seed, bits)
    lam1 = float(np.linalg.eigvalsh(A)[-1])
    ref = precise.refine_solve(A, g)
    err = np.linalg.norm(ref.dz - z) / np.linalg.norm(z)
    bound = ref.bound / np.linalg.norm(z)
    print(f"n={n} lam1={lam1:.1e}: FP64 Cholesky {ref.chol_err:.1e}, refined {err:.1e}, "
          f"certified bound {bound:.1e}")
    assert lam1 > 1e8                          # the plain solve is visibly inexact
    assert ref.chol_err > 1e3 * max(err, 1e-16)
    assert err <= ref.bound / np.linalg.norm(z)  # the bound holds
    assert bound < 1e-12                       # and certifies far below 1e-7


def test_dot2_residual_against_exact_rationals():
    rng = np.random.default_rng(9)
    n = 12
    M = rng.standard_normal((n, n)) * 10.0 ** rng.integers(-3, 6, size=(n, 1))
    A = M.T @ M
    z = rng.standard_normal(n) * 1e-3
    g = rng.standard_normal(n)
    r, e = precise.residual_dot2(A, z, g)
    for i in range(n):
        exact = -Fraction(g[i]) - Fraction(z[i]) - sum(Fraction(A[i, j]) * Fraction(z[j])
                                                       for j in range(n))
        dev = abs(Fraction(r[i]) - exact)
        assert dev <= Fraction(e[i])
        # as accurate as twice FP64: the deviation is at the rounding of the result itself
        assert float(dev) <= 2.3e-16 * abs(float(exact)) + 1e-28 * float(np.abs(A[i]) @ np.abs(z))
    # plain FP64 would miss by the cancellation's size; Dot2 does not
    plain = -g - z - A @ z
    assert np.max(np.abs(plain - r)) > 0.0


def _rest_problem(n, T, h, F, r, steps, taps):
    obs_step = np.repeat(np.array(steps, dtype=np.int32), n)
    obs_idx = np.tile(np.arange(n, dtype=np.int32), len(steps))
    return fourdvar.Problem(n, T, h, F, obs_step, obs_idx, np.full(obs_step.size, F),
                            np.full(obs_step.size, 1.0 / r), np.full(n, F), taps)


def test_extended_hvp_matches_closed_form_better_than_fp64():
    # At x = F 1 with every variable observed at steps S and R = r I, A is circulant with
    # eigenvalue l_w^2 sum_{s in S} |R4(h mu_w)|^{2 s} / r, mu_w = F (e^{iw} - e^{-2iw}) - 1,
    # R4 the degree-4 Taylor polynomial; cos(w i) is an eigenvector.
    n, T, h, F, r = 24, 40, 0.05, 8.0, 0.5
    taps = bcov.gaussian_taps(2.0, 0.7)
    steps = [0, 13, 40]
    p = _rest_problem(n, T, h, F, r, steps, taps)
    lin = fourdvar.linearize(p, p.xb)
    pi = EXT("3.14159265358979323846264338327950288")
    tx = np.asarray(taps, dtype=EXT)
    errs_ext, errs_64 = [], []
    for j in (0, 1, 5, 7, 12):
        om = 2 * pi * j / n
        v = np.cos(om * np.arange(n).astype(EXT))
        zz = EXT(h) * (EXT(F) * (np.exp(1j * om) - np.exp(-2j * om)) - 1)
        R4 = 1 + zz + zz * zz / 2 + zz ** 3 / 6 + zz ** 4 / 24
        lw = tx[0] + 2 * sum(tx[d] * np.cos(om * d) for d in range(1, tx.size))
        a = lw * lw * sum(np.abs(R4) ** (2 * s) for s in steps) / EXT(r)
        exact = a * v
        ye = precise.hvp_ext(p, p.xb, v)
        y64 = fourdvar.hvp(p, lin, v.astype(np.float64))
        nrm = np.sqrt(np.sum(exact * exact))
        errs_ext.append(float(np.sqrt(np.sum((ye - exact) ** 2)) / nrm))
        errs_64.append(float(np.sqrt(np.sum((y64 - exact) ** 2)) / nrm))
    print("closed-form error, extended:", [f"{e:.1e}" for e in errs_ext])
    print("closed-form error, FP64:    ", [f"{e:.1e}" for e in errs_64])
    assert max(errs_ext) < 1e-6
    assert sum(errs_ext) < 0.01 * sum(errs_64)
    for ee, e6 in zip(errs_ext, errs_64):
        assert ee <= max(1e-18, 0.1 * e6)


def test_extended_hvp_agrees_with_fp64_on_a_chaotic_window():
    w = workload("l96_n40")
    p, _ = fourdvar.realize_l96(w, l96_draws(w, 0))
    lin = fourdvar.linearize(p, p.xb)
    W = np.random.default_rng(3).standard_normal((p.n, 4))
    a64 = fourdvar.hvp(p, lin, W)
    aex = precise.hvp_ext(p, p.xb, W)
    assert aex.dtype == EXT
    assert float(np.linalg.norm((aex - a64).astype(np.float64)) / np.linalg.norm(a64)) < 1e-9


def test_norm_L_is_largest_singular_value():
    for n, ell in ((40, 2.0), (64, 8.0), (30, 1.5)):
        taps = bcov.gaussian_taps(ell, 0.9)
        s = np.linalg.svd(bcov.dense_L(n, taps), compute_uv=False)
        assert abs(precise.norm_L(n, taps) - s[0]) <= 1e-13 * s[0]


def test_certify_reference_n40():
    w = workload("l96_n40")
    p, _ = fourdvar.realize_l96(w, l96_draws(w, 0))
    lin = fourdvar.linearize(p, p.xb)
    A = fourdvar.dense_A(p, lin)
    A = 0.5 * (A + A.T)
    c = precise.certify(p, p.xb, A, lin.g)
    ex = fourdvar.exact_solve(p, A, lin.g)
    # the plain Cholesky solve lies within its own rounding of the certified one
    assert np.linalg.norm(ex.dx - c["dx"]) / np.linalg.norm(c["dx"]) < 1e-11
    assert c["floor_la"] < 1e-14 and c["floor_op"] < 1e-9
    assert c["floor"] < 1e-7  # 1e-6 is certifiable at this size


def test_cost_and_gradient_by_central_differences():
    """J(v) = 1/2 v^T v + 1/2 (y - H(M(x_b + L v)))^T R^{-1} (...) (eq. 2 in control
    variables) and g = v - L^T G^T R^{-1} d (eq. 3) at v != 0: the central difference of J
    along e equals g^T e to O(eps^2)."""
    w = workload("l96_n40")
    p, _ = fourdvar.realize_l96(w, l96_draws(w, 0))
    rng = np.random.default_rng(11)
    v = 0.3 * rng.standard_normal(p.n)
    x = p.xb + bcov.apply_L(v, p.taps)
    lin = fourdvar.linearize(p, x, v)
    assert abs(lin.J - fourdvar.cost(p, v)) <= 1e-12 * abs(lin.J)
    errs = []
    for k in range(3):
        e = rng.standard_normal(p.n)
        e /= np.linalg.norm(e)
        ge = float(lin.g @ e)
        row = []
        for eps in (2e-4, 1e-4):
            fd = (fourdvar.cost(p, v + eps * e) - fourdvar.cost(p, v - eps * e)) / (2 * eps)
            row.append(abs(fd - ge) / abs(ge))
        errs.append(row)
        assert row[0] < 1e-5
        # second order: halving eps cuts the error about four times
        assert row[1] < 0.4 * row[0] or row[1] < 1e-9
    print("central-difference relative errors:", errs)


def test_lowprec_products_reduce_to_fp64_and_differ_at_fp32_rounding():
    """hvp_lowprec / grad_lowprec in FP64 are the oracle's own product and gradient bit for
    bit (same steps, same order); in FP32 they differ from them at FP32 rounding level."""
    w = workload("l96_n40")
    p, _ = fourdvar.realize_l96(w, l96_draws(w, 0))
    lin = fourdvar.linearize(p, p.xb)
    W = np.random.default_rng(5).standard_normal((p.n, 3))
    assert np.array_equal(precise.hvp_lowprec(p, lin, W, dtype=np.float64), fourdvar.hvp(p, lin, W))
    assert np.array_equal(precise.grad_lowprec(p, lin, dtype=np.float64), lin.g)
    e_h = np.linalg.norm(precise.hvp_lowprec(p, lin, W) - fourdvar.hvp(p, lin, W)) / \
        np.linalg.norm(fourdvar.hvp(p, lin, W))
    e_g = np.linalg.norm(precise.grad_lowprec(p, lin) - lin.g) / np.linalg.norm(lin.g)
    print(f"FP32 sweeps vs FP64: products {e_h:.1e}, gradient {e_g:.1e}")
    for e in (e_h, e_g):
        assert 1e-9 < e < 1e-4
