"""Pins of the oracle's Lorenz-96 model, TL and AD against closed forms and invariants.

None of these re-types the oracle's formulas: each checks a property fixed by
the mathematics (conservation identity, integrator order, finite differences,
transpose identity, exact Fourier multipliers at the rest state).
"""

import numpy as np
import pytest

from oracle import bcov, fourdvar, l96
from synthetic import l96_draws, workload


def _chaotic_state(n, seed=0, spin=500):
    rng = np.random.default_rng(seed)
    x = 8.0 + 0.1 * rng.standard_normal(n)
    return l96.forecast(x, spin, 0.05, 8.0)


def test_tendency_energy_identity():
    # sum_i x_i (x_{i+1} - x_{i-2}) x_{i-1} = 0, so x.f(x) = -x.x + F sum(x).
    rng = np.random.default_rng(1)
    for n in (4, 5, 40, 301):
        x = rng.standard_normal(n) * 3 + 2
        lhs = float(x @ l96.tendency(x, 8.0))
        rhs = -float(x @ x) + 8.0 * float(np.sum(x))
        assert abs(lhs - rhs) <= 1e-12 * (abs(rhs) + float(x @ x))


def test_rest_state_is_stationary():
    x = np.full(40, 8.0)
    assert np.all(l96.tendency(x, 8.0) == 0.0)
    assert np.all(l96.forecast(x, 50, 0.05, 8.0) == 8.0)


def test_rk4_is_fourth_order():
    x0 = _chaotic_state(40)
    tau = 0.4
    ref = l96.forecast(x0, 256, tau / 256, 8.0)
    errs = []
    for steps in (8, 16, 32):
        errs.append(np.linalg.norm(l96.forecast(x0, steps, tau / steps, 8.0) - ref))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 12.0 < r1 < 20.0 and 13.0 < r2 < 19.0, (r1, r2)


def _window_tl(stages, d, h):
    for t in range(stages.shape[0]):
        d = l96.tl_step(stages[t], d, h)
    return d


def _window_ad(stages, lam, h):
    for t in range(stages.shape[0] - 1, -1, -1):
        lam = l96.ad_step(stages[t], lam, h)
    return lam


def test_tl_matches_central_differences_second_order():
    n, T, h = 40, 10, 0.05
    x0 = _chaotic_state(n, 2)
    stages, _ = l96.trajectory(x0, T, h, 8.0)
    rng = np.random.default_rng(3)
    d = rng.standard_normal(n)
    tl = _window_tl(stages, d, h)
    errs = []
    for eps in (1e-2, 1e-3):
        fd = (l96.forecast(x0 + eps * d, T, h, 8.0) - l96.forecast(x0 - eps * d, T, h, 8.0)) / (2 * eps)
        errs.append(np.linalg.norm(fd - tl) / np.linalg.norm(tl))
    # central differences converge at slope 2: a tenfold smaller step -> ~100x smaller error
    assert errs[1] < 1e-5
    assert 50.0 < errs[0] / errs[1] < 200.0, errs


def test_adjoint_dot_product():
    n, T, h = 64, 40, 0.05
    x0 = _chaotic_state(n, 4)
    stages, _ = l96.trajectory(x0, T, h, 8.0)
    rng = np.random.default_rng(5)
    for _ in range(5):
        d = rng.standard_normal(n)
        w = rng.standard_normal(n)
        Md = _window_tl(stages, d, h)
        Mtw = _window_ad(stages, w, h)
        lhs, rhs = float(Md @ w), float(d @ Mtw)
        assert abs(lhs - rhs) <= 1e-13 * np.linalg.norm(Md) * np.linalg.norm(w)


def _rk4_poly(z):
    return 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24


def test_tl_and_ad_fourier_multipliers_at_rest_state():
    # At x = F 1 the Jacobian is circulant with eigenvalue F (e^{iw} - e^{-2iw}) - 1
    # and RK4 on a linear constant system is the degree-4 Taylor polynomial.
    n, T, h, F = 36, 7, 0.05, 8.0
    stages, _ = l96.trajectory(np.full(n, F), T, h, F)
    om = 2 * np.pi * np.arange(n) / n
    mu = F * (np.exp(1j * om) - np.exp(-2j * om)) - 1.0
    mult = _rk4_poly(h * mu) ** T
    rng = np.random.default_rng(6)
    v = rng.standard_normal(n)
    tl_exact = np.real(np.fft.ifft(np.fft.fft(v) * mult))
    ad_exact = np.real(np.fft.ifft(np.fft.fft(v) * np.conj(mult)))
    assert np.allclose(_window_tl(stages, v, h), tl_exact, rtol=0, atol=1e-12 * np.linalg.norm(tl_exact))
    assert np.allclose(_window_ad(stages, v, h), ad_exact, rtol=0, atol=1e-12 * np.linalg.norm(ad_exact))


def test_gaussian_square_root_correlation():
    # B = L^2 approximates the Gaussian correlation exp(-d^2 / (2 ell^2)), variance sigma_b^2.
    for ell, tol in ((2.0, 1e-7), (8.0, 1e-12)):
        taps = bcov.gaussian_taps(ell, 1.0)
        n = 4 * taps.size + 16
        Lm = bcov.dense_L(n, taps)
        B = Lm @ Lm
        d = np.minimum(np.arange(n), n - np.arange(n))
        assert np.max(np.abs(B[0] - np.exp(-d * d / (2 * ell * ell)))) < tol
    # apply_L agrees with the dense circulant, including wrap-around for tiny n
    taps = bcov.gaussian_taps(2.0, 1.3)
    for n in (5, 12, 40):
        x = np.random.default_rng(n).standard_normal((n, 3))
        assert np.allclose(bcov.apply_L(x, taps), bcov.dense_L(n, taps) @ x, atol=1e-14)


def test_fixed_point_hessian_spectrum_closed_form():
    # Every variable observed at steps S, R = r I, state at rest: A is circulant with
    # eigenvalues l_w^2 sum_{s in S} |R(h mu_w)|^{2 s} / r (2-fold degenerate).
    n, T, h, F, r = 24, 8, 0.05, 8.0, 0.5
    taps = bcov.gaussian_taps(2.0, 0.7)
    steps = [0, 3, 8]
    obs_step = np.repeat(np.array(steps, dtype=np.int32), n)
    obs_idx = np.tile(np.arange(n, dtype=np.int32), len(steps))
    p = fourdvar.Problem(n, T, h, F, obs_step, obs_idx, np.full(obs_step.size, F),
                         np.full(obs_step.size, 1.0 / r), np.full(n, F), taps)
    lin = fourdvar.linearize(p, p.xb)
    A = fourdvar.dense_A(p, lin)
    om = 2 * np.pi * np.arange(n) / n
    mu = F * (np.exp(1j * om) - np.exp(-2j * om)) - 1.0
    lw = taps[0] + 2 * sum(taps[d] * np.cos(om * d) for d in range(1, taps.size))
    amp = sum(np.abs(_rk4_poly(h * mu)) ** (2 * s) for s in steps)
    expect = np.sort(lw * lw * amp / r)[::-1]
    got = np.sort(np.linalg.eigvalsh(0.5 * (A + A.T)))[::-1]
    assert np.allclose(got, expect, rtol=1e-11, atol=1e-12 * expect[0])
    assert np.allclose(lin.g, 0.0)  # y equals the rest-state values: zero innovation


def test_hessian_symmetric_and_psd():
    w = workload("l96_n40")
    dr = l96_draws(w, 0)
    p, _ = fourdvar.realize_l96(w, dr)
    lin = fourdvar.linearize(p, p.xb)
    A = fourdvar.dense_A(p, lin)
    rng = np.random.default_rng(7)
    for _ in range(4):
        u, v = rng.standard_normal(p.n), rng.standard_normal(p.n)
        Au, Av = A @ u, A @ v
        assert abs(Au @ v - u @ Av) <= 1e-13 * np.linalg.norm(Au) * np.linalg.norm(v)
    lam = np.linalg.eigvalsh(0.5 * (A + A.T))
    assert lam.min() >= -1e-12 * lam.max()
    assert p.nobs == 200
