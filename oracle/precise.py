"""Extended-precision certificates of the exact inner-loop minimiser (the FP64 floors).

TEST INFRASTRUCTURE ONLY (see the package docstring).

RIOT approximates the exact minimiser of eq. 3, dz* = -(I + A)^{-1} g (Section 2.2: the
randomized range finder replaces the Krylov basis of eq. 4), and the increment dx* = L dz*.
When the leading eigenvalue of A is near 1e12, a plain FP64 solve of I + A can be wrong in
the fifth digit, and an FP64 evaluation of A itself carries rounding of order u * lambda_1.
This module bounds both effects with more than FP64 precision instead of estimating them
from the disagreement of two FP64 solvers:

1. Linear-algebra floor (``refine_solve``). Iterative refinement of the FP64 Cholesky
   solution of (I + A) dz = -g, with every residual r = -g - dz - A dz formed by the
   compensated dot product Dot2 (as accurate as twice FP64 precision) from the FP64 entries
   of A. A is positive semi-definite, so every eigenvalue of I + A is at least 1 and
   ||(I + A)^{-1}||_2 <= 1; the bound of ``refine_solve`` uses this with a second residual
   and the rounding bounds of both residuals, so the condition number of I + A enters only
   through the size of the last correction, never as a factor of the bound.
2. Operator floor (``hvp_ext``, ``certify``). The Hessian-probe product applied to the
   refined dz, once in FP64 and once with the whole window (trajectory, RK4 stage states,
   TL, AD, R^{-1}, L) re-integrated in np.longdouble (64-bit significand, unit roundoff
   2^-64 on x86-64) from the same FP64 inputs. To first order a change E of the operator
   moves the minimiser by -(I + A)^{-1} E dz*, so L (I + A)^{-1} (A_fp64 - A_ext) dz is how
   far an FP64 evaluation of the problem moves the increment dx* (a measurement, not a
   bound: it is the shift for the FP64 evaluations at hand).
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import bcov, fourdvar, l96

EXT = np.longdouble
U64 = math.ldexp(1.0, -53)  # unit roundoff of FP64


def ext_problem(p: fourdvar.Problem) -> fourdvar.Problem:
    """The same problem with every real input widened (exactly) to extended precision."""
    return dataclasses.replace(p, h=EXT(p.h), F=EXT(p.F), y=np.asarray(p.y, dtype=EXT),
                               rinv=np.asarray(p.rinv, dtype=EXT),
                               xb=np.asarray(p.xb, dtype=EXT), taps=np.asarray(p.taps, dtype=EXT))


def hvp_ext(p: fourdvar.Problem, x: np.ndarray, W: np.ndarray) -> np.ndarray:
    """A W with the trajectory at x, the TL and AD sweeps, R^{-1} and L all in extended
    precision (the steps of fourdvar.hvp, same order). Returns an extended-precision array."""
    q = ext_problem(p)
    stages, _ = l96.trajectory(np.asarray(x, dtype=EXT), q.nsteps, q.h, q.F, dtype=EXT)
    Wx = np.asarray(W, dtype=EXT)
    z = fourdvar.tangent_window(q, stages, bcov.apply_L(Wx, q.taps))
    rz = (q.rinv[:, None] * z) if z.ndim == 2 else q.rinv * z
    return bcov.apply_L(fourdvar.adjoint_window(q, stages, rz), q.taps)


def norm_L(n: int, taps: np.ndarray) -> float:
    """||L||_2 of the symmetric circulant: max over the DFT frequencies of |symbol|."""
    w = taps.size - 1
    om = 2.0 * np.pi * np.arange(n) / n
    sym = taps[0] + 2.0 * sum(taps[d] * np.cos(om * d) for d in range(1, w + 1))
    return float(np.max(np.abs(sym)))


# Error-free transformations (Knuth's TwoSum; Dekker's TwoProduct with Veltkamp's split, so no
# fused multiply-add is needed) and the compensated dot product Dot2 of Ogita, Rump & Oishi,
# "Accurate sum and dot product" (SIAM J. Sci. Comput. 26, 2005).

_SPLITTER = 134217729.0  # 2^27 + 1


def _two_sum(a, b):
    s = a + b
    bb = s - a
    return s, (a - (s - bb)) + (b - bb)


def _two_prod(a, b):
    p = a * b
    c = _SPLITTER * a
    ah = c - (c - a)
    al = a - ah
    c = _SPLITTER * b
    bh = c - (c - b)
    bl = b - bh
    return p, al * bl - (((p - ah * bh) - al * bh) - ah * bl)


def residual_dot2(A: np.ndarray, z: np.ndarray, g: np.ndarray):
    """r = -g - z - A z for symmetric FP64 A, each component a Dot2 over its n + 2 terms.

    Returns (r, e) with |r - r_exact| <= e component by component: Dot2 is as accurate as a
    sum in twice the working precision, |res - s| <= u |s| + gamma_k^2 sum |terms| with k the
    number of products (Ogita, Rump & Oishi 2005, Prop. 5.3); the TwoProduct errors are summed
    too, so k = 2 (n + 2) is used here, and |s| <= |res| + e gives the factor 2 on u.
    """
    n = z.size
    At = np.asfortranarray(A)           # column j of A = row j (A symmetric)
    s, c = _two_sum(-np.asarray(g, dtype=np.float64), -z)
    for j in range(n):
        pj, qj = _two_prod(At[:, j], -z[j])
        s, e = _two_sum(s, pj)
        c = c + (e + qj)
    r = s + c
    k = 2 * (n + 2)
    gk = k * U64 / (1.0 - k * U64)
    mag = np.abs(A) @ np.abs(z) + np.abs(z) + np.abs(g)
    return r, 2.0 * U64 * np.abs(r) + 1.01 * gk * gk * mag


@dataclasses.dataclass
class Refined:
    dz: np.ndarray          # refined solution (FP64)
    bound: float            # rigorous bound on ||dz - dz*||_2 (dz* = exact solution)
    resid: list[float]      # ||r||_2 before each correction (the FP64 Cholesky start first)
    chol_err: float         # ||dz_chol - dz||_2 / ||dz||_2 of the plain FP64 Cholesky solve


def refine_solve(A: np.ndarray, g: np.ndarray, max_iters: int = 12) -> Refined:
    """Solve (I + A) dz = -g for symmetric positive semi-definite FP64 A (certificate 1 of
    the module doc): FP64 Cholesky, then refinement with Dot2 residuals.

    Certificate at the returned dz: with r the Dot2 residual and c = (I + A)^{-1} r solved
    in FP64, dz* - dz = (I + A)^{-1} r_exact = c + (I + A)^{-1} (r_exact - (I + A) c), and
    ||(I + A)^{-1}||_2 <= 1, so
        ||dz* - dz||_2 <= ||c|| + ||r - fl((I + A) c)|| + ||e_r|| + ||e_2||
    with e_r the Dot2 bound and e_2 = gamma_{n+3} (|A| |c| + |c| + |r|) the FP64 rounding of
    the second residual (Higham, Accuracy and Stability of Numerical Algorithms, Sec. 3.1).
    """
    n = g.size
    A64 = np.asarray(A, dtype=np.float64)
    g64 = np.asarray(g, dtype=np.float64)
    C = np.linalg.cholesky(np.eye(n) + A64)

    def solve64(b):
        return np.linalg.solve(C.T, np.linalg.solve(C, b))

    z0 = solve64(-g64)
    z = z0.copy()
    hist = []
    for _ in range(max_iters):  # until the correction is below the rounding of dz
        r, _ = residual_dot2(A64, z, g64)
        hist.append(float(np.linalg.norm(r)))
        c = solve64(r)
        z = z + c
        if np.linalg.norm(c) <= U64 * np.linalg.norm(z):
            break
    r, er = residual_dot2(A64, z, g64)
    hist.append(float(np.linalg.norm(r)))
    c = solve64(r)
    t = r - (c + A64 @ c)
    k = n + 3
    e2 = (k * U64 / (1.0 - k * U64)) * (np.abs(A64) @ np.abs(c) + np.abs(c) + np.abs(r))
    bound = (float(np.linalg.norm(c)) + float(np.linalg.norm(t)) + float(np.linalg.norm(er))
             + float(np.linalg.norm(e2)))
    chol_err = float(np.linalg.norm(z0 - z) / np.linalg.norm(z))
    return Refined(z, bound, hist, chol_err)


def certify(p: fourdvar.Problem, x: np.ndarray, A: np.ndarray, g: np.ndarray) -> dict:
    """Both certificates for the problem linearised at x (A and g from the FP64 oracle).

    Returns the refined dz and dx = L dz and the relative floors of the increment error
    ||dx - dx*|| / ||dx*||:
      floor_la  rigorous, from the refinement bound (certificate 1);
      floor_op  measured: the first-order shift of dx* when A's FP64 evaluation is replaced
                by the extended-precision one, ||L (I + A)^{-1} E dz|| / ||dx|| with
                E dz = (A_fp64 - A_ext) dz, for both FP64 evaluations of A at hand (the
                product sweeps of fourdvar.hvp and the dense matrix the solve used), the
                larger one; (I + A)^{-1} is applied with the FP64 Cholesky factor;
      op_bound  the cruder bound ||L||_2 ||E dz|| / ||dx|| (||(I + A)^{-1}|| <= 1), which
                ignores that FP64 rounding of the sweeps grows along the unstable, strongly
                observed directions, where (I + A)^{-1} damps it;
      floor     floor_la + floor_op + the rounding of the stored vectors.
    """
    ref = refine_solve(A, g)
    dz64 = ref.dz
    dxx = bcov.apply_L(dz64.astype(EXT), np.asarray(p.taps, dtype=EXT))
    nL = norm_L(p.n, p.taps)
    ndx = float(np.sqrt(np.sum(dxx * dxx)))
    lin = fourdvar.linearize(p, x)
    aex = hvp_ext(p, x, dz64)
    e_sweep = (fourdvar.hvp(p, lin, dz64).astype(EXT) - aex).astype(np.float64)
    e_dense = (np.asarray(A, dtype=np.float64).astype(EXT) @ dz64.astype(EXT) - aex).astype(np.float64)
    C = np.linalg.cholesky(np.eye(p.n) + np.asarray(A, dtype=np.float64))

    def shift(e):
        s = np.linalg.solve(C.T, np.linalg.solve(C, e))
        return float(np.linalg.norm(bcov.apply_L(s, p.taps))) / ndx

    floor_op = max(shift(e_sweep), shift(e_dense))
    op_bound = nL * float(np.linalg.norm(e_sweep)) / ndx
    floor_la = nL * ref.bound / ndx
    return {
        "dz": dz64, "dx": dxx.astype(np.float64),
        "floor_la": floor_la, "floor_op": floor_op, "op_bound": op_bound,
        "floor": floor_la + floor_op + 2.0 * U64,
        "resid": ref.resid, "bound_dz": ref.bound, "norm_L": nL,
        "chol_err": ref.chol_err,
    }


def hvp_lowprec(p: fourdvar.Problem, lin: fourdvar.Linearization, W: np.ndarray,
                dtype=np.float32) -> np.ndarray:
    """A W with the TL and AD sweeps in a narrower type: the FP64 trajectory's stage states
    rounded to ``dtype``, L and L^T in FP64 around the sweeps, R^{-1} rounded to ``dtype``
    (the reduced-precision tangent-linear/adjoint variant). Its distance to fourdvar.hvp is
    the rounding floor that variant cannot beat. Returns FP64."""
    q = dataclasses.replace(p, h=dtype(p.h), rinv=np.asarray(p.rinv, dtype=dtype))
    stages = lin.stages.astype(dtype)
    LW = bcov.apply_L(np.asarray(W, dtype=np.float64), p.taps).astype(dtype)
    z = fourdvar.tangent_window(q, stages, LW)
    rz = (q.rinv[:, None] * z) if z.ndim == 2 else q.rinv * z
    lam0 = fourdvar.adjoint_window(q, stages, rz).astype(np.float64)
    return bcov.apply_L(lam0, p.taps)


def grad_lowprec(p: fourdvar.Problem, lin: fourdvar.Linearization, v: np.ndarray | None = None,
                 dtype=np.float32) -> np.ndarray:
    """g = v - L^T G^T R^{-1} d with the adjoint sweep in ``dtype`` (stage states and the
    R^{-1}-weighted innovation rounded to it; L in FP64), as hvp_lowprec. Returns FP64."""
    q = dataclasses.replace(p, h=dtype(p.h))
    stages = lin.stages.astype(dtype)
    f = (np.asarray(p.rinv) * lin.d).astype(dtype)
    lam0 = fourdvar.adjoint_window(q, stages, f).astype(np.float64)
    g = -bcov.apply_L(lam0, p.taps)
    return g if v is None else g + v
