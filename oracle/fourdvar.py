"""Incremental 4D-Var inner loop: exact solution, RIOT replica, CG and Lanczos.

Notation (Section 2.1, eq. 3): control dz, increment dx = L dz, B = L L^T,
innovation d = y - H(x) (eq. 3's sign), G = stacked Jacobians H_t M_{0->t} of
the observed window, A = L^T G^T R^{-1} G L (the prior-preconditioned Hessian
minus I, Section 2.2 after eq. 4), gradient at dz = 0 of the outer-loop cost in
control variables g = v - L^T G^T R^{-1} d. The inner-loop minimiser is
dz* = -(I + A)^{-1} g.

Observation operator: point values of state variables at window steps; R is
diagonal (entries 1 / rinv).
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import bcov, l96


@dataclass
class Problem:
    """Statement of one inner-loop problem (eq. 2 / eq. 3 inputs)."""

    n: int
    nsteps: int
    h: float
    F: float
    obs_step: np.ndarray
    obs_idx: np.ndarray
    y: np.ndarray
    rinv: np.ndarray
    xb: np.ndarray
    taps: np.ndarray

    @property
    def nobs(self) -> int:
        return int(self.obs_step.size)


def realize_l96(w, draws: dict, taps: np.ndarray | None = None) -> tuple[Problem, np.ndarray]:
    """Build a twin-experiment problem from seeded draws.

    Truth: nonlinear spin-up of the perturbed rest state; observations: truth
    trajectory sampled at the observation points plus noise; background:
    truth + L xi. Returns (problem, truth initial state).
    """
    if taps is None:
        taps = bcov.gaussian_taps(w.ell, w.sigma_b)
    truth0 = l96.forecast(np.asarray(draws["x0"], dtype=np.float64), w.spinup, w.dt, w.forcing)
    _, states = l96.trajectory(truth0, w.nsteps, w.dt, w.forcing)
    obs_step = np.asarray(draws["obs_step"])
    obs_idx = np.asarray(draws["obs_idx"])
    y = states[obs_step, obs_idx] + draws["obs_noise"]
    xb = truth0 + bcov.apply_L(draws["bg_noise"], taps)
    prob = Problem(w.n, w.nsteps, w.dt, w.forcing, obs_step, obs_idx, y,
                   np.asarray(draws["rinv"], dtype=np.float64), xb, taps)
    return prob, truth0


# --------------------------------------------------------------------------
# Linearisation (Alg. 3: integrate and store the trajectory, innovation)
# --------------------------------------------------------------------------

@dataclass
class Linearization:
    stages: np.ndarray   # (T, 4, n) RK4 stage states
    states: np.ndarray   # (T+1, n) trajectory
    d: np.ndarray        # innovation y - H(x) per observation
    g: np.ndarray        # control-space gradient v - L^T G^T R^{-1} d
    J: float             # cost 1/2 v^T v + 1/2 d^T R^{-1} d


def adjoint_window(p: Problem, stages: np.ndarray, forcing: np.ndarray) -> np.ndarray:
    """G^T f: adjoint sweep injecting H_t^T f_t at each observed step.

    ``forcing`` has shape (nobs,) or (nobs, m). Returns lambda_0 (n,) or (n, m).
    """
    shape = (p.n,) + forcing.shape[1:]
    lam = np.zeros(shape, dtype=np.result_type(forcing, stages))
    for t in range(p.nsteps, -1, -1):
        sel = p.obs_step == t
        if np.any(sel):
            np.add.at(lam, p.obs_idx[sel], forcing[sel])
        if t > 0:
            lam = l96.ad_step(stages[t - 1], lam, p.h)
    return lam


def tangent_window(p: Problem, stages: np.ndarray, dx0: np.ndarray) -> np.ndarray:
    """G dx0: tangent-linear sweep sampled at the observations -> (nobs,) or (nobs, m)."""
    dt = np.result_type(dx0, stages)
    out = np.zeros((p.nobs,) + dx0.shape[1:], dtype=dt)
    d = np.array(dx0, dtype=dt)
    for t in range(p.nsteps + 1):
        sel = np.nonzero(p.obs_step == t)[0]
        if sel.size:
            out[sel] = d[p.obs_idx[sel]]
        if t < p.nsteps:
            d = l96.tl_step(stages[t], d, p.h)
    return out


def linearize(p: Problem, x: np.ndarray, v: np.ndarray | None = None) -> Linearization:
    """Outer-loop linearisation at x (Alg. 3 first steps; gradient per eq. 3)."""
    stages, states = l96.trajectory(x, p.nsteps, p.h, p.F)
    d = p.y - states[p.obs_step, p.obs_idx]
    if v is None:
        v = np.zeros(p.n)
    lam0 = adjoint_window(p, stages, p.rinv * d)
    g = v - bcov.apply_L(lam0, p.taps)
    J = 0.5 * float(v @ v) + 0.5 * float(np.sum(p.rinv * d * d))
    return Linearization(stages, states, d, g, J)


def hvp(p: Problem, lin: Linearization, W: np.ndarray) -> np.ndarray:
    """Hessian-probe products A W = L^T G^T R^{-1} G L W (Alg. 3, y_i = A w_i)."""
    W = np.asarray(W, dtype=np.float64)
    z = tangent_window(p, lin.stages, bcov.apply_L(W, p.taps))
    rz = (p.rinv[:, None] * z) if z.ndim == 2 else p.rinv * z
    return bcov.apply_L(adjoint_window(p, lin.stages, rz), p.taps)


def dense_A(p: Problem, lin: Linearization, batch: int = 256) -> np.ndarray:
    """Explicit A formed column by column from HVPs on the identity."""
    A = np.empty((p.n, p.n))
    for c0 in range(0, p.n, batch):
        c1 = min(p.n, c0 + batch)
        E = np.zeros((p.n, c1 - c0))
        E[np.arange(c0, c1), np.arange(c1 - c0)] = 1.0
        A[:, c0:c1] = hvp(p, lin, E)
    return A


def obs_jacobian(p: Problem, lin: Linearization) -> np.ndarray:
    """G (nobs x n) formed from tangent-linear sweeps of the identity."""
    return tangent_window(p, lin.stages, np.eye(p.n))


# --------------------------------------------------------------------------
# Exact inner-loop solution and posterior covariance
# --------------------------------------------------------------------------

@dataclass
class Exact:
    lam: np.ndarray    # eigenvalues of A, descending
    V: np.ndarray      # eigenvectors (columns)
    dz: np.ndarray     # -(I + A)^{-1} g
    dx: np.ndarray     # L dz
    dofs: float        # trace(A (I + A)^{-1})


def exact_solve(p: Problem, A: np.ndarray, g: np.ndarray) -> Exact:
    """Exact minimiser of eq. 3 by Cholesky, and the exact spectrum by eigh."""
    Asym = 0.5 * (A + A.T)
    lam, V = np.linalg.eigh(Asym)
    lam, V = lam[::-1], V[:, ::-1]
    C = np.linalg.cholesky(np.eye(p.n) + Asym)
    dz = -np.linalg.solve(C.T, np.linalg.solve(C, g))
    dx = bcov.apply_L(dz, p.taps)
    dofs = float(np.sum(lam / (1.0 + lam)))
    return Exact(lam, V, dz, dx, dofs)


def exact_posterior(p: Problem, A: np.ndarray):
    """Exact posterior covariances: control space (I+A)^{-1} and state space L P_z L^T."""
    Pz = np.linalg.inv(np.eye(p.n) + 0.5 * (A + A.T))
    Lm = bcov.dense_L(p.n, p.taps)
    return Pz, Lm @ Pz @ Lm.T


# --------------------------------------------------------------------------
# RIOT: randomized SVD of A (Alg. 3, precond = false)
# --------------------------------------------------------------------------

@dataclass
class RSVD:
    lam: np.ndarray     # Ritz values, descending (m)
    V: np.ndarray       # Ritz vectors Q Z (n x m)
    Q: np.ndarray       # orthonormal basis of Y
    Y: np.ndarray       # final Hessian-probe block
    K: np.ndarray       # symmetrised single-pass estimate of Q^T A Q
    k_asym: float       # ||K - K^T|| / ||K|| before symmetrisation


def orth(Y: np.ndarray) -> np.ndarray:
    """Householder QR of Y with R's diagonal made positive (unique Q for full rank)."""
    Q, R = np.linalg.qr(Y)
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s


def rsvd(apply_A, Omega: np.ndarray, q: int = 0) -> RSVD:
    """Randomized eigendecomposition of A as in Alg. 3.

    Y = A Omega; q power steps (Q0 = orth(Y), Omega_eff = Q0, Y = A Q0; the
    power step is Halko et al.'s subspace iteration, which the algorithm itself
    does not list); Q = orth(Y); solve K (Q^T Omega_eff) = Q^T Y; symmetrise K;
    K = Z Lambda Z^T; V = Q Z.
    """
    Om = np.asarray(Omega, dtype=np.float64)
    Y = apply_A(Om)
    for _ in range(q):
        Om = orth(Y)
        Y = apply_A(Om)
    Q = orth(Y)
    B1 = Q.T @ Y
    B2 = Q.T @ Om
    K = np.linalg.solve(B2.T, B1.T).T
    nk = np.linalg.norm(K)
    k_asym = float(np.linalg.norm(K - K.T) / nk) if nk > 0 else 0.0
    K = 0.5 * (K + K.T)
    lam, Z = np.linalg.eigh(K)
    lam, Z = lam[::-1], Z[:, ::-1]
    return RSVD(lam, Q @ Z, Q, Y, K, k_asym)


def proj_residual(Q: np.ndarray, AQ: np.ndarray) -> float:
    """||A Q - Q Q^T A Q||_F / ||A Q||_F for orthonormal Q: zero exactly when span(Q) is an
    invariant subspace of A (the quality measure of a sketch basis)."""
    R = AQ - Q @ (Q.T @ AQ)
    return float(np.linalg.norm(R) / np.linalg.norm(AQ))


def choose_update(lam_k: float) -> str:
    """Adaptive rule of eq. 11: LRA when the last kept eigenvalue is >= 1, else LRU."""
    return "lra" if lam_k >= 1.0 else "lru"


def increment(p: Problem, lam: np.ndarray, V: np.ndarray, g: np.ndarray,
              k: int | None = None, mode: str = "adaptive"):
    """Adaptive increment (eqs. 8-11 in eq. 10's increment form; Alg. 3 update).

    LRA: dz = -sum_i (1 + l_i)^{-1} v_i v_i^T g
    LRU: dz = -(I - sum_i l_i / (1 + l_i) v_i v_i^T) g
    Returns (dz, dx = L dz, dofs = sum l_i / (1 + l_i), mode used).
    """
    k = lam.size if k is None else k
    lk, Vk = lam[:k], V[:, :k]
    if mode == "adaptive":
        mode = choose_update(float(lk[-1]))
    c = Vk.T @ g
    if mode == "lra":
        dz = -(Vk @ (c / (1.0 + lk)))
    elif mode == "lru":
        dz = -(g - Vk @ (c * lk / (1.0 + lk)))
    else:
        raise ValueError(mode)
    dofs = float(np.sum(lk / (1.0 + lk)))
    return dz, bcov.apply_L(dz, p.taps), dofs, mode


def posterior_cov(p: Problem, lam: np.ndarray, V: np.ndarray, k: int | None = None,
                  mode: str = "adaptive", dense: bool = False):
    """Low-rank posterior covariance in state space (eqs. 8, 9 with symmetric L).

    LRU: P_a = B + W diag(-l/(1+l)) W^T;  LRA: P_a = W diag(1/(1+l)) W^T;
    W = L V. Returns (W, coef, diag(P_a), dense P_a or None, mode).
    """
    k = lam.size if k is None else k
    lk, Vk = lam[:k], V[:, :k]
    if mode == "adaptive":
        mode = choose_update(float(lk[-1]))
    W = bcov.apply_L(Vk, p.taps)
    Lm = bcov.dense_L(p.n, p.taps)
    if mode == "lru":
        coef = -lk / (1.0 + lk)
        base_diag = np.sum(Lm * Lm, axis=1)
    else:
        coef = 1.0 / (1.0 + lk)
        base_diag = np.zeros(p.n)
    diag = base_diag + np.sum(W * W * coef[None, :], axis=1)
    P = None
    if dense:
        P = (W * coef[None, :]) @ W.T
        if mode == "lru":
            P = P + Lm @ Lm.T
    return W, coef, diag, P, mode


# --------------------------------------------------------------------------
# Iterative baselines: CG (eq. 4) and the Lanczos form of Alg. 1
# --------------------------------------------------------------------------

def cg(apply_IA, g: np.ndarray, iters: int, rtol: float = 0.0):
    """Hestenes-Stiefel CG on (I + A) dz = -g from dz = 0; returns all iterates."""
    x = np.zeros_like(g)
    r = -g.copy()
    pdir = r.copy()
    rr = float(r @ r)
    r0 = np.sqrt(rr)
    its = []
    for _ in range(iters):
        qv = apply_IA(pdir)
        alpha = rr / float(pdir @ qv)
        x = x + alpha * pdir
        r = r - alpha * qv
        its.append(x.copy())
        rr_new = float(r @ r)
        if rtol > 0 and np.sqrt(rr_new) <= rtol * r0:
            break
        pdir = r + (rr_new / rr) * pdir
        rr = rr_new
    return np.array(its).T if its else np.zeros((g.size, 0))


def krylov_minimizer(apply_A, g: np.ndarray, q: int) -> np.ndarray:
    """eq. 4: dz_q = [Q Q^T (A + I) Q Q^T]^+ b over the Krylov basis of {b, A b, ...}.

    b = -g here (eq. 3's right-hand side in this sign convention); the basis
    is orthonormalised column by column with two Gram-Schmidt passes.
    """
    b = -g
    cols = [b / np.linalg.norm(b)]
    for _ in range(1, q):
        w = apply_A(cols[-1])
        for _ in range(2):
            for c in cols:
                w = w - (c @ w) * c
        cols.append(w / np.linalg.norm(w))
    Q = np.array(cols).T
    M = Q.T @ (apply_A(Q) + Q)
    return Q @ np.linalg.solve(M, Q.T @ b)


def lanczos_varcg(apply_A, g: np.ndarray, m: int):
    """Alg. 1 inner loop: m Lanczos steps with full re-orthogonalisation.

    Returns (dz, ritz values, ritz vectors U = Q Z). With b = g (the gradient),
    the increment is dz = -sum (1 + l_i)^{-1} u_i u_i^T b.
    """
    n = g.size
    Q = np.zeros((n, m + 1))
    alpha = np.zeros(m)
    beta = np.zeros(m)
    Q[:, 0] = g / np.linalg.norm(g)
    used = m
    for i in range(m):
        w = apply_A(Q[:, i])
        alpha[i] = Q[:, i] @ w
        r = w - alpha[i] * Q[:, i]
        if i > 0:
            r = r - beta[i - 1] * Q[:, i - 1]
        for _ in range(2):
            r = r - Q[:, :i + 1] @ (Q[:, :i + 1].T @ r)
        beta[i] = np.linalg.norm(r)
        if beta[i] <= 1e-14 * max(1.0, abs(alpha[i])):
            used = i + 1
            break
        Q[:, i + 1] = r / beta[i]
    T = np.diag(alpha[:used]) + np.diag(beta[:used - 1], 1) + np.diag(beta[:used - 1], -1)
    lam, Z = np.linalg.eigh(T)
    U = Q[:, :used] @ Z
    dz = -(U @ ((U.T @ g) / (1.0 + lam)))
    return dz, lam[::-1], U[:, ::-1]


# --------------------------------------------------------------------------
# Outer loop (Alg. 3 with precond = false) and the full cost of eq. 2
# --------------------------------------------------------------------------

def cost(p: Problem, v: np.ndarray) -> float:
    """eq. 2 written in control variables: x = x_b + L v."""
    x = p.xb + bcov.apply_L(v, p.taps)
    _, states = l96.trajectory(x, p.nsteps, p.h, p.F)
    d = p.y - states[p.obs_step, p.obs_idx]
    return 0.5 * float(v @ v) + 0.5 * float(np.sum(p.rinv * d * d))


def outer_loop(p: Problem, n_outer: int, solver) -> list[dict]:
    """Run n_outer outer loops; solver(lin) -> dz. Records J before each loop."""
    v = np.zeros(p.n)
    x = p.xb.copy()
    hist = []
    for k in range(n_outer):
        lin = linearize(p, x, v)
        dz = solver(k, lin)
        hist.append({"J": lin.J, "gnorm": float(np.linalg.norm(lin.g))})
        v = v + dz
        x = x + bcov.apply_L(dz, p.taps)
    hist.append({"J": cost(p, v), "gnorm": float("nan")})
    return hist


# --------------------------------------------------------------------------
# Deterministic LRA/LRU choice by two nonlinear runs (Section 3.2.1)
# --------------------------------------------------------------------------

def increment_select(p: Problem, lam: np.ndarray, V: np.ndarray, g: np.ndarray,
                     v: np.ndarray | None = None, k: int | None = None):
    """The deterministic alternative to eq. 11's rule suggested in the first-inner-loop
    discussion of the small black-carbon problem: form both the LRA and the LRU increment
    from the same Ritz pairs, integrate the nonlinear model from both updated states, and
    keep the increment whose non-quadratic cost (eq. 2 in control variables, x = x_b + L v)
    is lower. A tie keeps LRA, as eq. 11 does at lambda_k = 1; a candidate whose window
    blows up (non-finite cost) never wins over a finite one.

    Returns (dz, dx, mode, J_lra, J_lru).
    """
    v = np.zeros(p.n) if v is None else np.asarray(v, dtype=np.float64)
    dz_a, dx_a, _, _ = increment(p, lam, V, g, k, "lra")
    dz_u, dx_u, _, _ = increment(p, lam, V, g, k, "lru")
    with np.errstate(over="ignore", invalid="ignore"):
        J_a = cost(p, v + dz_a)
        J_u = cost(p, v + dz_u)
    if not np.isfinite(J_u) or (np.isfinite(J_a) and J_a <= J_u):
        return dz_a, dx_a, "lra", J_a, J_u
    return dz_u, dx_u, "lru", J_a, J_u


# --------------------------------------------------------------------------
# RIOT-PSAS: the randomized solve in observation space (Appendix algorithm)
# --------------------------------------------------------------------------

def psas_hvp(p: Problem, lin: Linearization, W: np.ndarray) -> np.ndarray:
    """A_hat W with A_hat = R^{-1/2} G B G^T R^{-1/2} (p x p), B = L L^T = L^2: one adjoint
    sweep forced by the scaled probe, B, one tangent-linear sweep sampled at the observations,
    scaled again. R is diagonal, so its inverse square-root factor is diag(sqrt(rinv))."""
    W = np.asarray(W, dtype=np.float64)
    D = np.sqrt(p.rinv)
    Dw = (D[:, None] * W) if W.ndim == 2 else D * W
    X = adjoint_window(p, lin.stages, Dw)
    X = bcov.apply_L(bcov.apply_L(X, p.taps), p.taps)
    Z = tangent_window(p, lin.stages, X)
    return (D[:, None] * Z) if Z.ndim == 2 else D * Z


def psas_rhs(p: Problem, lin: Linearization, x: np.ndarray) -> np.ndarray:
    """R^{-1/2} (d - b') with d = y - H(x) (eq. 3's sign) and b' = G (x_b - x): the right-hand
    side of the dual solve at the current outer loop (b' = 0 at the first one, x = x_b)."""
    bp = tangent_window(p, lin.stages, p.xb - np.asarray(x, dtype=np.float64))
    return np.sqrt(p.rinv) * (lin.d - bp)


def psas_increment(p: Problem, lin: Linearization, lam: np.ndarray, U: np.ndarray,
                   rhs: np.ndarray, x: np.ndarray, k: int | None = None, mode: str = "adaptive"):
    """Dual increment from the k leading Ritz pairs (lam, U) of A_hat:
      LRA: dw = R^{-1/2} (sum_i (1 + l_i)^{-1} u_i u_i^T) rhs
      LRU: dw = R^{-1/2} (I - sum_i l_i / (1 + l_i) u_i u_i^T) rhs
    (eq. 11's rule on l_k), dx = B G^T dw, and the new state x_new = x_b + dx: the algorithm's
    update x_{k-1} + B H^T dw is the Gauss-Newton step only from x_b, since its dw already
    carries b' = G (x_b - x_{k-1}) (the two agree at the first outer loop, x = x_b).
    Returns (dw, dx, x_new, mode)."""
    k = lam.size if k is None else k
    lk, Uk = lam[:k], U[:, :k]
    if mode == "adaptive":
        mode = choose_update(float(lk[-1]))
    c = Uk.T @ rhs
    if mode == "lra":
        t = Uk @ (c / (1.0 + lk))
    elif mode == "lru":
        t = rhs - Uk @ (c * lk / (1.0 + lk))
    else:
        raise ValueError(mode)
    dw = np.sqrt(p.rinv) * t
    dx = bcov.apply_L(bcov.apply_L(adjoint_window(p, lin.stages, dw), p.taps), p.taps)
    return dw, dx, p.xb + dx, mode


# --------------------------------------------------------------------------
# Spectral preconditioner and rotation across outer loops (Alg. 3, precond / rotation)
# --------------------------------------------------------------------------

def precond_factor_apply(V: np.ndarray, lt: np.ndarray, X: np.ndarray, power: float) -> np.ndarray:
    """(I + V (lt^power - 1) V^T) X for orthonormal V (n x m_j) and lt = lambda + 1 (m_j):
    power -1/2 is the factor P'_j of eq. 7's spectral preconditioner, +1/2 its inverse."""
    return X + V @ ((lt ** power - 1.0)[:, None] * (V.T @ X)) if X.ndim == 2 else \
        X + V @ ((lt ** power - 1.0) * (V.T @ X))


def precond_apply(levels: list, X: np.ndarray, op: str) -> np.ndarray:
    """P_k = P'_1 P'_2 ... P'_{k-1} (the symmetric factors of the earlier outer loops, `levels`
    = [(V_1, lt_1), ..., (V_{k-1}, lt_{k-1})]) applied to X:
      'P'    P X     (P'_{k-1} first),
      'PT'   P^T X   (P'_1 first; every factor is symmetric),
      'Pinv' P^{-1} X = P'_{k-1}^{-1} ... P'_1^{-1} X (P'_1^{-1} first)."""
    X = np.array(X, dtype=np.float64)
    if op == "P":
        for V, lt in reversed(levels):
            X = precond_factor_apply(V, lt, X, -0.5)
    elif op == "PT":
        for V, lt in levels:
            X = precond_factor_apply(V, lt, X, -0.5)
    elif op == "Pinv":
        for V, lt in levels:
            X = precond_factor_apply(V, lt, X, 0.5)
    else:
        raise ValueError(op)
    return X


def precond_hvp(p: Problem, lin: Linearization, levels: list, W: np.ndarray) -> np.ndarray:
    """A_hat_k W = P^T (I + A) P W - W (Alg. 3's preconditioned operator, P = P_k)."""
    PW = precond_apply(levels, W, "P")
    return precond_apply(levels, PW + hvp(p, lin, PW), "PT") - np.asarray(W, dtype=np.float64)


def rotate_probes(levels: list, resolved: list, Omega: np.ndarray) -> np.ndarray:
    """Rotation of Alg. 3: U_k = orthonormal basis (QR) of [P_1 V_1, ..., P_{k-1} V_{k-1}]
    (`resolved`, each block the earlier loop's Ritz vectors mapped by that loop's own
    preconditioner), then omega <- P_k^{-1} (I - U_k U_k^T) omega."""
    if not resolved:
        return np.array(Omega, dtype=np.float64)
    U = orth(np.hstack(resolved))
    Om = np.asarray(Omega, dtype=np.float64)
    return precond_apply(levels, Om - U @ (U.T @ Om), "Pinv")


def riot_outer_loops(p: Problem, probes: list, k_outer: int, precond: bool, rotation: bool,
                     q: int = 0):
    """Alg. 3 over k_outer outer loops with the spectral preconditioner (and rotation).

    At loop k: linearise at x_{k-1} (g = v - L G^T R^{-1} d), b = P_k^T g (reading: the
    algorithm's b + v_{k-1} written for P = I), rotated probes if asked, RSVD of
    A_hat_k = P_k^T (I + A) P_k - I on probes[k] (q power steps), adaptive increment dw from b,
    dv = P_k dw, v_k = v_{k-1} + dv, x_k = x_{k-1} + L dv (so x_k = x_b + L v_k throughout), and
    the new factor P'_k from (V, lambda + 1) with lambda clamped at 0 (A_hat is positive
    semi-definite; a negative Ritz value is rounding). Returns a list of per-loop records
    (J at the linearisation, lambda, mode) and the final (v, x, J).
    """
    v = np.zeros(p.n)
    x = p.xb.copy()
    levels, resolved, hist = [], [], []
    for k in range(k_outer):
        lin = linearize(p, x, v)
        b = precond_apply(levels, lin.g, "PT") if precond else lin.g
        Om = probes[k]
        if precond and rotation:
            Om = rotate_probes(levels, resolved, Om)
        op = (lambda X, lin=lin: precond_hvp(p, lin, levels, X)) if precond else \
            (lambda X, lin=lin: hvp(p, lin, X))
        rs = rsvd(op, Om, q=q)
        mode = choose_update(float(rs.lam[-1]))
        c = rs.V.T @ b
        if mode == "lra":
            dw = -(rs.V @ (c / (1.0 + rs.lam)))
        else:
            dw = -(b - rs.V @ (c * rs.lam / (1.0 + rs.lam)))
        dv = precond_apply(levels, dw, "P") if precond else dw
        hist.append({"J": lin.J, "lam": rs.lam, "V": rs.V, "mode": mode, "dv": dv,
                     "probe_norm_ratio": float(np.linalg.norm(probes[k]) / np.linalg.norm(Om))})
        if precond:
            resolved.append(precond_apply(levels, rs.V, "P"))
            levels.append((rs.V, 1.0 + np.maximum(rs.lam, 0.0)))
        v = v + dv
        x = x + bcov.apply_L(dv, p.taps)
    return hist, v, x, cost(p, v)


# --------------------------------------------------------------------------
# VarBL: block Lanczos started from perturbed gradients (Alg. 2)
# --------------------------------------------------------------------------

def gradient_sample(p: Problem, x: np.ndarray, v: np.ndarray, eps_b: np.ndarray | None,
                    eps_o: np.ndarray) -> np.ndarray:
    """One realisation of the gradient (Alg. 2's sampling loop): the state and control moved by
    the background draw, x_j = x + L eps_b, v_j = v + eps_b (eps_b = None: the unperturbed
    first sample), the observations by the observation draw, y_j = y - R^{1/2} eps_o (eq. 3's
    sign of d; the algorithm writes d with the opposite sign and + L_R eps), and
    b_j = v_j - L G_j^T R^{-1} (y_j - H(M(x_j))) with G_j the Jacobian at x_j."""
    v = np.asarray(v, dtype=np.float64)
    if eps_b is not None:
        x = x + bcov.apply_L(eps_b, p.taps)
        v = v + eps_b
    pj = Problem(p.n, p.nsteps, p.h, p.F, p.obs_step, p.obs_idx,
                 p.y - eps_o / np.sqrt(p.rinv), p.rinv, p.xb, p.taps)
    return linearize(pj, x, v).g


def block_lanczos(apply_A, Bg: np.ndarray, iters: int, g: np.ndarray):
    """Alg. 2's inner loop: Q_1 = orth(gradient samples Bg, n x l); for i = 1 .. iters:
    Y_i = A Q_i, M_i = Q_i^T Y_i, and (i < iters) R = Y_i - Q_i M_i - Q_{i-1} W_{i-1}^T,
    orthogonalised against every earlier block (twice), Q_{i+1} W_i = R (QR). T is the block
    tridiagonal matrix of the M_i and W_i, T = Z Lambda Z^T, U = Q Z, and the increment
    dv = -sum (1 + l_i)^{-1} u_i u_i^T g (the LRA form the algorithm uses; reading: its b is
    the gradient of the current linearisation, as in Alg. 1).
    Returns (dv, lambda descending, U, Q, T)."""
    n, l = Bg.shape
    Q1 = orth(Bg)
    blocks = [Q1]
    Ms, Ws = [], []
    for i in range(iters):
        Qi = blocks[-1]
        Y = apply_A(Qi)
        M = Qi.T @ Y
        Ms.append(M)
        if i == iters - 1:
            break
        R = Y - Qi @ M
        if i > 0:
            R = R - blocks[-2] @ Ws[-1].T
        Qall = np.hstack(blocks)
        for _ in range(2):
            R = R - Qall @ (Qall.T @ R)
        Qn, W = np.linalg.qr(R)
        s = np.sign(np.diag(W))
        s[s == 0] = 1.0
        Qn, W = Qn * s, s[:, None] * W
        blocks.append(Qn)
        Ws.append(W)
    k = len(Ms)
    T = np.zeros((k * l, k * l))
    for i, M in enumerate(Ms):
        T[i * l:(i + 1) * l, i * l:(i + 1) * l] = M
    for i, W in enumerate(Ws):
        T[(i + 1) * l:(i + 2) * l, i * l:(i + 1) * l] = W
        T[i * l:(i + 1) * l, (i + 1) * l:(i + 2) * l] = W.T
    T = 0.5 * (T + T.T)
    lam, Z = np.linalg.eigh(T)
    lam, Z = lam[::-1], Z[:, ::-1]
    Q = np.hstack(blocks)
    U = Q @ Z
    dv = -(U @ ((U.T @ g) / (1.0 + lam)))
    return dv, lam, U, Q, T
