"""Tracer source inversion on a periodic 2-D grid (test oracle, plain NumPy FP64).

Test infrastructure only: nothing in the product path imports this module.

Model (the paper's black-carbon inversion of Sec. 3.2 uses a transport model whose
emissions enter through a lognormal transform of the controls; this is a synthetic
stand-in of the same character). Concentration c on an N x N periodic grid (dx = 1,
index [y, x]), explicit upwind advection by a positive wind (u(y) = u0 + u1 sin(2 pi y/N)
along x, v along y) and 5-point diffusion K:

  c_{t+1}[y,x] = a0(y) c[y,x] + aW(y) c[y,x-1] + aS c[y-1,x] + aE c[y,x+1] + aN c[y+1,x]
                 + dt e_t[y,x],
  a0 = 1 - dt (u + v) - 4 dt K,  aW = dt (u + K),  aS = dt (v + K),  aE = aN = dt K,

c_0 = 0, emissions e_t = E * exp(s[tau(t)]) upsampled from (N/b) x (N/b) blocks of b x b
cells, tau(t) = t // (T / ntb). Observations: c_{t_o}[y_o, x_o] with t_o in 1..T.
Controls s (ntb x Nb x Nb, time-block major). B = sigma^2 (C1 kron C1) per time block with
C1[i,j] = exp(-d_ij / ell), d the periodic distance on the block axis; its square root is
L = sigma (L1 kron L1), L1 the symmetric square root of C1 (eigenvalues clipped at 0).
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Grid:
    N: int
    T: int
    dt: float
    u0: float
    u1: float
    v: float
    K: float
    block: int
    ntb: int

    @property
    def Nb(self) -> int:
        return self.N // self.block

    @property
    def ncontrol(self) -> int:
        return self.ntb * self.Nb * self.Nb

    def coeffs(self):
        """Stencil coefficients: a0(y), aW(y) per row and the constants aS, aE, aN."""
        y = np.arange(self.N, dtype=np.float64)
        u = self.u0 + self.u1 * np.sin(2.0 * np.pi * y / self.N)
        a0 = 1.0 - self.dt * (u + self.v) - 4.0 * self.dt * self.K
        aW = self.dt * (u + self.K)
        return a0, aW, self.dt * (self.v + self.K), self.dt * self.K, self.dt * self.K

    def tau(self, t: int) -> int:
        return t // (self.T // self.ntb)


def step_A(g: Grid, c: np.ndarray) -> np.ndarray:
    """A c (transport and diffusion of one step) for c of shape (N, N)."""
    a0, aW, aS, aE, aN = g.coeffs()
    return (a0[:, None] * c + aW[:, None] * np.roll(c, 1, axis=1) + aS * np.roll(c, 1, axis=0)
            + aE * np.roll(c, -1, axis=1) + aN * np.roll(c, -1, axis=0))


def step_AT(g: Grid, lam: np.ndarray) -> np.ndarray:
    """A^T lam, written out from the entries of A (row y's coefficients a0(y), aW(y))."""
    a0, aW, aS, aE, aN = g.coeffs()
    return (a0[:, None] * lam + aW[:, None] * np.roll(lam, -1, axis=1)
            + aS * np.roll(lam, -1, axis=0) + aE * np.roll(lam, 1, axis=1)
            + aN * np.roll(lam, 1, axis=0))


def up(g: Grid, S: np.ndarray) -> np.ndarray:
    """Block field (Nb, Nb) -> cell field (N, N)."""
    return np.repeat(np.repeat(S, g.block, axis=0), g.block, axis=1)


def down(g: Grid, F: np.ndarray) -> np.ndarray:
    """Cell field (N, N) -> sums over each block (Nb, Nb) (the transpose of up)."""
    return F.reshape(g.Nb, g.block, g.Nb, g.block).sum(axis=(1, 3))


@dataclass
class Obs:
    t: np.ndarray
    y: np.ndarray
    x: np.ndarray


def forward(g: Grid, E: np.ndarray, s: np.ndarray, obs: Obs):
    """Concentrations at the observations and the final field, for controls s (ncontrol,)."""
    S = s.reshape(g.ntb, g.Nb, g.Nb)
    c = np.zeros((g.N, g.N))
    out = np.zeros(obs.t.size)
    for t in range(g.T):
        c = step_A(g, c) + g.dt * E * np.exp(up(g, S[g.tau(t)]))
        sel = np.nonzero(obs.t == t + 1)[0]
        out[sel] = c[obs.y[sel], obs.x[sel]]
    return out, c


def tangent(g: Grid, E: np.ndarray, s_b: np.ndarray, obs: Obs, ds: np.ndarray) -> np.ndarray:
    """G ds: derivative of the observations at s_b along ds (ncontrol,) or (ncontrol, m)."""
    ds = np.asarray(ds, dtype=np.float64)
    cols = ds.reshape(g.ncontrol, -1)
    Sb = s_b.reshape(g.ntb, g.Nb, g.Nb)
    out = np.zeros((obs.t.size, cols.shape[1]))
    for j in range(cols.shape[1]):
        dS = cols[:, j].reshape(g.ntb, g.Nb, g.Nb)
        dc = np.zeros((g.N, g.N))
        for t in range(g.T):
            tb = g.tau(t)
            W = E * np.exp(up(g, Sb[tb]))
            dc = step_A(g, dc) + g.dt * W * up(g, dS[tb])
            sel = np.nonzero(obs.t == t + 1)[0]
            out[sel, j] = dc[obs.y[sel], obs.x[sel]]
    return out[:, 0] if ds.ndim == 1 else out


def adjoint(g: Grid, E: np.ndarray, s_b: np.ndarray, obs: Obs, f: np.ndarray) -> np.ndarray:
    """G^T f for observation-space f (nobs,) or (nobs, m)."""
    f = np.asarray(f, dtype=np.float64)
    cols = f.reshape(obs.t.size, -1)
    Sb = s_b.reshape(g.ntb, g.Nb, g.Nb)
    out = np.zeros((g.ncontrol, cols.shape[1]))
    for j in range(cols.shape[1]):
        gS = np.zeros((g.ntb, g.Nb, g.Nb))
        lam = np.zeros((g.N, g.N))
        for t in range(g.T, 0, -1):
            sel = np.nonzero(obs.t == t)[0]
            np.add.at(lam, (obs.y[sel], obs.x[sel]), cols[sel, j])
            # lam is the adjoint of c_t; c_t came from step t-1 with emissions tau(t-1)
            tb = g.tau(t - 1)
            W = E * np.exp(up(g, Sb[tb]))
            gS[tb] += down(g, g.dt * W * lam)
            lam = step_AT(g, lam)
        out[:, j] = gS.ravel()
    return out[:, 0] if f.ndim == 1 else out


def sqrt_corr_1d(n: int, ell: float) -> np.ndarray:
    """Symmetric square root of C1[i,j] = exp(-d_ij / ell) (periodic d), eigenvalues >= 0."""
    i = np.arange(n)
    d = np.abs(i[:, None] - i[None, :])
    d = np.minimum(d, n - d)
    C = np.exp(-d / ell)
    w, U = np.linalg.eigh(C)
    return (U * np.sqrt(np.clip(w, 0.0, None))) @ U.T


def apply_L(g: Grid, L1: np.ndarray, sigma: float, z: np.ndarray) -> np.ndarray:
    """L z = sigma (L1 kron L1) z per time block, z (ncontrol,) or (ncontrol, m)."""
    z = np.asarray(z, dtype=np.float64)
    cols = z.reshape(g.ncontrol, -1)
    out = np.empty_like(cols)
    for j in range(cols.shape[1]):
        Z = cols[:, j].reshape(g.ntb, g.Nb, g.Nb)
        out[:, j] = np.stack([sigma * (L1 @ Z[k] @ L1.T) for k in range(g.ntb)]).ravel()
    return out[:, 0] if z.ndim == 1 else out


@dataclass
class Inversion:
    grid: Grid
    E: np.ndarray
    obs: Obs
    y: np.ndarray
    rinv: np.ndarray
    L1: np.ndarray
    sigma: float
    s_true: np.ndarray


def hvp(p: Inversion, s_b: np.ndarray, W: np.ndarray) -> np.ndarray:
    """Prior-preconditioned Hessian minus I applied to W: L G^T R^{-1} G L W."""
    z = tangent(p.grid, p.E, s_b, p.obs, apply_L(p.grid, p.L1, p.sigma, W))
    rz = p.rinv[:, None] * z if z.ndim == 2 else p.rinv * z
    return apply_L(p.grid, p.L1, p.sigma, adjoint(p.grid, p.E, s_b, p.obs, rz))


def gradient(p: Inversion, s_b: np.ndarray, v: np.ndarray | None = None) -> np.ndarray:
    """Control-space gradient v - L G^T R^{-1} d with d = y - H(M(s_b)) (eq. 3's sign)."""
    hx, _ = forward(p.grid, p.E, s_b, p.obs)
    d = p.y - hx
    g = -apply_L(p.grid, p.L1, p.sigma, adjoint(p.grid, p.E, s_b, p.obs, p.rinv * d))
    return g if v is None else v + g


def realize(draws: dict) -> Inversion:
    """Twin experiment from seeded draws: s_true = L xi, y = H(M(s_true)) (1 + 0.1 eps)."""
    gp = draws["grid"]
    g = Grid(**gp)
    L1 = sqrt_corr_1d(g.Nb, draws["ell"])
    s_true = apply_L(g, L1, draws["sigma"], draws["xi"])
    obs = Obs(draws["obs_t"], draws["obs_y"], draws["obs_x"])
    y_true, _ = forward(g, draws["E"], s_true, obs)
    sig = draws["rel_err"] * y_true
    y = y_true + sig * draws["obs_noise"]
    return Inversion(g, draws["E"], obs, y, 1.0 / (sig * sig), L1, draws["sigma"], s_true)
