"""Lorenz-96 model, its RK4 integrator, tangent-linear and exact discrete adjoint.

Model: Section 3.1.1, the Lorenz-96 equation dx_i/dt = (x_{i+1} - x_{i-2}) x_{i-1}
- x_i + F with periodic indices. The paper does not name its integrator; this
oracle uses the classical fourth-order Runge-Kutta scheme (reading recorded in
the design notes). Arrays may be 1-D (n,) or 2-D (n, m) with one column per
independent state / perturbation; the base state is always 1-D.
"""

from __future__ import annotations

import numpy as np


def _sh(a: np.ndarray, k: int) -> np.ndarray:
    """Return b with b[i] = a[(i + k) mod n] along axis 0."""
    return np.roll(a, -k, axis=0)


def tendency(x: np.ndarray, F: float) -> np.ndarray:
    """Lorenz-96 right-hand side (Section 3.1.1 model equation)."""
    return (_sh(x, 1) - _sh(x, -2)) * _sh(x, -1) - x + F


def jac_vec(x: np.ndarray, e: np.ndarray) -> np.ndarray:
    """Jacobian of the tendency at x applied to e (tangent-linear of the model equation).

    (J e)_i = (e_{i+1} - e_{i-2}) x_{i-1} + (x_{i+1} - x_{i-2}) e_{i-1} - e_i
    """
    if e.ndim == 2:
        x = x[:, None]
    return (_sh(e, 1) - _sh(e, -2)) * _sh(x, -1) + (_sh(x, 1) - _sh(x, -2)) * _sh(e, -1) - e


def jac_t_vec(x: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Transpose Jacobian at x applied to w (adjoint of the model equation).

    (J^T w)_j = x_{j-2} w_{j-1} - x_{j+1} w_{j+2} + (x_{j+2} - x_{j-1}) w_{j+1} - w_j
    """
    if w.ndim == 2:
        x = x[:, None]
    return (_sh(x, -2) * _sh(w, -1) - _sh(x, 1) * _sh(w, 2)
            + (_sh(x, 2) - _sh(x, -1)) * _sh(w, 1) - w)


def rk4_stages(x: np.ndarray, h: float, F: float):
    """One classical RK4 step: returns (stage states (4, n), next state).

    Stage states are the points where the tendency is evaluated:
    x1 = x, x2 = x + h/2 k1, x3 = x + h/2 k2, x4 = x + h k3.
    """
    k1 = tendency(x, F)
    x2 = x + 0.5 * h * k1
    k2 = tendency(x2, F)
    x3 = x + 0.5 * h * k2
    k3 = tendency(x3, F)
    x4 = x + h * k3
    k4 = tendency(x4, F)
    xn = x + (h / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
    return np.stack([x, x2, x3, x4]), xn


def forecast(x: np.ndarray, nsteps: int, h: float, F: float) -> np.ndarray:
    """Integrate the nonlinear model nsteps steps and return the final state."""
    for _ in range(nsteps):
        _, x = rk4_stages(x, h, F)
    return x


def trajectory(x0: np.ndarray, nsteps: int, h: float, F: float, dtype=np.float64):
    """Nonlinear trajectory of one window (Alg. 3, 'integrate and store trajectory').

    Returns (stages, states): stages[t] holds the four RK4 stage states of step
    t -> t+1 (shape (nsteps, 4, n)); states[t] is x_t for t = 0..nsteps.
    ``dtype`` is the arithmetic type (np.longdouble for the extended-precision floors).
    """
    n = x0.size
    stages = np.empty((nsteps, 4, n), dtype=dtype)
    states = np.empty((nsteps + 1, n), dtype=dtype)
    x = np.array(x0, dtype=dtype)
    h, F = dtype(h), dtype(F)
    states[0] = x
    for t in range(nsteps):
        stages[t], x = rk4_stages(x, h, F)
        states[t + 1] = x
    return stages, states


def tl_step(st: np.ndarray, d: np.ndarray, h: float) -> np.ndarray:
    """Tangent-linear of one RK4 step about stage states st (4, n)."""
    d1 = jac_vec(st[0], d)
    e2 = d + 0.5 * h * d1
    d2 = jac_vec(st[1], e2)
    e3 = d + 0.5 * h * d2
    d3 = jac_vec(st[2], e3)
    e4 = d + h * d3
    d4 = jac_vec(st[3], e4)
    return d + (h / 6.0) * (d1 + 2.0 * d2 + 2.0 * d3 + d4)


def ad_step(st: np.ndarray, lam: np.ndarray, h: float) -> np.ndarray:
    """Exact discrete adjoint of tl_step (transpose of the same linear map).

    Derived by reversing tl_step statement by statement: the adjoint of
    d' = d + h/6 (d1 + 2 d2 + 2 d3 + d4) seeds d1..d4 with h/6, h/3, h/3, h/6
    times lam, then each stage e_s = d + c d_{s-1} passes its adjoint back to
    d and to d_{s-1}.
    """
    a4 = (h / 6.0) * lam
    a3 = (h / 3.0) * lam
    a2 = (h / 3.0) * lam
    a1 = (h / 6.0) * lam
    out = lam.copy()
    s = jac_t_vec(st[3], a4)      # adjoint of e4
    out += s
    a3 = a3 + h * s
    s = jac_t_vec(st[2], a3)      # adjoint of e3
    out += s
    a2 = a2 + 0.5 * h * s
    s = jac_t_vec(st[1], a2)      # adjoint of e2
    out += s
    a1 = a1 + 0.5 * h * s
    out += jac_t_vec(st[0], a1)   # adjoint of d (stage 1 input)
    return out
