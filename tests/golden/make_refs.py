"""Write the oracle reference problems used by the accuracy checks and the benchmark.

Calls only the CPU oracle (oracle/) and the seeded draws (synthetic/). For each
workload and seed it stores the problem statement (background, observations,
R^{-1}, covariance taps), the gradient and cost at the background, the exact
spectrum, and the exact inner-loop minimiser of eq. 3:
  dz, dx          refined with Dot2 residuals and certified (oracle/precise.py);
  dz_chol, dx_chol the plain FP64 Cholesky solve, dz_eig, dx_eig the solve through
                  the eigendecomposition (both kept to show their own errors);
  floor_la        certified bound of ||dx - dx*|| / ||dx*|| of the refined solution;
  floor_op        the first-order shift of dx* when the FP64 Hessian-probe product is
                  replaced by the extended-precision (np.longdouble) one, measured on dz
                  (op_bound: the cruder norm bound of the same effect);
  floor           floor_la + floor_op (+ the rounding of the stored vectors): how close an
                  increment computed in FP64 can be certified to come to dx*.

Usage: python tests/golden/make_refs.py [workload ...]
"""

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import bcov, fourdvar, precise  # noqa: E402
from synthetic import l96_draws, workload  # noqa: E402


def make(name: str, seed: int = 0):
    t0 = time.time()
    w = workload(name)
    p, truth = fourdvar.realize_l96(w, l96_draws(w, seed))
    lin = fourdvar.linearize(p, p.xb)
    A = fourdvar.dense_A(p, lin)
    A = 0.5 * (A + A.T)
    ex = fourdvar.exact_solve(p, A, lin.g)
    dz_eig = -(ex.V @ ((ex.V.T @ lin.g) / (1.0 + ex.lam)))
    dx_eig = bcov.apply_L(dz_eig, p.taps)
    cert = precise.certify(p, p.xb, A, lin.g)
    dx = cert["dx"]
    chol_err = float(np.linalg.norm(ex.dx - dx) / np.linalg.norm(dx))
    eig_err = float(np.linalg.norm(dx_eig - dx) / np.linalg.norm(dx))
    out = os.path.join(HERE, f"ref_{name}_s{seed}.npz")
    np.savez_compressed(out, n=p.n, nsteps=p.nsteps, dt=p.h, forcing=p.F, obs_step=p.obs_step,
                        obs_idx=p.obs_idx, y=p.y, rinv=p.rinv, xb=p.xb, taps=p.taps, g=lin.g,
                        J=lin.J, dz=cert["dz"], dx=dx, dz_chol=ex.dz, dx_chol=ex.dx,
                        dz_eig=dz_eig, dx_eig=dx_eig, floor=cert["floor"],
                        floor_la=cert["floor_la"], floor_op=cert["floor_op"],
                        op_bound=cert["op_bound"],
                        chol_err=chol_err, eig_err=eig_err, lam=ex.lam, truth0=truth)
    print(f"{out}: floor {cert['floor']:.2e} (certified linear algebra {cert['floor_la']:.2e}, "
          f"FP64 vs extended operator {cert['floor_op']:.2e}, its norm bound "
          f"{cert['op_bound']:.2e}); FP64 Cholesky {chol_err:.2e}, "
          f"eigendecomposition {eig_err:.2e}; lam1 {ex.lam[0]:.3e}, "
          f"#lam>1 {int(np.sum(ex.lam > 1))}, {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    for nm in (sys.argv[1:] or ["l96_n40", "l96_n4096"]):
        make(nm)
