"""Write the oracle reference problems used by the accuracy checks and the benchmark.

Calls only the CPU oracle (oracle/) and the seeded draws (synthetic/). For each
workload and seed it stores the problem statement (background, observations,
R^{-1}, covariance taps), the gradient at the background and the exact
inner-loop minimiser computed two ways (Cholesky of I + A and its
eigendecomposition); their difference is the FP64 floor of the reference.

Usage: python tests/golden/make_refs.py [workload ...]
"""

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import bcov, fourdvar  # noqa: E402
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
    floor = float(np.linalg.norm(dx_eig - ex.dx) / np.linalg.norm(ex.dx))
    out = os.path.join(HERE, f"ref_{name}_s{seed}.npz")
    np.savez_compressed(out, n=p.n, nsteps=p.nsteps, dt=p.h, forcing=p.F, obs_step=p.obs_step,
                        obs_idx=p.obs_idx, y=p.y, rinv=p.rinv, xb=p.xb, taps=p.taps, g=lin.g,
                        J=lin.J, dz=ex.dz, dx=ex.dx, dz_eig=dz_eig, dx_eig=dx_eig, floor=floor,
                        lam=ex.lam, truth0=truth)
    print(f"{out}: floor {floor:.2e}, lam1 {ex.lam[0]:.3e}, #lam>1 {int(np.sum(ex.lam > 1))}, "
          f"{time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    for nm in (sys.argv[1:] or ["l96_n40", "l96_n4096"]):
        make(nm)
