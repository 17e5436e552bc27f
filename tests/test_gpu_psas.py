"""RIOT-PSAS (Appendix algorithm) on the GPU against the FP64 oracle: the observation-space
operator A_hat = R^{-1/2} G B G^T R^{-1/2}, its randomized eigendecomposition through the sketch
handle on the same probes, the dual increment at the first outer loop and at a later one
(x != x_b), and the full-rank case, where the dual step is the primal Gauss-Newton step.

Two problems: the n = 40 window (200 observations, more than controls) and a window with
fewer observations than controls (n = 256, 8 of every 8th variable... 32 variables at 4
steps = 128 observations), which is where the dual's smaller linear algebra pays off.
"""

import numpy as np
import pytest

from oracle import bcov, fourdvar
from synthetic import probe_block
from tests._problems import oracle_problem, rel, riot_for, to_np

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("name,over", [("l96_n40", {}),
                                       ("l96_n40", dict(n=256, nsteps=24, var_stride=8,
                                                        step_stride=6))])
def test_psas_matches_oracle(name, over):
    from paper_1906_01413_amd import Sketch
    w, p = oracle_problem(name, 1, **over)
    no = p.nobs
    r = riot_for(p, m_max=max(no, 32))
    for outer, v in enumerate((np.zeros(p.n), 0.1 * np.random.default_rng(9).standard_normal(p.n))):
        x = p.xb + bcov.apply_L(v, p.taps)
        lin = fourdvar.linearize(p, x, v)
        d, g, _ = r.linearize(x, v=v)
        # the operator on a few probes
        W = probe_block(21, outer, no, 5)
        e_op = rel(to_np(r.psas_hess_apply(W)), fourdvar.psas_hvp(p, lin, W))
        # right-hand side (b' = G (x_b - x) at the later outer loop)
        rhs = r.psas_rhs(d, None if outer == 0 else p.xb - x)
        rhs_o = fourdvar.psas_rhs(p, lin, x)
        e_rhs = rel(to_np(rhs), rhs_o)
        # randomized eigendecomposition of A_hat on the same probes, then the increment
        m = min(30, no)
        Om = probe_block(22, outer, no, m)
        Y = r.psas_hess_apply(Om)
        lam, U, info = Sketch(no, m).eig(Om, Y)
        ro = fourdvar.rsvd(lambda X: fourdvar.psas_hvp(p, lin, X), Om, q=0)
        e_lam = float(np.max(np.abs(to_np(lam) - ro.lam)) / ro.lam[0])
        dw, dx, mode = r.psas_increment(lam, U, rhs)
        dwo, dxo, _, modeo = fourdvar.psas_increment(p, lin, ro.lam, ro.V, rhs_o, x)
        e_dx = rel(to_np(dx), dxo)
        print(f"{name} n={p.n} p={no} outer {outer}: operator {e_op:.1e}, rhs {e_rhs:.1e}, "
              f"Ritz values {e_lam:.1e} of lam1, dw {rel(to_np(dw), dwo):.1e}, dx {e_dx:.1e}, "
              f"mode {mode}")
        assert e_op < 1e-11 and e_rhs < 1e-11
        assert e_lam < 1e-10 and info.orth_err < 1e-11
        assert mode == modeo
        assert e_dx < 1e-9 and rel(to_np(dw), dwo) < 1e-9
        # full rank: the dual step is the primal Gauss-Newton step (Woodbury)
        Omf = probe_block(23, outer, no, no)
        Yf = r.psas_hess_apply(Omf)
        lamf, Uf, _ = Sketch(no, no).eig(Omf, Yf)
        _, dxf, _ = r.psas_increment(lamf, Uf, rhs)
        A = fourdvar.dense_A(p, lin)
        dz = -np.linalg.solve(np.eye(p.n) + 0.5 * (A + A.T), lin.g)
        x_primal = x + bcov.apply_L(dz, p.taps)
        e_gn = np.linalg.norm(p.xb + to_np(dxf) - x_primal) / np.linalg.norm(x_primal - x)
        print(f"   full rank: dual state vs primal Gauss-Newton step {e_gn:.1e}")
        assert e_gn < 1e-8
