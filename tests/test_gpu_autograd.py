"""Checkpointed observation map, its tangent and adjoint, and the PyTorch autograd wrapper.

A handle built with ckpt_stride = c keeps the Lorenz-96 trajectory only at every c-th
step; the tangent and adjoint recompute one segment's RK4 stage states at a time. Checked
against the FP64 oracle (observed values, tangent-linear and adjoint window sweeps),
against the same library's whole-window TL/AD calls, with the adjoint dot-product identity,
and through torch.autograd (reverse mode against central finite differences and the
library's own 4D-Var gradient; forward mode against the tangent). Windows whose length is
not a multiple of c and observations on segment boundaries and at step 0 are included.
"""

import numpy as np
import pytest

from oracle import fourdvar, l96
from tests._problems import oracle_problem, rel, to_np

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _handle(p, c, m_max=4):
    from paper_1906_01413_amd import Riot
    return Riot(p.n, p.nsteps, p.h, p.F, p.obs_step, p.obs_idx, p.y, p.rinv, p.taps, m_max,
                ckpt_stride=c)


def _with_step0_obs(p):
    """Add observations at step 0 (two variables) to exercise the first segment's step 0."""
    import dataclasses
    extra_i = np.array([0, p.n // 2], dtype=np.int32)
    return dataclasses.replace(
        p, obs_step=np.concatenate([np.zeros(2, np.int32), p.obs_step]),
        obs_idx=np.concatenate([extra_i, p.obs_idx]), y=np.concatenate([np.zeros(2), p.y]),
        rinv=np.concatenate([np.ones(2), p.rinv]))


@pytest.mark.parametrize("c", [8, 7, 40, 1])
def test_checkpointed_map_tangent_adjoint_match_oracle(c):
    _, p = oracle_problem("l96_n40")
    p = _with_step0_obs(p)
    r = _handle(p, c)
    stages, states = l96.trajectory(p.xb, p.nsteps, p.h, p.F)
    ck, obs = r.ckpt_forward(p.xb)
    assert rel(to_np(obs), states[p.obs_step, p.obs_idx]) < 1e-12
    nseg = (p.nsteps + c - 1) // c
    for s in range(nseg + 1):
        step = min(s * c, p.nsteps)
        assert rel(to_np(ck[:, s]), states[step]) < 1e-12, s
    rng = np.random.default_rng(c)
    dX = rng.standard_normal((p.n, 3))
    dObs = r.ckpt_tangent(ck, dX)
    assert rel(to_np(dObs), fourdvar.tangent_window(p, stages, dX)) < 1e-11
    gO = rng.standard_normal((p.nobs, 3))
    gX = r.ckpt_adjoint(ck, gO)
    assert rel(to_np(gX), fourdvar.adjoint_window(p, stages, gO)) < 1e-11
    # adjoint identity on the device results
    lhs = np.sum(to_np(dObs) * gO)
    rhs = np.sum(dX * to_np(gX))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)


def test_checkpointed_equals_whole_window_at_full_size():
    """n = 4096, T = 100, stride 10 against the whole-window TL/AD of a plain handle."""
    import os

    from paper_1906_01413_amd import Riot
    ref = os.path.join(os.path.dirname(__file__), "golden", "ref_l96_n4096_s0.npz")
    if not os.path.exists(ref):
        pytest.skip("reference problem not generated")
    z = dict(np.load(ref, allow_pickle=False))
    args = (int(z["n"]), int(z["nsteps"]), float(z["dt"]), float(z["forcing"]), z["obs_step"],
            z["obs_idx"], z["y"], z["rinv"], z["taps"], 4)
    full = Riot(*args)
    ckh = Riot(*args, ckpt_stride=10)
    print(f"workspace: whole window {full.workspace_bytes / 2**20:.1f} MiB, "
          f"stride 10 {ckh.workspace_bytes / 2**20:.1f} MiB")
    assert ckh.workspace_bytes < full.workspace_bytes
    full.linearize(z["xb"])
    ck, _ = ckh.ckpt_forward(z["xb"])
    rng = np.random.default_rng(5)
    dX = rng.standard_normal((full.n, 4))
    gO = rng.standard_normal((full.nobs, 4))
    assert rel(to_np(ckh.ckpt_tangent(ck, dX)), to_np(full.tl_apply(dX))) < 1e-13
    assert rel(to_np(ckh.ckpt_adjoint(ck, gO)), to_np(full.ad_apply(gO))) < 1e-13


def test_autograd_reverse_mode_matches_finite_differences_and_library_gradient():
    from paper_1906_01413_amd.autograd import observe
    _, p = oracle_problem("l96_n40")
    r = _handle(p, 8)
    y = torch.tensor(p.y, device="cuda")
    rinv = torch.tensor(p.rinv, device="cuda")

    def loss(x):
        d = y - observe(x, r)
        return 0.5 * torch.sum(rinv * d * d)

    x0 = torch.tensor(p.xb, device="cuda", requires_grad=True)
    (g,) = torch.autograd.grad(loss(x0), x0)
    # central differences along random directions: error O(eps^2)
    rng = np.random.default_rng(3)
    for _ in range(3):
        u = torch.tensor(rng.standard_normal(p.n), device="cuda")
        eps = 1e-5
        with torch.no_grad():
            fd = (loss(x0 + eps * u) - loss(x0 - eps * u)).item() / (2 * eps)
        an = torch.dot(g, u).item()
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1.0), (fd, an)
    # the library's 4D-Var gradient at v = 0 is g = -L G^T R^{-1} d = L (d loss / d x)
    full = _handle(p, 0)
    _, gl, _ = full.linearize(p.xb)
    assert rel(to_np(full.apply_L(g)), to_np(gl)) < 1e-11
    # and the oracle's gradient
    lin = fourdvar.linearize(p, p.xb)
    assert rel(to_np(full.apply_L(g)), lin.g) < 1e-11


def test_autograd_forward_mode_is_the_tangent():
    import torch.autograd.forward_ad as fwAD

    from paper_1906_01413_amd.autograd import observe
    _, p = oracle_problem("l96_n40")
    r = _handle(p, 8)
    stages, _ = l96.trajectory(p.xb, p.nsteps, p.h, p.F)
    u = np.random.default_rng(9).standard_normal(p.n)
    with fwAD.dual_level():
        x = fwAD.make_dual(torch.tensor(p.xb, device="cuda"), torch.tensor(u, device="cuda"))
        out = observe(x, r)
        tangent = fwAD.unpack_dual(out).tangent
    assert rel(to_np(tangent), fourdvar.tangent_window(p, stages, u)) < 1e-11
