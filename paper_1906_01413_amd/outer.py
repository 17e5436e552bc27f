"""Outer loops of incremental 4D-Var with the RIOT inner loop (Alg. 3), through the C ABI.

Every numerical step is a library call; this module only sequences them and keeps the
device buffers of the preconditioner levels alive between loops.

riot_outer_loops runs Alg. 3 with or without the spectral preconditioner (eqs. 6-7) and the
rotation of the probes: at loop k, linearise at x_{k-1}; b = P_k^T g (the algorithm's
b + v_{k-1}, written for P = I, read as P_k^T applied to the whole gradient); probes rotated
to P_k^{-1} (I - U_k U_k^T) omega when asked; Ritz pairs of A_hat_k = P_k^T (I + A) P_k - I
through the sketch handle; the adaptive increment dw from b; dv = P_k dw; v_k = v_{k-1} + dv,
x_k = x_{k-1} + L dv; then the factor P'_k from the new pairs.
"""

from __future__ import annotations

import torch

from .riot import Sketch


def riot_outer_loops(r, xb, probes, k_outer, precond=False, rotation=False, q=0, p_os=0):
    """r: a Riot handle (m_max >= the probes' width); xb: background [n] (device or host);
    probes: k_outer probe blocks [n x m] (device, column-major). Without the preconditioner
    the inner loop is riot_rsvd (q power steps; p_os of the m probes counted as oversampling)
    and riot_increment. Returns (records, v, x, J), records[k] = dict(J = cost at the
    linearisation, lam = Ritz values, mode = update)."""
    dev = r.device
    n = r.n
    x = torch.tensor(xb, dtype=torch.float64, device=dev) if not torch.is_tensor(xb) else xb.clone()
    v = torch.zeros(n, dtype=torch.float64, device=dev)
    levels, resolved, recs = [], [], []
    J = None
    for k in range(k_outer):
        d, g, J = r.linearize(x, v=v)
        m = probes[k].shape[1]
        if not precond:
            lam, V, _ = r.rsvd(m - p_os, p_os, q=q, Omega=probes[k], want_info=False)
            dz, _, _, mode = r.increment(lam, V, g)
            recs.append({"J": J, "lam": lam.detach().cpu().numpy(), "mode": mode})
            r.outer_update(dz, v, x)
            continue
        sk = Sketch(n, m, device=dev)
        b = g.clone()
        if precond and levels:
            r.precond_apply(levels, _col(b), "PT")
        Om = probes[k]
        if precond and rotation and resolved:
            cat = torch.cat(resolved, dim=1).t().contiguous().t()
            U = r.orth(cat)
            Om = Om.clone()
            r.project_out(U, Om)
            r.precond_apply(levels, Om, "Pinv")
        if precond:
            Y = r.precond_hess_apply(levels, Om)
        else:
            Y = r.hess_apply(Om)
        lam, V, _ = sk.eig(Om, Y, want_info=False)
        dw, _, mode = sk.increment(lam, V, b)
        dv = dw
        if precond and levels:
            r.precond_apply(levels, _col(dv), "P")
        recs.append({"J": J, "lam": lam.detach().cpu().numpy(), "mode": mode})
        if precond:
            PV = V.clone()
            if levels:
                r.precond_apply(levels, PV, "P")
            resolved.append(PV)
            levels.append((V, lam))
        r.outer_update(dv, v, x)
    _, _, J = r.linearize(x, v=v)
    return recs, v, x, J


def _col(vec):
    """A contiguous [n] tensor seen as an n x 1 column-major block sharing its storage."""
    return vec.view(-1, 1)


def varbl_inner(r, x, v, eps_b, eps_o, iters):
    """One VarBL inner loop (Alg. 2): l gradient samples (the first unperturbed in the state,
    eps_b[:, 0] unused), linearisation at x, block Lanczos with `iters` blocks. eps_b [n x l]
    and eps_o [nobs x l] are device draws. Returns (lambda, U, dz, dx, g)."""
    l = eps_o.shape[1]
    B = torch.empty((l, r.n), dtype=torch.float64, device=r.device).t()
    for j in range(l):
        r.gradient_sample(x, v, None if j == 0 else eps_b[:, j].contiguous(),
                          eps_o[:, j].contiguous(), out=B[:, j])
    _, g, _ = r.linearize(x, v=v, want_cost=False)
    lam, U, dz, dx = r.block_lanczos(B, g, iters)
    return lam, U, dz, dx, g
