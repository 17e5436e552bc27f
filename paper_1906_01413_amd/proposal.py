"""Cycled Lorenz-96 4D-Var with a learned sketch proposal.

Alg. 3 needs a probe block whose range covers the dominant eigenvectors of the
prior-preconditioned Hessian A (Section 2.2). Across assimilation cycles those
eigenvectors follow the flow, so a network that reads the background state can propose
most of the block. Here a periodic 1-D conv net (C ABI riot_net_*) maps the background
x_b of a cycle to k_net columns; p_gauss Gaussian probes complete the block, and the
projected residual rho = ||A Q - Q Q^T A Q||_F / ||A Q||_F judges the result, with a
plain Gaussian sketch of m_ref probes as the fallback.

Every step runs in the library: truth and background forecasts (riot_forecast), truth
observations (the innovation at the truth with y = 0 is -H(M(x_t))), the RSVD
(riot_rsvd), the increment (riot_increment, eqs. 8-11), the judge (riot_hess_apply +
riot_proj_residual), the exact increment for error checks (riot_cg to 1e-12), and the
network's forward, loss, backward and Adam kernels. PyTorch holds device memory only.
"""

from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np
import torch

from .riot import ProposalNet, Riot, gaussian_taps


@dataclass
class CycleStats:
    """Per-cycle results of the comparison at one background (same A for every method)."""
    cycle: int
    rho: dict = field(default_factory=dict)        # method -> projected residual
    capture: dict = field(default_factory=dict)    # method -> weighted capture of ref. V_64
    dx_err: dict = field(default_factory=dict)     # method -> ||dx - dx*|| / ||dx*|| (exact cycles)
    ms: dict = field(default_factory=dict)         # method -> sketch + eigen-solve time
    cg_iters: int = 0                              # CG iterations of the exact increment
    fallback: bool = False


class CycledL96:
    """A twin experiment of chained 4D-Var windows (n, T, observations of the workload),
    one outer loop per cycle, driven by the library."""

    def __init__(self, w, draws, m_max, device="cuda"):
        self.w, self.dr, self.dev = w, draws, torch.device(device)
        nobs = draws["obs_step"].size
        self.r = Riot(w.n, w.nsteps, w.dt, w.forcing, draws["obs_step"], draws["obs_idx"],
                      np.zeros(nobs), draws["rinv"], gaussian_taps(w.ell, w.sigma_b), m_max,
                      device=device)
        self.zero_y = torch.zeros(nobs, dtype=torch.float64, device=self.dev)
        x0 = torch.tensor(draws["x0"], device=self.dev)
        self.truth = self.r.forecast(x0, w.spinup)
        self.xb = self.truth + self.r.apply_L(torch.tensor(draws["bg_noise"], device=self.dev))
        self.cycle = 0

    def observe(self):
        """Truth observations of this cycle's window, then linearise at the background:
        returns the gradient g (eq. 3 at dz = 0) and the cost J."""
        r = self.r
        r.set_obs(self.zero_y)
        d, _, _ = r.linearize(self.truth, want_cost=False)
        noise = torch.tensor(self.dr["obs_noise"][self.cycle], device=self.dev)
        r.set_obs(noise - d)
        _, g, J = r.linearize(self.xb)
        return g.clone(), J

    def window_states(self, snapshots: int):
        """The network's input for this cycle: the background forecast at `snapshots` evenly
        spaced steps of the window (step 0 = x_b), shape (snapshots, n)."""
        xs = [self.xb]
        if snapshots > 1:
            stride = self.w.nsteps // (snapshots - 1)
            for _ in range(snapshots - 1):
                xs.append(self.r.forecast(xs[-1], stride))
        return torch.stack(xs)

    def advance(self, dx):
        """Analysis x_a = x_b + dx at the window start; both runs forecast one window."""
        T = self.w.nsteps
        self.xb = self.r.forecast(self.xb + dx, T)
        self.truth = self.r.forecast(self.truth, T)
        self.cycle += 1


def _timed(fn):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, (time.perf_counter() - t0) * 1e3


def weighted_capture(Q, Vref, w):
    """sum_i w_i ||Q^T v_i||^2 / sum_i w_i for orthonormal Q: the share of the reference
    eigenvectors (weights w) inside span(Q). An evaluation metric, computed on the host."""
    Qh, Vh, wh = (t.cpu().numpy() for t in (Q, Vref, w))
    c = np.sum((Qh.T @ Vh) ** 2, axis=0)
    return float(np.sum(wh * c) / np.sum(wh))


def collect(exp: CycledL96, cycles: int, k_net: int, m_ref: int, seed: int, snapshots: int = 1):
    """Cycles 1..cycles with the reference sketch (m_ref Gaussian probes, one power step):
    the leading k_net Ritz pairs of each cycle are the training targets. Also records the
    projected residual of a plain m_ref-probe sketch (q = 0), whose median over these
    cycles is the proposal's fallback threshold."""
    n, r = exp.w.n, exp.r
    X = torch.empty((cycles, snapshots, n), dtype=torch.float64, device=exp.dev)
    V = torch.empty((cycles, k_net, n), dtype=torch.float64, device=exp.dev)
    lam = torch.empty((cycles, k_net), dtype=torch.float64, device=exp.dev)
    rho_ref = []
    for c in range(cycles):
        g, _ = exp.observe()
        X[c] = exp.window_states(snapshots)
        lq, Vq, _ = r.rsvd(m_ref - 16, 16, q=1, seed=seed + 7919 * c, want_info=False)
        V[c] = Vq.t()[:k_net]
        lam[c] = lq[:k_net]
        lp, Vp, _ = r.rsvd(m_ref - 16, 16, q=0, seed=seed + 7919 * c + 1, want_info=False)
        rho_ref.append(r.proj_residual(Vp, r.hess_apply(Vp)))
        _, dx, _, _ = r.increment(lq, Vq, g, k=m_ref - 16, want_host=False)
        exp.advance(dx)
    return X, V, lam, np.asarray(rho_ref)


def train(net: ProposalNet, X, V, lam, steps: int, batch: int, lr: float, seed: int,
          shift_step: int = 0):
    """Adam on the eigenvalue-weighted capture loss over the collected cycles; returns the
    mean batch loss per step. shift_step > 0: each sample is rotated by a random multiple
    of shift_step grid points (state and eigenvectors together), an exact symmetry of the
    problem when the model is translation invariant and the observation network repeats
    with that period."""
    rng = np.random.default_rng(seed)
    ncyc, n = X.shape[0], X.shape[-1]
    losses = []
    order = rng.permutation(ncyc)
    pos = 0
    ar = torch.arange(n, device=X.device)
    for _ in range(steps):
        if pos + batch > ncyc:
            order, pos = rng.permutation(ncyc), 0
        idx = torch.as_tensor(order[pos: pos + batch], device=X.device)
        pos += batch
        xb, Vb, wb = X[idx], V[idx], lam[idx]
        if shift_step:
            s = torch.as_tensor(rng.integers(0, n // shift_step, batch) * shift_step, device=X.device)
            src = (ar[None, :] - s[:, None]) % n          # rolled[b, i] = orig[b, i - s_b]
            xb = torch.gather(xb, 2, src[:, None, :].expand_as(xb))
            Vb = torch.gather(Vb, 2, src[:, None, :].expand_as(Vb))
        losses.append(float(np.mean(net.train_step(xb, Vb, wb, lr))))
    return np.asarray(losses)


def evaluate(exp: CycledL96, net: ProposalNet, cycles: int, k_net: int, p_gauss: int, m_ref: int,
             tau: float, exact_every: int, seed: int, Vref_q: int = 1, snapshots: int = 1):
    """Cycles after training. At each background the learned block [N(x_b), G_p] (m =
    k_net + p_gauss), a Gaussian block of the same size and a Gaussian block of m_ref are
    sketched on the same A; rho judges each. The cycle advances with the learned result,
    or with the m_ref Gaussian one when rho_learned > tau (fallback). Every exact_every-th
    cycle also compares the increments with the exact one (CG to 1e-12) and the captured
    share of a reference eigenbasis (m_ref probes, Vref_q power steps)."""
    n, r = exp.w.n, exp.r
    m = k_net + p_gauss
    out = []
    Om = torch.empty((m, n), dtype=torch.float64, device=exp.dev).t()  # column-major n x m
    for c in range(cycles):
        st = CycleStats(exp.cycle)
        g, _ = exp.observe()
        res = {}

        def learned():
            net.propose(exp.window_states(snapshots), Om)
            r.philox_normal(n, p_gauss, seed + 31 * exp.cycle + 3, out=Om[:, k_net:])
            return r.rsvd(k_net, p_gauss, q=0, Omega=Om, want_info=False)

        (res["learned"], st.ms["learned"]) = _timed(learned)
        (res["gauss_m"], st.ms["gauss_m"]) = _timed(
            lambda: r.rsvd(k_net, p_gauss, q=0, seed=seed + 31 * exp.cycle + 1, want_info=False))
        (res["gauss_ref"], st.ms["gauss_ref"]) = _timed(
            lambda: r.rsvd(m_ref - 16, 16, q=0, seed=seed + 31 * exp.cycle + 2, want_info=False))
        for key, (lm, Vm, _) in res.items():
            st.rho[key] = r.proj_residual(Vm, r.hess_apply(Vm))
        keep = {"learned": k_net, "gauss_m": k_net, "gauss_ref": m_ref - 16}
        incs = {key: r.increment(res[key][0], res[key][1], g, k=keep[key], want_host=False)[1].clone()
                for key in res}
        st.fallback = bool(st.rho["learned"] > tau)
        if exact_every and c % exact_every == 0:
            dz_star, _, st.cg_iters = r.cg(g, 4000, 1e-12)
            dx_star = r.apply_L(dz_star)
            nrm = float(torch.linalg.vector_norm(dx_star))
            for key, dx in incs.items():
                st.dx_err[key] = float(torch.linalg.vector_norm(dx - dx_star)) / nrm
            lq, Vq, _ = r.rsvd(m_ref - 16, 16, q=Vref_q, seed=seed + 31 * exp.cycle + 4,
                               want_info=False)
            for key, (lm, Vm, _) in res.items():
                st.capture[key] = weighted_capture(Vm, Vq[:, :k_net], lq[:k_net])
            # the network's own columns, before the Hessian acts on them
            Qn = torch.as_tensor(np.linalg.qr(Om[:, :k_net].cpu().numpy())[0])
            st.capture["net_columns"] = weighted_capture(Qn, Vq[:, :k_net], lq[:k_net])
            st.capture["net_columns_unweighted"] = weighted_capture(
                Qn, Vq[:, :k_net], torch.ones(k_net, dtype=torch.float64))
        exp.advance(incs["gauss_ref"] if st.fallback else incs["learned"])
        out.append(st)
    return out


def summarize(stats):
    """Medians and means over the evaluated cycles."""
    keys = list(stats[0].rho)
    s = {"cycles": len(stats), "fallbacks": int(sum(x.fallback for x in stats))}
    for extra in ("net_columns", "net_columns_unweighted"):
        vals = [x.capture[extra] for x in stats if extra in x.capture]
        if vals:
            s[extra + "_capture_mean"] = float(np.mean(vals))
    for key in keys:
        s[key] = {
            "rho_median": float(np.median([x.rho[key] for x in stats])),
            "ms_median": float(np.median([x.ms[key] for x in stats])),
        }
        errs = [x.dx_err[key] for x in stats if key in x.dx_err]
        caps = [x.capture[key] for x in stats if key in x.capture]
        if errs:
            s[key]["dx_err_mean"] = float(np.mean(errs))
            s[key]["capture_mean"] = float(np.mean(caps))
    return s


def net_shapes(cfg: dict):
    """(cout, cin, width) of each layer of the configured network, in parameter order."""
    C, W, L = cfg["channels"], cfg["width"], cfg["layers"]
    cins = [cfg["snapshots"]] + [C] * (L - 1)
    couts = [C] * (L - 1) + [cfg["k_net"] // cfg["segments"]]
    return [(co, ci, W) for co, ci in zip(couts, cins)]


def run_experiment(w, draws, cfg: dict, init_params, seed: int = 0, train_cycles=None,
                   test_cycles=None, train_steps=None, device="cuda"):
    """The whole cycled comparison: collect training data over train_cycles cycles, train
    the network from init_params ([(W, b)] per layer) on the GPU, then evaluate on
    test_cycles further cycles. Returns a summary dict (times in seconds)."""
    train_cycles = cfg["train_cycles"] if train_cycles is None else train_cycles
    test_cycles = cfg["cycles"] - cfg["train_cycles"] if test_cycles is None else test_cycles
    train_steps = cfg["train_steps"] if train_steps is None else train_steps
    k, snap = cfg["k_net"], cfg["snapshots"]
    t0 = time.perf_counter()
    exp = CycledL96(w, draws, cfg["m_ref"], device=device)
    X, V, lam, rho_ref = collect(exp, train_cycles, k, cfg["m_ref"], seed + 1, snapshots=snap)
    torch.cuda.synchronize()
    t_collect = time.perf_counter() - t0
    net = ProposalNet(w.n, k=k, channels=cfg["channels"], layers=cfg["layers"],
                      width=cfg["width"], batch_max=cfg["batch"], segments=cfg["segments"],
                      in_channels=snap, device=device)
    net.set_params(np.concatenate([np.concatenate([np.ravel(W), b]) for W, b in init_params]))
    t0 = time.perf_counter()
    losses = train(net, X, V, lam, train_steps, cfg["batch"], cfg["lr"], seed + 2,
                   shift_step=cfg["shift_step"])
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    tau = float(np.median(rho_ref))
    t0 = time.perf_counter()
    stats = evaluate(exp, net, test_cycles, k, cfg["p_gauss"], cfg["m_ref"], tau,
                     cfg["exact_every"], seed + 5, snapshots=snap)
    t_eval = time.perf_counter() - t0
    s = summarize(stats)
    s.update({
        "train_cycles": train_cycles, "test_cycles": test_cycles, "train_steps": train_steps,
        "tau_rho_gauss_ref_median": tau,
        "train_loss_first": float(losses[0]), "train_loss_last": float(np.mean(losses[-20:])),
        # a random k-dimensional subspace holds k / n of any fixed vector's energy on average
        "random_columns_capture": k / w.n,
        "rho_ratio_learned_over_gauss_m_median": float(np.median(
            [x.rho["learned"] / x.rho["gauss_m"] for x in stats])),
        "collect_s": t_collect, "train_s": t_train, "train_ms_per_step": 1e3 * t_train / train_steps,
        "evaluate_s": t_eval,
    })
    return s
