"""Workload parameters and seeded random draws.

Nothing here integrates a model or applies a covariance: the module only
states sizes and draws numbers. Streams come from
``numpy.random.SeedSequence(seed).spawn`` in a fixed order so that every
consumer that asks for the same (seed, stream) pair gets the same numbers:

    stream 0  initial-condition perturbation of the truth spin-up
    stream 1  observation noise
    stream 2  background-error draw (multiplied by B^{1/2} by the consumer)
    stream 3  probe blocks, one child stream per outer loop
    stream 4  per-problem structure of batched workloads
    stream 5  tracer source-inversion structure; cycled-run observation noise
"""

from __future__ import annotations

from dataclasses import dataclass, replace

import numpy as np

_N_STREAMS = 6


@dataclass(frozen=True)
class L96Workload:
    """Sizes of one Lorenz-96 4D-Var inner-loop workload.

    Observation layout: variables i with i % var_stride == 0 (0-based) are
    observed at steps step_stride, 2*step_stride, ..., nsteps (step 0 is not
    observed). Observation errors are N(0, obs_sigma^2), R = obs_sigma^2 I.
    The background covariance is a Gaussian correlation of length ``ell``
    cells scaled by sigma_b^2.
    """

    name: str
    n: int
    nsteps: int
    dt: float = 0.05
    forcing: float = 8.0
    spinup: int = 1000
    spinup_sigma: float = 0.1  # std of the N(0, 0.01) initial perturbation
    var_stride: int = 2
    step_stride: int = 4
    obs_sigma: float = 1.0
    ell: float = 2.0
    sigma_b: float = 1.0
    k: int = 20
    p_os: int = 10
    q: int = 1
    outer: int = 3

    @property
    def m(self) -> int:
        return self.k + self.p_os

    @property
    def nobs(self) -> int:
        nv = (self.n + self.var_stride - 1) // self.var_stride
        return nv * (self.nsteps // self.step_stride)


WORKLOADS = {
    # Lorenz-96, n=40, window 40 steps, 200 observations, rank 20 + 10, q=1.
    "l96_n40": L96Workload("l96_n40", n=40, nsteps=40, var_stride=2, step_stride=4,
                           ell=2.0, k=20, p_os=10, q=1, outer=3),
    # Lorenz-96, n=4096, window 100 steps, every 4th variable every 5 steps,
    # length-8 correlation, 256 + 16 probes.
    "l96_n4096": L96Workload("l96_n4096", n=4096, nsteps=100, var_stride=4,
                             step_stride=5, ell=8.0, k=256, p_os=16, q=0, outer=1),
    # Cycled Lorenz-96 window, n=2048, 50 steps, every 2nd variable every 5 steps
    # (10240 observations), length-8 correlation; run for CYCLED["cycles"] windows.
    "l96_n2048": L96Workload("l96_n2048", n=2048, nsteps=50, var_stride=2,
                             step_stride=5, ell=8.0, k=112, p_os=16, q=0, outer=1),
}


def workload(name: str, **overrides) -> L96Workload:
    """Return a named workload, optionally with some fields replaced."""
    w = WORKLOADS[name]
    return replace(w, **overrides) if overrides else w


def obs_locations(n: int, nsteps: int, var_stride: int, step_stride: int):
    """Observation (step, variable) pairs, sorted by step then variable."""
    steps = np.arange(step_stride, nsteps + 1, step_stride, dtype=np.int32)
    vars_ = np.arange(0, n, var_stride, dtype=np.int32)
    obs_step = np.repeat(steps, vars_.size).astype(np.int32)
    obs_idx = np.tile(vars_, steps.size).astype(np.int32)
    return obs_step, obs_idx


def _streams(seed: int):
    return np.random.SeedSequence(seed).spawn(_N_STREAMS)


def l96_draws(w: L96Workload, seed: int) -> dict:
    """Random draws that define one realisation of a Lorenz-96 workload.

    Returns standard-normal noise arrays; scaling by the workload's sigmas
    is plain multiplication, done here so every consumer uses identical
    numbers. The background draw is left unscaled (the consumer multiplies
    it by its own B^{1/2}).
    """
    ss = _streams(seed)
    g0 = np.random.default_rng(ss[0])
    g1 = np.random.default_rng(ss[1])
    g2 = np.random.default_rng(ss[2])
    obs_step, obs_idx = obs_locations(w.n, w.nsteps, w.var_stride, w.step_stride)
    return {
        "x0": w.forcing + w.spinup_sigma * g0.standard_normal(w.n),
        "obs_noise": w.obs_sigma * g1.standard_normal(obs_step.size),
        "bg_noise": g2.standard_normal(w.n),
        "obs_step": obs_step,
        "obs_idx": obs_idx,
        "rinv": np.full(obs_step.size, 1.0 / (w.obs_sigma ** 2)),
    }


def probe_block(seed: int, outer: int, n: int, m: int) -> np.ndarray:
    """Gaussian probe block Omega (n x m, Fortran order) for one outer loop."""
    ss = _streams(seed)[3].spawn(outer + 1)[outer]
    g = np.random.default_rng(ss)
    return np.asfortranarray(g.standard_normal((n, m)))


# Batches of independent Lorenz-96 problems of uneven size: n uniform on
# {40, 80, ..., 2040} plus 2048, window uniform on 20..200 steps, a random
# fraction rho ~ U[0.25, 0.5] of the variables observed every 4th step, R = I,
# Gaussian B of length 2 cells, m = min(n/2, 128) + 8 probes. The truth is spun
# up 300 steps (about 40 e-folding times of the model's leading Lyapunov mode),
# shorter than the single-problem recipe to keep a 1000-problem batch cheap.
BATCH_N_VALUES = tuple(range(40, 2041, 40)) + (2048,)


def batch_workloads(nprob: int, seed: int):
    """Per-problem (workload, draws) of a seeded batch of uneven problems."""
    ss = _streams(seed)[4]
    rng = np.random.default_rng(ss)
    sizes = rng.choice(np.asarray(BATCH_N_VALUES), size=nprob)
    steps = rng.integers(20, 201, size=nprob)
    rhos = rng.uniform(0.25, 0.5, size=nprob)
    child = ss.spawn(nprob)
    out = []
    for j in range(nprob):
        n, T, rho = int(sizes[j]), int(steps[j]), float(rhos[j])
        m = min(n // 2, 128) + 8
        w = L96Workload(f"batch{j}", n=n, nsteps=T, spinup=300, var_stride=1, step_stride=4,
                        ell=2.0, sigma_b=1.0, k=m - 8, p_os=8, q=0, outer=1)
        g = np.random.default_rng(child[j])
        nv = int(round(rho * n))
        vars_ = np.sort(g.choice(n, size=nv, replace=False)).astype(np.int32)
        st = np.arange(4, T + 1, 4, dtype=np.int32)
        obs_step = np.repeat(st, nv).astype(np.int32)
        obs_idx = np.tile(vars_, st.size).astype(np.int32)
        draws = {
            "x0": w.forcing + w.spinup_sigma * g.standard_normal(n),
            "obs_noise": w.obs_sigma * g.standard_normal(obs_step.size),
            "bg_noise": g.standard_normal(n),
            "obs_step": obs_step,
            "obs_idx": obs_idx,
            "rinv": np.ones(obs_step.size),
        }
        out.append((w, draws))
    return out


# Tracer source inversion on a periodic 2-D grid: grid sizes, wind, diffusion, control
# blocks, observation tracks. "ad2_n512": 512 x 512 cells, 96 steps of dt = 0.1 (Courant
# number (7 + 1) 0.1 + 4 K dt = 0.84), 4 x 4-cell control blocks x 4 time blocks = 65536
# controls, 10 random-walk tracks of 400 samples. "ad2_n64", "ad2_n128_b2": small versions
# for checks.
ADV_GRIDS = {
    "ad2_n512": dict(N=512, T=96, dt=0.1, u0=5.0, u1=2.0, v=1.0, K=0.1, block=4, ntb=4,
                     tracks=10, samples=400),
    "ad2_n64": dict(N=64, T=24, dt=0.1, u0=5.0, u1=2.0, v=1.0, K=0.1, block=4, ntb=4,
                    tracks=10, samples=40),
    # two tiles across x, 2 x 2-cell control blocks
    "ad2_n128_b2": dict(N=128, T=10, dt=0.1, u0=5.0, u1=2.0, v=1.0, K=0.1, block=2, ntb=2,
                        tracks=6, samples=30),
}


def advdiff_draws(name: str, seed: int) -> dict:
    """Seeded inputs of one source-inversion problem: grid, prior emission field E (a sum
    of periodic Gaussian bumps on a floor), observation tracks (one-cell random-walk moves,
    sample times uniform on 1..T, sorted), control-space draw xi, observation noise, and
    the B parameters (exponential correlation length 3 blocks, sigma 0.5, R sigma = 10 %)."""
    spec = dict(ADV_GRIDS[name])
    tracks, samples = spec.pop("tracks"), spec.pop("samples")
    N, T = spec["N"], spec["T"]
    ss = _streams(seed)
    g = np.random.default_rng(ss[5])
    yy, xx = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    E = np.full((N, N), 0.1)
    for _ in range(8):
        cy, cx = g.uniform(0, N, size=2)
        r = g.uniform(N / 32, N / 8)
        a = g.uniform(0.5, 2.0)
        dy = np.minimum(np.abs(yy - cy), N - np.abs(yy - cy))
        dx = np.minimum(np.abs(xx - cx), N - np.abs(xx - cx))
        E += a * np.exp(-(dy * dy + dx * dx) / (2.0 * r * r))
    steps = np.array([[0, 1], [0, -1], [1, 0], [-1, 0]])
    ot, oy, ox = [], [], []
    for _ in range(tracks):
        pos = g.integers(0, N, size=2)
        times = np.sort(g.integers(1, T + 1, size=samples))
        for k in range(samples):
            if k:
                pos = (pos + steps[g.integers(0, 4)]) % N
            ot.append(times[k])
            oy.append(pos[0])
            ox.append(pos[1])
    nb = N // spec["block"]
    ncontrol = spec["ntb"] * nb * nb
    gx = np.random.default_rng(ss[2])
    gn = np.random.default_rng(ss[1])
    return {
        "grid": spec,
        "E": E,
        "obs_t": np.asarray(ot, dtype=np.int32),
        "obs_y": np.asarray(oy, dtype=np.int32),
        "obs_x": np.asarray(ox, dtype=np.int32),
        "xi": gx.standard_normal(ncontrol),
        "obs_noise": gn.standard_normal(len(ot)),
        "ell": 3.0,
        "sigma": 0.5,
        "rel_err": 0.1,
    }


# Cycled Lorenz-96 with a learned sketch proposal: the windows of "l96_n2048" chained for
# 200 cycles (the analysis at a window's start, forecast 50 steps, is the next
# background). Cycles 1..100 provide training data (leading Hessian eigenvectors),
# cycles 101..200 compare the learned proposal (k_net network columns plus p_gauss
# Gaussian probes) with Gaussian sketches of the same size and of m_ref probes. The
# network: `layers` periodic conv1d layers of `width` taps and `channels` channels, input
# the background forecast at `snapshots` evenly spaced steps of the window, output head
# of `segments` segments; Adam for `train_steps` steps of `batch` cycles at rate `lr`,
# samples rotated by random multiples of `shift_step` points (the observation period).
CYCLED = dict(workload="l96_n2048", cycles=200, train_cycles=100, k_net=64, p_gauss=16,
              m_ref=128, exact_every=10, layers=4, channels=64, width=9, snapshots=6,
              segments=16, train_steps=4000, batch=16, lr=1e-3, shift_step=2)


def cycled_draws(seed: int, cycles: int) -> dict:
    """Truth spin-up perturbation, first-background draw (unscaled) and per-cycle
    observation noise (cycles x nobs) of the cycled n = 2048 run."""
    w = WORKLOADS[CYCLED["workload"]]
    ss = _streams(seed)
    g0 = np.random.default_rng(ss[0])
    g2 = np.random.default_rng(ss[2])
    g5 = np.random.default_rng(ss[5])
    obs_step, obs_idx = obs_locations(w.n, w.nsteps, w.var_stride, w.step_stride)
    return {
        "x0": w.forcing + w.spinup_sigma * g0.standard_normal(w.n),
        "bg_noise": g2.standard_normal(w.n),
        "obs_noise": w.obs_sigma * g5.standard_normal((cycles, obs_step.size)),
        "obs_step": obs_step,
        "obs_idx": obs_idx,
        "rinv": np.full(obs_step.size, 1.0 / (w.obs_sigma ** 2)),
    }


def net_init(seed: int, shapes) -> list:
    """He-normal weights (std sqrt(2 / (cin * width))) and zero biases for conv layers of
    the given (cout, cin, width) shapes."""
    g = np.random.default_rng(np.random.SeedSequence(seed).spawn(1)[0])
    out = []
    for cout, cin, width in shapes:
        W = g.standard_normal((cout, cin, width)) * np.sqrt(2.0 / (cin * width))
        out.append((W, np.zeros(cout)))
    return out
