#!/usr/bin/env python
"""Benchmark of the RIOT inner loop on one MI355X.

One step = one pass of the whole inner loop on the stored synthetic problem:
linearise (trajectory, innovation, gradient), randomized eigendecomposition of
the prior-preconditioned Hessian with device-drawn Philox probes (batched
TL/AD Hessian-probe products, CholeskyQR, K solve, eigen-solve, Ritz
vectors), adaptive increment and low-rank posterior covariance factors.

Prints one JSON line. `value` is Hessian-vector products per second over the
whole step (m (1 + q) products per step). The `roofline` object covers the
dominant kernel, the batched TL/AD integration, timed with HIP events on the
stream it runs on. The `cpu_baseline` object times the FP64 CPU oracle on a
bounded sample of the same workload. The `inner_loop` object reports the time
to reach a relative increment error target, RSVD against plain GPU CG, using
the stored exact solution of the same problem as the yardstick.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_VALU_TFLOPS = 78.6   # 256 CU x 2.4 GHz x 128 FP64 flop/clk (FMA = 2)
PEAK_HBM_GBS = 8000.0

# HBM-side traffic of one 272-column TL/AD launch at n = 4096, T = 100 (E = 16), from two
# rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE; KiB per dispatch). Each counter is scaled by
# what it reads for a plain 256 MiB device copy (FETCH_SIZE 131087 KiB for 262144 KiB read,
# WRITE_SIZE 262144 KiB for 262144 KiB written). Valid only for the kernel source it was
# measured on (sha256 of l96.hip); any other source reports traffic as null.
TLAD_COUNTERS = {
    "l96_sha256": "ed4b794e07e4faaa71aba13c0d74b17c460184496f34ee982540e0daebe220b7",
    "n": 4096, "nsteps": 100, "m": 272,
    "fetch_kib": 119633.75, "write_kib": 53856.0,
    "fetch_scale": 262144.0 / 131086.69, "write_scale": 1.0,
}

WORKLOADS = {
    # name: (k, p_os, q) of the randomized eigendecomposition
    "l96_n4096": (256, 16, 0),
    "l96_n40": (20, 10, 1),
}


def tlad_flops_per_column(n: int, T: int, nobs: int) -> float:
    """Algorithmic FP64 flops of one TL + AD window sweep (FMA = 2 flops).

    Per state element and RK4 step: TL 37 (four Jacobian products at 6, three
    stage updates at 2, the final combination 7), AD 41 (four transposed
    Jacobian products at 7, stage and accumulation updates 13); plus one
    multiply per observation for R^{-1}.
    """
    return float(n) * T * (37 + 41) + nobs


def hvp_flops(n: int, T: int, nobs: int, w: int) -> float:
    """Flops of one Hessian-vector product: TL/AD sweep plus L and L^T (3w + 1 each)."""
    return tlad_flops_per_column(n, T, nobs) + 2.0 * n * (3 * w + 1)


def tlad_traffic_bytes(n: int, T: int, m: int):
    """Counter-derived HBM bytes per TL/AD launch, or None if not measured for this source."""
    import hashlib

    c = TLAD_COUNTERS
    src = os.path.join(ROOT, "paper_1906_01413_amd", "csrc", "l96.hip")
    with open(src, "rb") as fh:
        digest = hashlib.sha256(fh.read()).hexdigest()
    if digest != c["l96_sha256"] or (n, T, m) != (c["n"], c["nsteps"], c["m"]):
        return None
    return 1024.0 * (c["fetch_kib"] * c["fetch_scale"] + c["write_kib"] * c["write_scale"])


def load_problem(name: str, seed: int):
    path = os.path.join(ROOT, "tests", "golden", f"ref_{name}_s{seed}.npz")
    if not os.path.exists(path):
        raise SystemExit(f"missing {path}: run `python tests/golden/make_refs.py {name}`")
    z = np.load(path, allow_pickle=False)
    return {k: z[k] for k in z.files}


_POOL_STATE = {}


def _pool_init(prob):
    """Worker set-up: the oracle problem and its linearisation, built once per process."""
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    from oracle import fourdvar
    p = fourdvar.Problem(int(prob["n"]), int(prob["nsteps"]), float(prob["dt"]),
                         float(prob["forcing"]), prob["obs_step"], prob["obs_idx"], prob["y"],
                         prob["rinv"], prob["xb"], prob["taps"])
    _POOL_STATE["p"] = p
    _POOL_STATE["lin"] = fourdvar.linearize(p, p.xb)


def _pool_hvp(W):
    from oracle import fourdvar
    return fourdvar.hvp(_POOL_STATE["p"], _POOL_STATE["lin"], W)


def cpu_baseline(prob: dict, m: int, budget_s: float = 12.0) -> dict:
    """The FP64 CPU oracle on a bounded sample of the same workload.

    * Hessian-probe products over all host cores: a process pool (one worker per core the
      process may run on, at most 16, one BLAS thread each) applies the oracle's product to
      chunks of one m-column probe block; the main value is that rate.
    * The same products in one process (single-core figure).
    * The oracle's RSVD inner loop (probe products on the pool, then Householder QR, the K
      solve, the eigendecomposition and the increment in the main process) and the oracle's
      plain CG (one product per iteration, sequential), per iteration.
    """
    import multiprocessing as mp

    from oracle import fourdvar
    from synthetic import probe_block

    _pool_init(prob)
    p, lin = _POOL_STATE["p"], _POOL_STATE["lin"]
    cores = min(len(os.sched_getaffinity(0)), 16)
    chunk = max(1, (m + cores - 1) // cores)
    W = probe_block(11, 0, p.n, m)
    parts = [W[:, c: c + chunk] for c in range(0, m, chunk)]
    ctx = mp.get_context("fork")
    with ctx.Pool(cores, initializer=_pool_init, initargs=(prob,)) as pool:
        pool.map(_pool_hvp, [P[:, :1] for P in parts])  # warm every worker
        t0 = time.perf_counter()
        Y = np.concatenate(pool.map(_pool_hvp, parts), axis=1)
        t_pool = time.perf_counter() - t0
        # oracle RSVD inner loop on the pool (k + p_os = m probes, q = 0, all m pairs kept)
        t0 = time.perf_counter()
        Yr = np.concatenate(pool.map(_pool_hvp, parts), axis=1)
        Q = fourdvar.orth(Yr)
        K = np.linalg.solve((Q.T @ W).T, (Q.T @ Yr).T).T
        lam, Z = np.linalg.eigh(0.5 * (K + K.T))
        lam, Z = lam[::-1], Z[:, ::-1]
        fourdvar.increment(p, lam, Q @ Z, lin.g)
        t_rsvd = time.perf_counter() - t0
    del Y
    # one process: products until the budget is spent
    cols, done, t_one = 8, 0, 0.0
    while done < m and t_one < budget_s:
        t0 = time.perf_counter()
        fourdvar.hvp(p, lin, W[:, done: done + cols])
        t_one += time.perf_counter() - t0
        done += cols
    # plain CG, sequential products
    its = 20
    t0 = time.perf_counter()
    fourdvar.cg(lambda x: x + fourdvar.hvp(p, lin, x), lin.g, its)
    t_cg = (time.perf_counter() - t0) / its
    try:
        import numpy.__config__  # noqa: F401
        blas = "1 per worker (OMP_NUM_THREADS)"
    except Exception:
        blas = "unknown"
    return {"value": m / t_pool, "unit": "HVP/s", "cores": cores, "kind": "oracle",
            "sample": f"one {m}-column probe block of Hessian-probe products (NumPy FP64) on the "
                      f"same n={p.n}, T={p.nsteps} problem, {cores} worker processes, "
                      f"{t_pool:.2f} s",
            "host_cores_visible": len(os.sched_getaffinity(0)), "blas_threads": blas,
            "single_core_hvp_per_s": done / t_one,
            "oracle_rsvd_inner_loop_s": t_rsvd,
            "oracle_rsvd_config": f"m={m}, q=0, probe products on {cores} processes",
            "oracle_cg_s_per_iteration": t_cg}


ACCURACY_SWEEP = {
    # (m, q) settings tried in order of cost for the RSVD side
    "l96_n4096": [(272, 0), (272, 1), (544, 0), (544, 1), (1088, 0), (1088, 1)],
    "l96_n40": [(20, 0), (20, 1), (30, 0), (30, 1), (35, 1), (40, 0)],
}


def time_to_accuracy(r, prob, xb, dev, target=1e-6, trials=5, cg_max=None, reps=5):
    """Inner-loop seconds to a relative increment error target, RSVD against plain GPU CG.

    Error = ||dx - dx*|| / ||dx*|| against the stored exact minimiser dx* of the
    same problem (eq. 3). The FP64 floor of that reference (two exact solves
    disagreeing) bounds what can be certified: the target used is
    max(target, 10 x floor). Timing starts with the trajectory already resident
    (the linearisation is included in both legs) and ends with dz resident.
    """
    import torch
    from paper_1906_01413_amd import empty_colmajor

    n, T = r.n, r.nsteps
    dxs = np.asarray(prob["dx"])
    floor = float(prob["floor"])
    # 1e-6 is claimed only where the certified floor is at most a tenth of it
    tgt = target if floor <= 0.1 * target else 10.0 * floor
    name = "l96_n4096" if n == 4096 else "l96_n40"
    stream = torch.cuda.current_stream(dev)

    def timed(fn, nrep):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(nrep):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            fn()
            b.record(stream)
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b) / 1e3)
        return float(np.median(ts))

    def err_of(dx):
        return float(np.linalg.norm(dx.cpu().numpy() - dxs) / np.linalg.norm(dxs))

    d, g, _ = r.linearize(xb, want_cost=False)
    rs_best = None
    sweep = []
    for (m, q) in ACCURACY_SWEEP[name]:
        if m > r.m_max or m > n:
            continue
        errs = []
        for s in range(trials):
            lam, V, _ = r.rsvd(m - min(16, m // 3), min(16, m // 3), q=q, seed=77 + s, want_info=False)
            _, dx, _, mode = r.increment(lam, V, g)
            errs.append(err_of(dx))
        emax = max(errs)

        def run(m=m, q=q):
            r.linearize(xb, want_cost=False, out=(d, g))
            lam, V, _ = r.rsvd(m - min(16, m // 3), min(16, m // 3), q=q, seed=77, want_info=False)
            r.increment(lam, V, g, want_host=False)
        sec = timed(run, reps)
        rec = {"m": m, "q": q, "max_err": emax, "seconds": sec, "mode": mode}
        sweep.append(rec)
        print(f"[bench] accuracy sweep m={m} q={q}: max err {emax:.2e}, {sec*1e3:.2f} ms, {mode}",
              file=sys.stderr, flush=True)
        if rs_best is None or emax < rs_best["max_err"]:
            rs_best = dict(rec)
        if emax <= tgt:
            rs_best = dict(rec)
            rs_best["reached"] = True
            break
    rs_best.setdefault("reached", False)

    # plain CG: find the first iterate within the target, then time that many iterations
    cg_max = cg_max or (6000 if n >= 1024 else 400)
    dz, its, used = r.cg(g, cg_max, rtol=0.0, record=True)
    dxi = r.apply_L(its).cpu().numpy()
    errs = np.linalg.norm(dxi - dxs[:, None], axis=0) / np.linalg.norm(dxs)
    hit = np.nonzero(errs <= tgt)[0]
    nstar = int(hit[0]) + 1 if hit.size else used
    cg = {"iters": nstar, "err": float(errs[nstar - 1]), "reached": bool(hit.size),
          "best_err": float(errs.min()), "best_iter": int(np.argmin(errs)) + 1}

    def run_cg(nstar=nstar):
        r.linearize(xb, want_cost=False, out=(d, g))
        r.cg(g, nstar, rtol=0.0, record=False)
    cg["seconds"] = timed(run_cg, max(2, reps // 2))
    del its, dxi
    out = {"target": target, "target_used": tgt, "reference_floor": floor,
           "floor_method": "certified: Dot2-refined exact solve of eq. 3 with a rigorous bound "
                           f"({float(prob['floor_la']):.1e}) plus the FP64-vs-longdouble "
                           f"Hessian-product discrepancy on dz* ({float(prob['floor_op']):.1e})",
           "error": "||dx - dx*|| / ||dx*|| against the oracle's exact minimiser",
           "workload": f"Lorenz-96 n={n}, T={T}, {int(prob['obs_step'].size)} obs",
           "rsvd": rs_best, "cg": cg, "rsvd_sweep": sweep}
    if rs_best["reached"] and cg["reached"]:
        out["speedup_rsvd_over_cg"] = cg["seconds"] / rs_best["seconds"]
    return out


def small_inner_loop(seed: int, dev) -> dict:
    """Time to 1e-6 at the small Lorenz-96 configuration (n = 40, T = 40, 200 observations,
    RSVD m = 30 with one power step as the reference setting), RSVD against plain GPU CG."""
    from paper_1906_01413_amd import Riot
    import torch

    prob = load_problem("l96_n40", seed)
    r = Riot(int(prob["n"]), int(prob["nsteps"]), float(prob["dt"]), float(prob["forcing"]),
             prob["obs_step"], prob["obs_idx"], prob["y"], prob["rinv"], prob["taps"], m_max=40)
    xb = torch.tensor(prob["xb"], device=dev)
    return time_to_accuracy(r, prob, xb, dev, reps=20)


def fp32_leg(prob, k, p_os, q, steps, warmup, dev, lam64, V64, g64) -> dict:
    """The FP32 TL/AD variant on the benchmarked workload: the same inner-loop step, the
    TL/AD launch alone, and the increment against the FP64 path's on the same Philox probes
    and against the stored exact minimiser."""
    import torch
    from paper_1906_01413_amd import Riot, empty_colmajor

    n, T = int(prob["n"]), int(prob["nsteps"])
    m = k + p_os
    nobs = int(prob["obs_step"].size)
    r = Riot(n, T, float(prob["dt"]), float(prob["forcing"]), prob["obs_step"], prob["obs_idx"],
             prob["y"], prob["rinv"], prob["taps"], m_max=m, prec=1)
    xb = torch.tensor(prob["xb"], device=dev)
    d = torch.empty(max(nobs, 1), dtype=torch.float64, device=dev)
    g = torch.empty(n, dtype=torch.float64, device=dev)
    lam = torch.empty(m, dtype=torch.float64, device=dev)
    V = empty_colmajor(n, m, dev)
    dz = torch.empty(n, dtype=torch.float64, device=dev)
    dx = torch.empty(n, dtype=torch.float64, device=dev)

    def step(i):
        r.linearize(xb, want_cost=False, out=(d, g), defer_gradient=True)
        r.rsvd(k, p_os, q=q, Omega=None, seed=1000 + i, want_info=False, lam=lam, V=V)
        r.increment(lam, V, g, k=m, want_host=False, dz=dz, dx=dx)

    for i in range(warmup):
        step(i)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(steps):
        step(i)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_step = e0.elapsed_time(e1) / steps
    X = empty_colmajor(n, m, dev)
    X.copy_(torch.randn(n, m, dtype=torch.float64, device=dev))
    Yo = empty_colmajor(n, m, dev)
    for _ in range(3):
        r.gn_apply(X, out=Yo)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(10):
        r.gn_apply(X, out=Yo)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_tlad = e0.elapsed_time(e1) / 10
    # accuracy on the same probes as an FP64 handle's RSVD (seed 4242)
    from paper_1906_01413_amd import Riot as _R
    r64 = _R(n, T, float(prob["dt"]), float(prob["forcing"]), prob["obs_step"], prob["obs_idx"],
             prob["y"], prob["rinv"], prob["taps"], m_max=m)
    _, g_64, _ = r64.linearize(xb)
    l64, V_64, _ = r64.rsvd(k, p_os, q=q, seed=4242, want_info=False)
    _, dx64, _, _ = r64.increment(l64, V_64, g_64)
    r.linearize(xb, want_cost=False, out=(d, g))
    r.rsvd(k, p_os, q=q, seed=4242, want_info=False, lam=lam, V=V)
    _, dx32, _, mode = r.increment(lam, V, g)
    a, b = dx32.cpu().numpy(), dx64.cpu().numpy()
    dxs = np.asarray(prob["dx"])
    return {"workload": "the benchmarked workload with RIOT_FP32_TLAD",
            "ms_per_step": ms_step, "hvp_per_s": m * (1 + q) / (ms_step / 1e3),
            "tlad_ms_per_launch": ms_tlad,
            "tlad_tflops": tlad_flops_per_column(n, T, nobs) * m / (ms_tlad / 1e3) / 1e12,
            "increment_err_vs_fp64_rsvd": float(np.linalg.norm(a - b) / np.linalg.norm(b)),
            "increment_err_vs_exact": float(np.linalg.norm(a - dxs) / np.linalg.norm(dxs)),
            "fp64_increment_err_vs_exact": float(np.linalg.norm(b - dxs) / np.linalg.norm(dxs)),
            "mode": mode}


def batch_leg(nprob: int, seed: int, dev, reps: int = 5) -> dict:
    """Many uneven problems at once: inputs built with the library, then autotune, one
    instrumented probe-product launch (load balance), eager runs and graph replays."""
    import torch
    from paper_1906_01413_amd import RiotBatch, gaussian_taps
    from synthetic import batch_workloads

    t_setup = time.perf_counter()
    bw = batch_workloads(nprob, seed)
    taps = gaussian_taps(2.0, 1.0)
    specs = []
    for w, dr in bw:
        specs.append(dict(n=w.n, nsteps=w.nsteps, dt=w.dt, forcing=w.forcing, obs_step=dr["obs_step"],
                          obs_idx=dr["obs_idx"], y=np.zeros(dr["obs_step"].size), rinv=dr["rinv"],
                          taps=taps, m=w.m))
    # twin experiment through the library: truth spin-up by riot_forecast, truth
    # observations from the innovation at the truth with y = 0 (d = -H(x)), background
    # truth + L xi by riot_apply_L
    b0 = RiotBatch(specs, device=dev)
    truth, xb = [], []
    with torch.cuda.stream(b0.stream):
        for j, (w, dr) in enumerate(bw):
            r = b0.problem(j)
            t0 = r.forecast(torch.tensor(dr["x0"], device=dev), w.spinup)
            truth.append(t0)
            xb.append(t0 + r.apply_L(torch.tensor(dr["bg_noise"], device=dev)))
        for j in range(nprob):
            b0.vec(j, b0.x).copy_(truth[j])
    b0.run(seed)
    torch.cuda.synchronize()
    dpack = b0.d.cpu().numpy()
    for j, (w, dr) in enumerate(bw):
        o0 = int(b0.off_obs[j])
        specs[j]["y"] = -dpack[o0: o0 + dr["obs_step"].size] + dr["obs_noise"]
    del b0
    torch.cuda.empty_cache()
    b = RiotBatch(specs, device=dev)
    with torch.cuda.stream(b.stream):
        for j in range(nprob):
            b.vec(j, b.x).copy_(xb[j])
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t_setup
    wg, wave, ms_tuned = b.autotune()
    ms_prof, busy, ntiles = b.profile()
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731

    def timed(fn, n):
        fn()
        torch.cuda.synchronize()
        a, c = ev(), ev()
        a.record(b.stream)
        for _ in range(n):
            fn()
        c.record(b.stream)
        torch.cuda.synchronize()
        return a.elapsed_time(c) / n

    ms_eager = timed(lambda: b.run(seed), reps)
    b.capture(seed)
    ms_graph = timed(b.replay, reps)
    sum_m = int(sum(b.m))
    flops = sum(mj * tlad_flops_per_column(nj, tj, ob)
                for mj, nj, tj, ob in zip(b.m, b.n, b.nsteps, b.nobs))
    ach = flops / (ms_tuned / 1e3) / 1e12
    return {
        "workload": f"{nprob} independent Lorenz-96 inner loops, n in 40..2048, T in 20..200, "
                    f"25-50% of variables observed every 4 steps, m = min(n/2,128)+8",
        "problems": nprob, "sum_m": sum_m, "sum_n": int(sum(b.n)),
        "pipeline_ms_graph": ms_graph, "pipeline_ms_eager": ms_eager,
        "hvp_per_s": sum_m / (ms_graph / 1e3),
        "hvp_launch_ms": ms_tuned,
        "hvp_launch_hvp_per_s": sum_m / (ms_tuned / 1e3),
        "tlad_tflops": ach, "tlad_frac_fp64_peak": ach / PEAK_FP64_VALU_TFLOPS,
        "load_balance": busy, "tiles": ntiles, "profiled_launch_ms": ms_prof,
        "layout": {"workgroups": wg, "member_per_wave_max_threads": wave},
        "setup_s": setup_s,
    }


def tracer_leg(seed: int, dev, m: int = 512, reps: int = 3) -> dict:
    """Source inversion at 512 x 512 cells, 96 steps, 65536 controls, 4000 observations:
    inputs built with the library (twin experiment: s_true = L xi, y from the forward
    model, R sigma = 10 %), then m Hessian-probe products, the RSVD through the sketch
    handle and the increment, timed with HIP events."""
    import torch
    from paper_1906_01413_amd import Sketch, Tracer, exp_corr_sqrt
    from synthetic import advdiff_draws

    t_setup = time.perf_counter()
    dr = advdiff_draws("ad2_n512", seed)
    gp = dr["grid"]
    L1 = exp_corr_sqrt(gp["N"] // gp["block"], dr["ell"])
    nobs = dr["obs_t"].size
    ones = np.ones(nobs)
    t0 = Tracer(gp, dr["E"], dr["obs_t"], dr["obs_y"], dr["obs_x"], ones, ones, L1, dr["sigma"], 1,
                device=dev)
    s_true = t0.apply_L(torch.tensor(dr["xi"], device=dev))[:, 0]
    y_true = t0.forward(s_true).cpu().numpy()
    del t0
    sig = dr["rel_err"] * y_true
    y = y_true + sig * dr["obs_noise"]
    tr = Tracer(gp, dr["E"], dr["obs_t"], dr["obs_y"], dr["obs_x"], y, 1.0 / (sig * sig), L1,
                dr["sigma"], m, device=dev)
    nc = tr.ncontrol
    tr.forward(torch.zeros(nc, dtype=torch.float64, device=dev))
    g, _, J = tr.gradient()
    gen = torch.Generator(device=dev).manual_seed(seed)
    Om = torch.randn(m, nc, dtype=torch.float64, device=dev, generator=gen).t()
    Y = torch.empty(m, nc, dtype=torch.float64, device=dev).t()
    sk = Sketch(nc, m, device=dev)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t_setup
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731

    def timed(fn, n):
        fn()
        torch.cuda.synchronize()
        a, b = ev(), ev()
        a.record()
        for _ in range(n):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / n

    ms_hvp = timed(lambda: tr.hess_apply(Om, out=Y), reps)
    res = {}

    def inner():
        tr.hess_apply(Om, out=Y)
        lam, V, _ = sk.eig(Om, Y, want_info=False)
        res["lv"] = (lam, V)

    ms_inner = timed(inner, reps)
    lam, V = res["lv"]
    dz, dofs, mode = sk.increment(lam, V, g)
    N, T = gp["N"], gp["T"]
    # bytes one probe must move per step when the sweeps run two steps per launch: the
    # field read and written once per two steps in the TL and in the AD sweep
    byts = 16.0 * N * N * T * m
    bw = byts / (ms_hvp / 1e3) / 1e9
    return {
        "workload": f"tracer source inversion: {N}x{N} periodic grid, {T} steps, {nc} controls, "
                    f"{nobs} track observations, {m} probes",
        "probes": m, "hvp_ms": ms_hvp, "hvp_per_s": m / (ms_hvp / 1e3),
        "inner_loop_ms": ms_inner, "dofs": dofs, "mode": mode, "cost_J": J,
        "roofline": {"bound": "hbm", "achieved": bw, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": bw / PEAK_HBM_GBS,
                     "algorithmic_bytes": byts,
                     "note": "16 N^2 bytes per probe and step: one field read and written per "
                             "two steps in the tangent and in the adjoint sweep",
                     "one_step_equivalent_GBs": 2.0 * bw},
        "setup_s": setup_s,
    }


def proposal_leg(seed: int) -> dict:
    """Cycled Lorenz-96 n = 2048 (window 50 steps, 10240 observations per window): training
    data from cycles 1-100, GPU training of the proposal network, cycles 101-200 judged
    learned (64 + 16 probes) against Gaussian 80 and Gaussian 128."""
    from paper_1906_01413_amd import proposal
    from synthetic import CYCLED, cycled_draws, net_init, workload

    cfg = dict(CYCLED)
    w = workload(cfg["workload"])
    s = proposal.run_experiment(w, cycled_draws(seed, cfg["cycles"]), cfg,
                                net_init(seed + 3, proposal.net_shapes(cfg)), seed=seed)
    # FP32 rate of the network's forward pass (the convolutions of the proposal's inference)
    import torch
    from paper_1906_01413_amd import ProposalNet
    nb = 16
    net = ProposalNet(w.n, k=cfg["k_net"], channels=cfg["channels"], layers=cfg["layers"],
                      width=cfg["width"], batch_max=nb, segments=cfg["segments"],
                      in_channels=cfg["snapshots"])
    xin = torch.randn(nb, cfg["snapshots"], w.n, dtype=torch.float64, device="cuda")
    for _ in range(3):
        net.forward(xin)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(20):
        net.forward(xin)
    e1.record()
    torch.cuda.synchronize()
    fwd_ms = e0.elapsed_time(e1) / 20
    fwd_flops = nb * sum(2.0 * w.n * ci * co * wd for co, ci, wd in net.layer_shapes())
    s["net_forward"] = {"batch": nb, "ms": fwd_ms, "tflops": fwd_flops / fwd_ms / 1e9,
                        "frac_fp32_vector_peak": fwd_flops / fwd_ms / 1e9 / 157.3,
                        "flops": fwd_flops}
    s["workload"] = (f"cycled Lorenz-96 n={w.n}, window {w.nsteps} steps, "
                     f"{cfg['train_cycles']} training + {cfg['cycles'] - cfg['train_cycles']} test cycles; "
                     f"net {cfg['layers']}x{cfg['channels']} conv1d width {cfg['width']}, "
                     f"{cfg['snapshots']} input fields, {cfg['segments']}-segment head, "
                     f"k={cfg['k_net']} + {cfg['p_gauss']} Gaussian vs Gaussian "
                     f"{cfg['k_net'] + cfg['p_gauss']} and {cfg['m_ref']}")
    return s


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="l96_n4096", choices=sorted(WORKLOADS))
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--prec", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-accuracy", action="store_true", help="skip the time-to-accuracy sweep")
    ap.add_argument("--hvp-reps", type=int, default=20)
    ap.add_argument("--fp32", type=int, default=1,
                    help="also run the FP32 TL/AD variant on the same workload (0 skips it)")
    ap.add_argument("--batch", type=int, default=1000,
                    help="problems in the batched-uneven leg (0 skips it)")
    ap.add_argument("--tracer", type=int, default=1,
                    help="run the tracer source-inversion leg (0 skips it)")
    ap.add_argument("--proposal", type=int, default=1,
                    help="run the cycled learned-proposal leg (0 skips it)")
    ap.add_argument("--counter-pass", action="store_true",
                    help="only launch the TL/AD kernel three times and a 256 MiB device copy "
                         "(calibration), for rocprofv3 --pmc runs; prints no JSON")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU sharding is a design note, not a measured path", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1906_01413_amd import Riot, empty_colmajor

    k, p_os, q = WORKLOADS[args.workload]
    m = k + p_os
    prob = load_problem(args.workload, args.seed)
    n, T = int(prob["n"]), int(prob["nsteps"])
    nobs = int(prob["obs_step"].size)
    w = int(prob["taps"].size - 1)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    prec = 1 if args.prec == "fp32" else 0
    r = Riot(n, T, float(prob["dt"]), float(prob["forcing"]), prob["obs_step"], prob["obs_idx"],
             prob["y"], prob["rinv"], prob["taps"], m_max=max(m, 1088 if n >= 1088 else m),
             prec=prec)
    xb = torch.tensor(prob["xb"], device=dev)
    d = torch.empty(max(nobs, 1), dtype=torch.float64, device=dev)
    g = torch.empty(n, dtype=torch.float64, device=dev)
    lam = torch.empty(m, dtype=torch.float64, device=dev)
    V = empty_colmajor(n, m, dev)
    dz = torch.empty(n, dtype=torch.float64, device=dev)
    dx = torch.empty(n, dtype=torch.float64, device=dev)
    Wc = empty_colmajor(n, m, dev)
    coef = torch.empty(m, dtype=torch.float64, device=dev)
    diag = torch.empty(n, dtype=torch.float64, device=dev)

    if args.counter_pass:
        Xin = empty_colmajor(n, m, dev)
        Xin.copy_(torch.randn(n, m, dtype=torch.float64, device=dev))
        Yout = empty_colmajor(n, m, dev)
        r.linearize(xb, want_cost=False, out=(d, g))
        for _ in range(3):
            r.gn_apply(Xin, out=Yout)
        a = torch.empty(32 * 1024 * 1024, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        a.fill_(1.0)
        b.copy_(a)
        torch.cuda.synchronize()
        print("[bench] counter pass done: 3 TL/AD launches, one 256 MiB copy", file=sys.stderr)
        return

    def step(i):
        # the gradient's adjoint sweep runs on the handle's second stream beside the RSVD,
        # which needs only the trajectory; the increment waits for it
        r.linearize(xb, want_cost=False, out=(d, g), defer_gradient=True)
        r.rsvd(k, p_os, q=q, Omega=None, seed=1000 + i, want_info=False, lam=lam, V=V)
        r.increment(lam, V, g, k=m, want_host=False, dz=dz, dx=dx)
        r.posterior_cov(lam, V, k=m, want_host=False, out=(Wc, coef, diag))

    print(f"[bench] workload {args.workload} n={n} T={T} m={m} q={q} prec={args.prec}: warmup",
          file=sys.stderr, flush=True)
    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    t0 = time.perf_counter()
    evs[0].record(stream)
    for i in range(args.steps):
        step(args.warmup + i)
        evs[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = evs[0].elapsed_time(evs[-1]) / args.steps
    per_step = np.array([evs[i].elapsed_time(evs[i + 1]) for i in range(args.steps)])
    hvps_per_step = m * (1 + q)
    value = hvps_per_step / (ms_step / 1e3)
    print(f"[bench] timed {args.steps} steps: {ms_step:.3f} ms/step (wall {wall:.3f} s)",
          file=sys.stderr, flush=True)

    # dominant kernel: the batched TL/AD sweep alone (riot_gn_apply is exactly one launch)
    Xin = empty_colmajor(n, m, dev)
    Xin.copy_(torch.randn(n, m, dtype=torch.float64, device=dev))
    Yout = empty_colmajor(n, m, dev)
    for _ in range(3):
        r.gn_apply(Xin, out=Yout)
    torch.cuda.synchronize()
    h0, h1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    h0.record(stream)
    for _ in range(args.hvp_reps):
        r.gn_apply(Xin, out=Yout)
    h1.record(stream)
    torch.cuda.synchronize()
    ms_tlad = h0.elapsed_time(h1) / args.hvp_reps
    flops = tlad_flops_per_column(n, T, nobs) * m
    achieved = flops / (ms_tlad / 1e3) / 1e12
    # full Hessian-probe product (L, TL/AD, L^T) for the HVP-only rate
    a0, a1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a0.record(stream)
    for _ in range(args.hvp_reps):
        r.hess_apply(Xin, out=Yout)
    a1.record(stream)
    torch.cuda.synchronize()
    ms_hvp = a0.elapsed_time(a1) / args.hvp_reps
    print(f"[bench] TL/AD kernel {ms_tlad:.3f} ms per {m}-column launch, "
          f"{achieved:.2f} TFLOP/s; Hessian-probe block {ms_hvp:.3f} ms", file=sys.stderr, flush=True)

    out = {
        "metric": "Hess-vec products/s; inner-loop s to 1e-6 rel. increment err, RSVD vs CG",
        "value": value,
        "unit": "HVP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "ms_per_step_median": float(np.median(per_step)),
        "ms_per_step_p90": float(np.percentile(per_step, 90)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == 0 else "f32 TL/AD, f64 linear algebra",
        "data": "synthetic (seeded Lorenz-96 twin experiment built by the CPU oracle)",
        "config": {"workload": f"Lorenz-96 n={n}, T={T} RK4 steps dt={float(prob['dt'])}, "
                               f"{nobs} obs, RSVD m={m} (k={k}+{p_os}), q={q}",
                   "n": n, "nsteps": T, "nobs": nobs, "m": m, "q": q, "seed": args.seed},
        "hvp_only": {"value": m / (ms_hvp / 1e3), "unit": "HVP/s",
                     "ms_per_block": ms_hvp, "flops_per_hvp": hvp_flops(n, T, nobs, w)},
        "roofline": {"bound": "alu", "kernel": "tlad_kernel (batched TL+AD sweep)",
                     "achieved": achieved, "peak": PEAK_FP64_VALU_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_VALU_TFLOPS,
                     "traffic": tlad_traffic_bytes(n, T, m),
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                                     "copy-calibrated)",
                     # probes in, products out, the four RK4 stage states of every step once
                     "algorithmic_bytes": 16.0 * n * m + 32.0 * n * (T + 1),
                     "ms_per_launch": ms_tlad, "flops_per_launch": flops},
    }

    if not args.no_accuracy:
        out["inner_loop"] = time_to_accuracy(r, prob, xb, dev)
        il = out["inner_loop"]
        print(f"[bench] inner loop n={n}: target {il['target_used']:.1e} (floor "
              f"{il['reference_floor']:.1e}); RSVD m={il['rsvd']['m']} q={il['rsvd']['q']} "
              f"err {il['rsvd']['max_err']:.2e} in {il['rsvd']['seconds']*1e3:.1f} ms; CG "
              f"{il['cg']['iters']} it. err {il['cg']['err']:.2e} in {il['cg']['seconds']*1e3:.1f} ms",
              file=sys.stderr, flush=True)
        if args.workload != "l96_n40":
            out["inner_loop_n40"] = small_inner_loop(args.seed, dev)
            il = out["inner_loop_n40"]
            print(f"[bench] inner loop n=40: RSVD m={il['rsvd']['m']} q={il['rsvd']['q']} err "
                  f"{il['rsvd']['max_err']:.2e} in {il['rsvd']['seconds']*1e3:.2f} ms; CG "
                  f"{il['cg']['iters']} it. err {il['cg']['err']:.2e} in "
                  f"{il['cg']['seconds']*1e3:.2f} ms", file=sys.stderr, flush=True)

    if args.fp32 and prec == 0:
        out["fp32_tlad"] = fp32_leg(prob, k, p_os, q, args.steps, args.warmup, dev, lam, V, g)
        fl = out["fp32_tlad"]
        print(f"[bench] FP32 TL/AD: {fl['ms_per_step']:.3f} ms/step, TL/AD launch "
              f"{fl['tlad_ms_per_launch']:.3f} ms; increment vs FP64 RSVD on the same probes "
              f"{fl['increment_err_vs_fp64_rsvd']:.2e}", file=sys.stderr, flush=True)

    if args.batch > 0:
        print(f"[bench] batched leg: {args.batch} problems", file=sys.stderr, flush=True)
        out["batch"] = batch_leg(args.batch, args.seed, dev)
        bl = out["batch"]
        print(f"[bench] batch: pipeline {bl['pipeline_ms_graph']:.2f} ms (graph), "
              f"{bl['pipeline_ms_eager']:.2f} ms (eager); probe products {bl['hvp_launch_ms']:.2f} ms, "
              f"load balance {bl['load_balance']:.3f}, layout {bl['layout']}", file=sys.stderr, flush=True)

    if args.tracer:
        print("[bench] tracer source-inversion leg", file=sys.stderr, flush=True)
        out["tracer"] = tracer_leg(args.seed, dev)
        tl = out["tracer"]
        print(f"[bench] tracer: {tl['probes']} probe products {tl['hvp_ms']:.1f} ms "
              f"({tl['roofline']['achieved']:.0f} GB/s), inner loop {tl['inner_loop_ms']:.1f} ms",
              file=sys.stderr, flush=True)

    if args.proposal:
        print("[bench] cycled learned-proposal leg", file=sys.stderr, flush=True)
        out["proposal"] = proposal_leg(args.seed)
        pl = out["proposal"]
        print(f"[bench] proposal: train {pl['train_ms_per_step']:.2f} ms/step, columns capture "
              f"{pl['net_columns_capture_mean']:.3f} (random {pl['random_columns_capture']:.3f}), "
              f"rho learned/gauss {pl['rho_ratio_learned_over_gauss_m_median']:.3f}, "
              f"fallbacks {pl['fallbacks']}/{pl['cycles']}", file=sys.stderr, flush=True)

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(prob, m)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
