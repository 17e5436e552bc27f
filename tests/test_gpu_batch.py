"""Batches of independent, unevenly sized problems (C ABI riot_batch_*).

Problems come from the seeded batch recipe (n from 40 to 2048, windows of 20-200 steps,
25-50 % of the variables observed every 4th step) and are built by the FP64 oracle. The
batch runs every problem's first inner loop at once: batched trajectories and gradients,
one persistent TL/AD launch over all (problem, probe) tiles, batched CholeskyQR, K,
eigen-solve and increment. Checked here:
  * gradients against the oracle;
  * Ritz values and increments against the oracle's RSVD on the same Philox probes
    (problem j draws stream j of the run's seed);
  * every problem against its own single-problem handle (same probes);
  * member-per-workgroup and member-per-wave layouts give the same results bit for bit
    (gradients, Ritz values and increments);
  * a captured HIP graph, replayed several times with other work in between, reproduces
    the eager run bit for bit.
"""

import numpy as np
import pytest

from oracle import fourdvar, philox
from synthetic import batch_workloads
from tests._problems import rel

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SEED = 4321
NPROB = 12


@pytest.fixture(scope="module")
def batch():
    from paper_1906_01413_amd import RiotBatch

    probs = [fourdvar.realize_l96(w, d)[0] for w, d in batch_workloads(NPROB, 3)]
    ms = [min(p.n // 2, 128) + 8 for p in probs]
    specs = [dict(n=p.n, nsteps=p.nsteps, dt=p.h, forcing=p.F, obs_step=p.obs_step,
                  obs_idx=p.obs_idx, y=p.y, rinv=p.rinv, taps=p.taps, m=m)
             for p, m in zip(probs, ms)]
    b = RiotBatch(specs)
    b.set_x([p.xb for p in probs])
    b.run(SEED)
    torch.cuda.synchronize()
    print("batch sizes n:", [p.n for p in probs], "T:", [p.nsteps for p in probs])
    return b, probs, ms


def _snapshot(b):
    torch.cuda.synchronize()
    return {k: getattr(b, k).detach().cpu().numpy().copy() for k in ("grad", "lam", "dx", "dz")}


def _same_run(got, ref, b):
    """Gradients, Ritz values and increments bit for bit: every reduction on the path sums
    in a fixed order (the work-queue counters only hand out tiles), so neither the layout
    nor a graph replay may change a single bit. Returns the first array that differs."""
    for k in ("grad", "lam", "dx", "dz"):
        if not np.array_equal(got[k], ref[k]):
            return k
    return None


def _gradient_floor(p, lin):
    """Relative change of the oracle's gradient when x moves by one ulp (random signs).

    Windows of up to 200 steps span about ten e-folding times of the model's leading
    Lyapunov mode, so two correct FP64 codes rounding differently agree only to about
    this; the bound is the tolerance's measured floor, not a fitted number.
    """
    rng = np.random.default_rng(1)
    xp = p.xb * (1.0 + 2.0 ** -52 * rng.choice([-1.0, 1.0], size=p.n))
    return rel(fourdvar.linearize(p, xp).g, lin.g)


def test_batch_gradients_match_oracle(batch):
    b, probs, ms = batch
    bad = []
    for j, p in enumerate(probs):
        lin = fourdvar.linearize(p, p.xb)
        g = b.vec(j, b.grad).cpu().numpy()
        e = rel(g, lin.g)
        floor = _gradient_floor(p, lin)
        tol = max(1e-10, 10.0 * floor)
        print(f"problem {j} (n={p.n}, T={p.nsteps}): gradient rel err {e:.2e}, "
              f"one-ulp floor {floor:.2e}")
        if not e < tol:
            bad.append((j, e, tol))
    assert not bad, bad


def test_batch_rsvd_matches_oracle_on_small_problems(batch):
    b, probs, ms = batch
    small = sorted(range(len(probs)), key=lambda j: probs[j].n * probs[j].nsteps * ms[j])[:3]
    for j in small:
        p, m = probs[j], ms[j]
        lin = fourdvar.linearize(p, p.xb)
        Om = philox.normal_columns(p.n, np.arange(m), seed=SEED, stream=j)
        ro = fourdvar.rsvd(lambda X: fourdvar.hvp(p, lin, X), Om, q=0)
        lam = b.lam_of(j).cpu().numpy()
        assert np.max(np.abs(lam - ro.lam)) <= 1e-9 * abs(ro.lam[0]), j
        _, dxo, _, modeo = fourdvar.increment(p, ro.lam, ro.V, lin.g)
        e = rel(b.vec(j, b.dx).cpu().numpy(), dxo)
        print(f"problem {j} (n={p.n}, T={p.nsteps}, m={m}): dx rel err {e:.2e}, {modeo}")
        assert e < 1e-8, (j, e)


def test_batch_matches_single_problem_handles(batch):
    b, probs, ms = batch
    for j, p in enumerate(probs):
        r = b.problem(j)
        with torch.cuda.stream(b.stream):
            Om = r.philox_normal(p.n, ms[j], seed=SEED, stream=j)
            lam, V, info = r.rsvd(ms[j] - 8, 8, q=0, Omega=Om)
        torch.cuda.synchronize()
        lb = b.lam_of(j).cpu().numpy()
        ls = lam.cpu().numpy()
        assert np.max(np.abs(lb - ls)) <= 1e-12 * abs(ls[0]), j
        assert info.orth_err < 1e-12


def test_batch_layouts_agree(batch):
    b, probs, ms = batch
    ref = _snapshot(b)
    for wg, wave in ((256, 0), (512, 64), (768, 64)):
        b.set_layout(wg, wave)
        b.run(SEED)
        bad = _same_run(_snapshot(b), ref, b)
        assert bad is None, (wg, wave, bad)
    wg, wave, ms_best = b.autotune()
    print(f"autotuned layout: {wg} workgroups, member-per-wave up to {wave} threads, {ms_best:.3f} ms")
    b.run(SEED)
    bad = _same_run(_snapshot(b), ref, b)
    assert bad is None, ("autotuned", bad)


def test_batch_graph_replays_reproduce_eager_run(batch):
    from paper_1906_01413_amd import RiotBatch  # noqa: F401

    b, probs, ms = batch
    b.run(SEED)
    ref = _snapshot(b)
    b.capture(SEED)
    for rep in range(3):
        b.replay()
        bad = _same_run(_snapshot(b), ref, b)
        assert bad is None, (rep, bad)
        # eager device work between replays
        x = torch.randn(1 << 20, device="cuda", dtype=torch.float64)
        (x * 2.0).sum().item()
