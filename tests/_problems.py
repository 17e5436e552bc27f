"""Shared test fixtures: oracle-built problems and their GPU handles."""

from __future__ import annotations

import numpy as np

from oracle import bcov, fourdvar
from synthetic import l96_draws, probe_block, workload


def oracle_problem(name="l96_n40", seed=0, **over):
    w = workload(name, **over)
    p, truth = fourdvar.realize_l96(w, l96_draws(w, seed))
    return w, p


def riot_for(p, m_max, prec=0, elems_per_lane=0):
    from paper_1906_01413_amd import Riot
    return Riot(p.n, p.nsteps, p.h, p.F, p.obs_step, p.obs_idx, p.y, p.rinv, p.taps, m_max,
                prec=prec, elems_per_lane=elems_per_lane)


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def to_np(t):
    return t.detach().cpu().numpy()
