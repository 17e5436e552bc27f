"""The C-ABI library loads and exports every symbol declared in include/riot.h (no GPU needed)."""

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "riot.h")).read()
    return sorted(set(re.findall(r"\b(riot_[a-zA-Z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("riot_init", "riot_hess_apply", "riot_rsvd", "riot_increment", "riot_posterior_cov"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1906_01413_amd.riot import EXPORTS, load_library
    lib = load_library()
    names = _declared()
    for nm in names:
        assert hasattr(lib, nm), nm
    assert set(EXPORTS) == set(names)


def _desc(**over):
    from paper_1906_01413_amd.riot import _Desc
    taps = np.array([0.6, 0.3, 0.1])
    obs_step = np.array([1, 2], dtype=np.int32)
    obs_idx = np.array([0, 5], dtype=np.int32)
    y = np.array([1.0, 2.0])
    rinv = np.array([1.0, 1.0])
    d = _Desc()
    d.n, d.nsteps, d.dt, d.forcing, d.nobs = 40, 4, 0.05, 8.0, 2
    P = lambda a, c: a.ctypes.data_as(ctypes.POINTER(c))  # noqa: E731
    d.obs_step, d.obs_idx = P(obs_step, ctypes.c_int32), P(obs_idx, ctypes.c_int32)
    d.y, d.rinv = P(y, ctypes.c_double), P(rinv, ctypes.c_double)
    d.l_halfwidth, d.l_taps = 2, P(taps, ctypes.c_double)
    d.m_max, d.prec, d.elems_per_lane = 8, 0, 0
    for k, v in over.items():
        setattr(d, k, v)
    return d, (taps, obs_step, obs_idx, y, rinv)


def test_workspace_bytes_validates_descriptor():
    from paper_1906_01413_amd.riot import load_library
    lib = load_library()
    d, keep = _desc()
    assert lib.riot_workspace_bytes(ctypes.byref(d)) > 0
    for bad in ({"n": 3}, {"m_max": 0}, {"dt": -1.0}, {"prec": 7}, {"elems_per_lane": 3},
                {"nsteps": -1}, {"m_max": 5000}):
        d2, keep2 = _desc(**bad)
        assert lib.riot_workspace_bytes(ctypes.byref(d2)) == 0, bad
    # observation outside the window is rejected
    d3, keep3 = _desc()
    keep3[1][1] = 9
    assert lib.riot_workspace_bytes(ctypes.byref(d3)) == 0
    # non-positive R^{-1} is rejected
    d4, keep4 = _desc()
    keep4[4][0] = 0.0
    assert lib.riot_workspace_bytes(ctypes.byref(d4)) == 0
    assert lib.riot_workspace_bytes(None) == 0


def test_status_strings_and_null_handles():
    from paper_1906_01413_amd.riot import load_library
    lib = load_library()
    assert lib.riot_status_str(0) == b"RIOT_OK"
    assert lib.riot_status_str(-3).startswith(b"RIOT_E_NOT_SPD")
    # every entry point rejects a NULL handle before touching the GPU
    vp = ctypes.c_void_p
    assert lib.riot_hess_apply(None, 1, vp(8), vp(16), 0) == -1
    assert lib.riot_rsvd(None, 1, 0, 0, None, 0, vp(8), vp(16), None) == -1
    assert lib.riot_linearize(None, vp(8), None, vp(8), vp(8), None) == -1
    assert lib.riot_increment(None, 1, vp(8), vp(8), vp(8), 0, vp(8), vp(8), None, None) == -1
    assert lib.riot_posterior_cov(None, 1, vp(8), vp(8), 0, vp(8), vp(8), None, None, None) == -1
    assert lib.riot_cg(None, vp(8), 1, 0.0, vp(8), None, None) == -1
    out = vp()
    assert lib.riot_init(None, vp(256), 1024, None, ctypes.byref(out)) == -1
    lib.riot_free(None)


def test_gaussian_taps_host_helper_matches_oracle():
    """riot_gaussian_taps (host code, no GPU) against the oracle's square-root taps."""
    import numpy as np

    from oracle.bcov import gaussian_taps as oracle_taps
    from paper_1906_01413_amd import gaussian_taps

    for ell, sb in ((2.0, 1.0), (8.0, 1.0), (1.5, 0.7)):
        a, b = gaussian_taps(ell, sb), oracle_taps(ell, sb)
        assert a.size == b.size
        assert np.max(np.abs(a - b)) <= 1e-15 * np.max(np.abs(b))


def test_exp_corr_sqrt_host_helper_matches_oracle():
    """riot_exp_corr_sqrt (circulant cosine spectrum, host code) against the oracle's
    eigendecomposition-based square root."""
    import numpy as np

    from oracle.advdiff import sqrt_corr_1d
    from paper_1906_01413_amd import exp_corr_sqrt

    for n, ell in ((16, 3.0), (128, 3.0), (37, 1.5)):
        a, b = exp_corr_sqrt(n, ell), sqrt_corr_1d(n, ell)
        assert np.max(np.abs(a - b)) < 1e-12, (n, ell)


def test_noalloc_entry_point_refuses_sizes_beyond_its_scratch():
    """riot_sketch_eig_noalloc checks arguments and the size of its static scratch on the host
    and returns before any HIP call, so these cases need no GPU."""
    from paper_1906_01413_amd.riot import load_library
    lib = load_library()
    vp = ctypes.c_void_p
    assert lib.riot_sketch_noalloc_max_bytes() == 32 << 20
    args = (vp(256), vp(512), vp(768), vp(1024), None, None)
    assert lib.riot_sketch_eig_noalloc(4096, 400, *args) == -9       # RIOT_E_SCRATCH
    assert lib.riot_sketch_eig_noalloc(65536, 512, *args) == -9
    assert lib.riot_sketch_eig_noalloc(40, 41, *args) == -1          # m > n
    assert lib.riot_sketch_eig_noalloc(40, 0, *args) == -1
    assert lib.riot_sketch_eig_noalloc(40, 30, None, *args[1:]) == -1
    assert lib.riot_status_str(-9).startswith(b"RIOT_E_SCRATCH")
    # the largest m that fits at the benchmarked n, as the header states
    fits = [m for m in range(256, 400) if lib.riot_sketch_workspace_bytes(4096, m) <= 32 << 20]
    assert max(fits) == 316
