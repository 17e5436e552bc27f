"""Thin Python binding of the RIOT C ABI (include/riot.h).

Argument marshalling only: every step of the inner loop runs in the HIP
library libriot.so. PyTorch supplies device memory and the stream. Matrices
follow the C ABI's column-major convention: an n x m block is a float64 CUDA
tensor of shape (n, m) with strides (1, n) (``colmajor`` below builds one).
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libriot.so")

RIOT_OK = 0
STATUS = {0: "RIOT_OK", -1: "RIOT_E_ARG", -2: "RIOT_E_HIP", -3: "RIOT_E_NOT_SPD",
          -4: "RIOT_E_SINGULAR", -5: "RIOT_E_NONFINITE", -6: "RIOT_E_NOCONV",
          -7: "RIOT_E_STATE", -8: "RIOT_E_WORKSPACE", -9: "RIOT_E_SCRATCH"}
FP64, FP32_TLAD = 0, 1
ADAPTIVE, LRA, LRU = 0, 1, 2
MODES = {"adaptive": ADAPTIVE, "lra": LRA, "lru": LRU}

EXPORTS = ("riot_workspace_bytes", "riot_init", "riot_free", "riot_set_pass_sync", "riot_status_str",
           "riot_linearize", "riot_linearize_deferred", "riot_join", "riot_hess_apply",
           "riot_rsvd", "riot_increment", "riot_increment_select", "riot_psas_hess_apply",
           "riot_psas_rhs", "riot_psas_increment", "riot_precond_apply", "riot_precond_hess_apply",
           "riot_orth", "riot_project_out", "riot_outer_update", "riot_gradient_sample",
           "riot_block_lanczos",
           "riot_posterior_cov", "riot_cg", "riot_forecast", "riot_apply_L",
           "riot_philox_normal", "riot_tl_apply", "riot_ad_apply", "riot_gn_apply",
           "riot_batch_workspace_bytes", "riot_batch_init", "riot_batch_free", "riot_batch_buffers",
           "riot_batch_run", "riot_batch_set_layout", "riot_batch_autotune", "riot_batch_capture",
           "riot_batch_replay", "riot_batch_problem", "riot_batch_profile", "riot_gaussian_taps",
           "riot_ckpt_forward", "riot_ckpt_tangent", "riot_ckpt_adjoint",
           "riot_sketch_workspace_bytes", "riot_sketch_init", "riot_sketch_free", "riot_sketch_eig",
           "riot_sketch_increment", "riot_sketch_eig_noalloc", "riot_sketch_noalloc_max_bytes",
           "riot_tracer_workspace_bytes", "riot_tracer_init", "riot_tracer_free", "riot_tracer_forward",
           "riot_tracer_tangent", "riot_tracer_adjoint", "riot_tracer_apply_L", "riot_tracer_hess_apply",
           "riot_tracer_gradient", "riot_exp_corr_sqrt", "riot_set_obs", "riot_proj_residual",
           "riot_sketch_residual", "riot_net_workspace_bytes", "riot_net_init", "riot_net_free",
           "riot_net_param_count", "riot_net_set_params", "riot_net_get_params", "riot_net_forward",
           "riot_net_backward", "riot_net_adam", "riot_net_capture_loss", "riot_net_train_step")


class RiotError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {STATUS.get(status, status)}")
        self.status = status


class _Desc(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32), ("nsteps", ctypes.c_int32),
        ("dt", ctypes.c_double), ("forcing", ctypes.c_double),
        ("nobs", ctypes.c_int32),
        ("obs_step", ctypes.POINTER(ctypes.c_int32)), ("obs_idx", ctypes.POINTER(ctypes.c_int32)),
        ("y", ctypes.POINTER(ctypes.c_double)), ("rinv", ctypes.POINTER(ctypes.c_double)),
        ("l_halfwidth", ctypes.c_int32), ("l_taps", ctypes.POINTER(ctypes.c_double)),
        ("m_max", ctypes.c_int32), ("prec", ctypes.c_int32), ("elems_per_lane", ctypes.c_int32),
        ("ckpt_stride", ctypes.c_int32),
    ]


class _BatchIO(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("x", "grad", "lambda_", "V", "dz", "dx", "d")]


class _TracerDesc(ctypes.Structure):
    _fields_ = [
        ("N", ctypes.c_int32), ("nsteps", ctypes.c_int32),
        ("dt", ctypes.c_double), ("u0", ctypes.c_double), ("u1", ctypes.c_double),
        ("v", ctypes.c_double), ("K", ctypes.c_double),
        ("block", ctypes.c_int32), ("ntb", ctypes.c_int32),
        ("E", ctypes.POINTER(ctypes.c_double)), ("nobs", ctypes.c_int32),
        ("obs_t", ctypes.POINTER(ctypes.c_int32)), ("obs_y", ctypes.POINTER(ctypes.c_int32)),
        ("obs_x", ctypes.POINTER(ctypes.c_int32)),
        ("y", ctypes.POINTER(ctypes.c_double)), ("rinv", ctypes.POINTER(ctypes.c_double)),
        ("L1", ctypes.POINTER(ctypes.c_double)), ("sigma", ctypes.c_double),
        ("m_max", ctypes.c_int32),
    ]


class _NetDesc(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int32) for k in ("n", "layers", "channels", "k", "width", "batch_max",
                                              "segments", "in_channels")]


class _RsvdInfo(ctypes.Structure):
    _fields_ = [("chol_shifts", ctypes.c_int32), ("qr_passes", ctypes.c_int32),
                ("k_asym", ctypes.c_double), ("orth_err", ctypes.c_double),
                ("kappa_est", ctypes.c_double), ("resid_est", ctypes.c_double)]


_lib = None


def load_library(path: str | None = None) -> ctypes.CDLL:
    """Load libriot.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or _LIB_PATH
    if not os.path.exists(p):
        raise ImportError(f"libriot.so not found at {p}: build it with "
                          "`python paper_1906_01413_amd/build_lib.py` (no CPU fallback exists)")
    lib = ctypes.CDLL(p)
    vp, i32, u64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64, ctypes.c_double
    sig = {
        "riot_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(_Desc)]),
        "riot_init": (i32, [ctypes.POINTER(_Desc), vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]),
        "riot_free": (None, [vp]),
        "riot_set_pass_sync": (i32, [vp, i32]),
        "riot_status_str": (ctypes.c_char_p, [i32]),
        "riot_linearize": (i32, [vp, vp, vp, vp, vp, ctypes.POINTER(dbl)]),
        "riot_linearize_deferred": (i32, [vp, vp, vp, vp, vp, ctypes.POINTER(dbl)]),
        "riot_join": (i32, [vp]),
        "riot_hess_apply": (i32, [vp, i32, vp, vp, i32]),
        "riot_rsvd": (i32, [vp, i32, i32, i32, vp, u64, vp, vp, ctypes.POINTER(_RsvdInfo)]),
        "riot_increment": (i32, [vp, i32, vp, vp, vp, i32, vp, vp, ctypes.POINTER(dbl),
                                 ctypes.POINTER(i32)]),
        "riot_increment_select": (i32, [vp, i32, vp, vp, vp, vp, vp, vp, vp, ctypes.POINTER(dbl),
                                        ctypes.POINTER(i32)]),
        "riot_posterior_cov": (i32, [vp, i32, vp, vp, i32, vp, vp, vp, vp, ctypes.POINTER(i32)]),
        "riot_psas_hess_apply": (i32, [vp, i32, vp, vp]),
        "riot_precond_apply": (i32, [vp, i32, vp, vp, vp, i32, i32, vp]),
        "riot_precond_hess_apply": (i32, [vp, i32, vp, vp, vp, i32, vp, vp]),
        "riot_orth": (i32, [vp, i32, vp, vp]),
        "riot_gradient_sample": (i32, [vp, vp, vp, vp, vp, vp]),
        "riot_block_lanczos": (i32, [vp, i32, i32, vp, vp, vp, vp, vp, vp]),
        "riot_project_out": (i32, [vp, i32, vp, i32, vp]),
        "riot_outer_update": (i32, [vp, vp, vp, vp]),
        "riot_psas_rhs": (i32, [vp, vp, vp, vp]),
        "riot_psas_increment": (i32, [vp, i32, vp, vp, vp, i32, vp, vp, ctypes.POINTER(i32)]),
        "riot_cg": (i32, [vp, vp, i32, dbl, vp, vp, ctypes.POINTER(i32)]),
        "riot_forecast": (i32, [vp, vp, i32, vp]),
        "riot_apply_L": (i32, [vp, i32, vp, vp]),
        "riot_philox_normal": (i32, [vp, i32, i32, u64, u64, vp]),
        "riot_tl_apply": (i32, [vp, i32, vp, vp]),
        "riot_ad_apply": (i32, [vp, i32, vp, vp]),
        "riot_gn_apply": (i32, [vp, i32, vp, vp]),
        "riot_batch_workspace_bytes": (ctypes.c_size_t, [i32, ctypes.POINTER(_Desc)]),
        "riot_batch_init": (i32, [i32, ctypes.POINTER(_Desc), vp, ctypes.c_size_t, vp,
                                  ctypes.POINTER(vp)]),
        "riot_batch_free": (None, [vp]),
        "riot_batch_buffers": (i32, [vp, ctypes.POINTER(_BatchIO)]),
        "riot_batch_run": (i32, [vp, u64]),
        "riot_batch_set_layout": (i32, [vp, i32, i32]),
        "riot_batch_autotune": (i32, [vp, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                      ctypes.POINTER(ctypes.c_float)]),
        "riot_batch_capture": (i32, [vp, u64]),
        "riot_batch_replay": (i32, [vp]),
        "riot_batch_problem": (i32, [vp, i32, ctypes.POINTER(vp)]),
        "riot_gaussian_taps": (i32, [dbl, dbl, i32, vp]),
        "riot_ckpt_forward": (i32, [vp, vp, vp, vp]),
        "riot_ckpt_tangent": (i32, [vp, i32, vp, vp, vp]),
        "riot_ckpt_adjoint": (i32, [vp, i32, vp, vp, vp]),
        "riot_sketch_workspace_bytes": (ctypes.c_size_t, [i32, i32]),
        "riot_sketch_init": (i32, [i32, i32, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]),
        "riot_sketch_free": (None, [vp]),
        "riot_sketch_eig": (i32, [vp, i32, vp, vp, vp, vp, ctypes.POINTER(_RsvdInfo)]),
        "riot_sketch_increment": (i32, [vp, i32, vp, vp, vp, i32, vp, ctypes.POINTER(dbl),
                                        ctypes.POINTER(i32)]),
        "riot_sketch_eig_noalloc": (i32, [i32, i32, vp, vp, vp, vp, vp, ctypes.POINTER(_RsvdInfo)]),
        "riot_sketch_noalloc_max_bytes": (ctypes.c_size_t, []),
        "riot_tracer_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(_TracerDesc)]),
        "riot_tracer_init": (i32, [ctypes.POINTER(_TracerDesc), vp, ctypes.c_size_t, vp,
                                   ctypes.POINTER(vp)]),
        "riot_tracer_free": (None, [vp]),
        "riot_tracer_forward": (i32, [vp, vp, vp]),
        "riot_tracer_tangent": (i32, [vp, i32, vp, vp]),
        "riot_tracer_adjoint": (i32, [vp, i32, vp, vp]),
        "riot_tracer_apply_L": (i32, [vp, i32, vp, vp]),
        "riot_tracer_hess_apply": (i32, [vp, i32, vp, vp]),
        "riot_tracer_gradient": (i32, [vp, vp, vp, vp, ctypes.POINTER(dbl)]),
        "riot_exp_corr_sqrt": (i32, [i32, dbl, vp]),
        "riot_batch_profile": (i32, [vp, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(dbl),
                                     ctypes.POINTER(i32)]),
        "riot_set_obs": (i32, [vp, vp]),
        "riot_proj_residual": (i32, [vp, i32, vp, vp, ctypes.POINTER(dbl)]),
        "riot_sketch_residual": (i32, [vp, i32, vp, vp, ctypes.POINTER(dbl)]),
        "riot_net_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(_NetDesc)]),
        "riot_net_init": (i32, [ctypes.POINTER(_NetDesc), vp, ctypes.c_size_t, vp,
                                ctypes.POINTER(vp)]),
        "riot_net_free": (None, [vp]),
        "riot_net_param_count": (ctypes.c_int64, [vp]),
        "riot_net_set_params": (i32, [vp, vp, vp]),
        "riot_net_get_params": (i32, [vp, vp, vp]),
        "riot_net_forward": (i32, [vp, i32, vp, vp, vp, i32]),
        "riot_net_backward": (i32, [vp, i32, vp]),
        "riot_net_adam": (i32, [vp, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                ctypes.c_float, i32]),
        "riot_net_capture_loss": (i32, [vp, i32, vp, vp, vp, ctypes.POINTER(dbl), vp]),
        "riot_net_train_step": (i32, [vp, i32, vp, vp, vp, ctypes.c_float, i32,
                                      ctypes.POINTER(dbl)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _lib = lib
    return lib


def _check(status: int, where: str):
    if status != RIOT_OK:
        raise RiotError(status, where)


def colmajor(x, device="cuda") -> torch.Tensor:
    """float64 tensor of shape (n, m) with column-major strides (1, n)."""
    t = torch.as_tensor(x, dtype=torch.float64)
    if t.dim() == 1:
        return t.to(device).contiguous()
    return t.t().contiguous().t().to(device) if t.device.type != "cuda" else t.t().contiguous().t()


def empty_colmajor(n: int, m: int, device="cuda") -> torch.Tensor:
    return torch.empty((m, n), dtype=torch.float64, device=device).t()


def _ptr(t):
    if t is None:
        return None
    assert t.is_cuda and t.dtype == torch.float64
    if t.dim() == 2:
        # a single column's second stride is immaterial (torch reports 1 or n)
        assert t.stride(0) == 1 and (t.shape[1] == 1 or t.stride(1) == t.shape[0]), \
            "expected column-major (1, n) strides"
    else:
        assert t.is_contiguous()
    return ctypes.c_void_p(t.data_ptr())


@dataclass
class RsvdInfo:
    chol_shifts: int
    qr_passes: int
    k_asym: float
    orth_err: float
    kappa_est: float = float("nan")
    resid_est: float = float("nan")


class Riot:
    """One inner-loop problem (eqs. 2-3) bound to a device workspace and a stream."""

    _pending = None  # (v, g) of a deferred gradient, kept allocated until the join

    def __init__(self, n, nsteps, dt, forcing, obs_step, obs_idx, y, rinv, taps, m_max,
                 prec=FP64, elems_per_lane=0, device="cuda", ckpt_stride=0):
        self.lib = load_library()
        self.n, self.nsteps, self.m_max = int(n), int(nsteps), int(m_max)
        self.device = torch.device(device)
        self._obs_step = np.ascontiguousarray(obs_step, dtype=np.int32)
        self._obs_idx = np.ascontiguousarray(obs_idx, dtype=np.int32)
        self._y = np.ascontiguousarray(y, dtype=np.float64)
        self._rinv = np.ascontiguousarray(rinv, dtype=np.float64)
        self._taps = np.ascontiguousarray(taps, dtype=np.float64)
        self.nobs = int(self._obs_step.size)
        d = _Desc()
        d.n, d.nsteps, d.dt, d.forcing, d.nobs = self.n, self.nsteps, float(dt), float(forcing), self.nobs
        P = lambda a, c: a.ctypes.data_as(ctypes.POINTER(c))  # noqa: E731
        d.obs_step, d.obs_idx = P(self._obs_step, ctypes.c_int32), P(self._obs_idx, ctypes.c_int32)
        d.y, d.rinv = P(self._y, ctypes.c_double), P(self._rinv, ctypes.c_double)
        d.l_halfwidth = int(self._taps.size - 1)
        d.l_taps = P(self._taps, ctypes.c_double)
        d.m_max, d.prec, d.elems_per_lane = self.m_max, int(prec), int(elems_per_lane)
        d.ckpt_stride = int(ckpt_stride)
        self.ckpt_stride = int(ckpt_stride)
        self._desc = d
        nbytes = self.lib.riot_workspace_bytes(ctypes.byref(d))
        if nbytes == 0:
            raise RiotError(-1, "riot_workspace_bytes")
        self.workspace_bytes = int(nbytes)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        _check(self.lib.riot_init(ctypes.byref(d), ctypes.c_void_p(aligned), ctypes.c_size_t(nbytes),
                                  ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
               "riot_init")
        self.h = h

    def close(self):
        if getattr(self, "h", None) and not getattr(self, "_borrowed", False):
            self.lib.riot_free(self.h)
        self.h = None

    def set_pass_sync(self, on: bool):
        """CholeskyQR passes launched on the host's reading of each pass's decision (True, the
        default) or all launched and predicated on the device (False)."""
        _check(self.lib.riot_set_pass_sync(self.h, 1 if on else 0), "riot_set_pass_sync")

    @classmethod
    def _bind(cls, lib, h, n, nsteps, m_max, nobs, device, stream, owner):
        """Wrap a handle owned by someone else (a batch's problem); it is never freed here."""
        self = cls.__new__(cls)
        self.lib, self.h, self._borrowed, self._owner = lib, h, True, owner
        self.n, self.nsteps, self.m_max, self.nobs = int(n), int(nsteps), int(m_max), int(nobs)
        self.device, self.stream = device, stream
        return self

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- calls ---------------------------------------------------------------
    def linearize(self, x, v=None, want_cost=True, out=None, defer_gradient=False):
        """Trajectory, innovation and gradient. With defer_gradient the gradient's adjoint
        sweep runs on the handle's second stream beside the calls that follow (rsvd,
        hess_apply); g is complete after join(), which increment() and every other call
        that may read it perform first."""
        x = colmajor(x, self.device)
        v = None if v is None else colmajor(v, self.device)
        if out is None:
            d = torch.empty(max(self.nobs, 1), dtype=torch.float64, device=self.device)
            g = torch.empty(self.n, dtype=torch.float64, device=self.device)
        else:
            d, g = out
        J = ctypes.c_double(0.0)
        fn = self.lib.riot_linearize_deferred if defer_gradient else self.lib.riot_linearize
        _check(fn(self.h, _ptr(x), _ptr(v), _ptr(d), _ptr(g),
                  ctypes.byref(J) if want_cost else None), "riot_linearize")
        # the second stream reads v and writes g until the join: keep both allocated
        self._pending = (v, g) if defer_gradient else None
        return d[: self.nobs], g, (J.value if want_cost else None)

    def join(self):
        """Wait (in the handle's stream order) for a deferred gradient."""
        _check(self.lib.riot_join(self.h), "riot_join")
        self._pending = None

    def hess_apply(self, W, add_identity=False, out=None):
        W = colmajor(W, self.device)
        if W.dim() == 1:
            W = W.reshape(-1, 1).t().contiguous().t()
        m = W.shape[1]
        Y = empty_colmajor(self.n, m, self.device) if out is None else out
        _check(self.lib.riot_hess_apply(self.h, m, _ptr(W), _ptr(Y), int(bool(add_identity))),
               "riot_hess_apply")
        return Y

    def set_obs(self, y):
        """New observed values (same locations); linearize again before the next products."""
        y = colmajor(np.ascontiguousarray(y, dtype=np.float64) if not torch.is_tensor(y) else y,
                     self.device)
        assert y.numel() == self.nobs
        _check(self.lib.riot_set_obs(self.h, _ptr(y)), "riot_set_obs")

    def proj_residual(self, Q, AQ):
        """||A Q - Q Q^T A Q||_F / ||A Q||_F for orthonormal Q and AQ = hess_apply(Q)."""
        rho = ctypes.c_double()
        _check(self.lib.riot_proj_residual(self.h, Q.shape[1], _ptr(Q), _ptr(AQ), ctypes.byref(rho)),
               "riot_proj_residual")
        return rho.value

    def rsvd(self, k, p_os, q=0, Omega=None, seed=0, want_info=True, lam=None, V=None):
        m = k + p_os
        Om = None if Omega is None else colmajor(Omega, self.device)
        lam = torch.empty(m, dtype=torch.float64, device=self.device) if lam is None else lam
        V = empty_colmajor(self.n, m, self.device) if V is None else V
        info = _RsvdInfo()
        _check(self.lib.riot_rsvd(self.h, k, p_os, q, _ptr(Om), ctypes.c_uint64(seed), _ptr(lam),
                                  _ptr(V), ctypes.byref(info) if want_info else None), "riot_rsvd")
        inf = RsvdInfo(info.chol_shifts, info.qr_passes, info.k_asym, info.orth_err, info.kappa_est,
                         info.resid_est) if want_info else None
        return lam, V, inf

    def increment(self, lam, V, g, k=None, mode="adaptive", want_host=True, dz=None, dx=None):
        k = lam.numel() if k is None else k
        dz = torch.empty(self.n, dtype=torch.float64, device=self.device) if dz is None else dz
        dx = torch.empty(self.n, dtype=torch.float64, device=self.device) if dx is None else dx
        dofs = ctypes.c_double(0.0)
        mu = ctypes.c_int32(0)
        _check(self.lib.riot_increment(self.h, k, _ptr(lam), _ptr(V), _ptr(g), MODES[mode], _ptr(dz),
                                       _ptr(dx), ctypes.byref(dofs) if want_host else None,
                                       ctypes.byref(mu) if want_host else None), "riot_increment")
        self._pending = None  # the library joined a deferred gradient first
        used = {LRA: "lra", LRU: "lru"}.get(mu.value) if want_host else None
        return dz, dx, (dofs.value if want_host else None), used

    def increment_select(self, lam, V, g, x, v=None, k=None):
        """Both updates, two nonlinear windows, the lower non-quadratic cost kept
        (riot_increment_select). Returns (dz, dx, mode, (J_lra, J_lru))."""
        k = lam.numel() if k is None else int(k)
        dz = torch.empty(self.n, dtype=torch.float64, device=self.device)
        dx = torch.empty(self.n, dtype=torch.float64, device=self.device)
        Jh = (ctypes.c_double * 2)()
        mu = ctypes.c_int32(0)
        xx = colmajor(x, self.device)
        vv = None if v is None else colmajor(v, self.device)
        _check(self.lib.riot_increment_select(self.h, k, _ptr(lam), _ptr(V), _ptr(g), _ptr(xx),
                                              _ptr(vv), _ptr(dz), _ptr(dx),
                                              ctypes.cast(Jh, ctypes.POINTER(ctypes.c_double)),
                                              ctypes.byref(mu)), "riot_increment_select")
        self._pending = None
        return dz, dx, {LRA: "lra", LRU: "lru"}[mu.value], (Jh[0], Jh[1])

    # -- spectral preconditioner and rotation (Alg. 3) ------------------------
    @staticmethod
    def _levels(levels):
        nl = len(levels)
        Vp = (ctypes.c_void_p * max(nl, 1))(*[ctypes.c_void_p(V.data_ptr()) for V, _ in levels])
        lp = (ctypes.c_void_p * max(nl, 1))(*[ctypes.c_void_p(lam.data_ptr()) for _, lam in levels])
        mj = (ctypes.c_int32 * max(nl, 1))(*[int(V.shape[1]) for V, _ in levels])
        for V, lam in levels:
            _ptr(V), _ptr(lam)  # layout checks
        return nl, Vp, mj, lp

    def precond_apply(self, levels, X, op):
        """In place: op 'P', 'PT' or 'Pinv' of the preconditioner built from levels
        [(V_j, lambda_j), ...] (device tensors)."""
        X = self._block(X) if X.dim() == 1 else X
        nl, Vp, mj, lp = self._levels(levels)
        _check(self.lib.riot_precond_apply(self.h, nl, Vp, mj, lp, {"P": 0, "PT": 1, "Pinv": 2}[op],
                                           X.shape[1], _ptr(X)), "riot_precond_apply")
        return X

    def precond_hess_apply(self, levels, W, out=None):
        W = self._block(W)
        Y = empty_colmajor(self.n, W.shape[1], self.device) if out is None else out
        nl, Vp, mj, lp = self._levels(levels)
        _check(self.lib.riot_precond_hess_apply(self.h, nl, Vp, mj, lp, W.shape[1], _ptr(W),
                                                _ptr(Y)), "riot_precond_hess_apply")
        return Y

    def orth(self, X):
        X = self._block(X)
        Q = empty_colmajor(self.n, X.shape[1], self.device)
        _check(self.lib.riot_orth(self.h, X.shape[1], _ptr(X), _ptr(Q)), "riot_orth")
        return Q

    def project_out(self, U, X):
        """In place: X <- (I - U U^T) X."""
        _check(self.lib.riot_project_out(self.h, U.shape[1], _ptr(U), X.shape[1], _ptr(X)),
               "riot_project_out")
        return X

    def outer_update(self, dv, v, x):
        """In place: v += dv, x += L dv."""
        _check(self.lib.riot_outer_update(self.h, _ptr(dv), _ptr(v), _ptr(x)), "riot_outer_update")

    # -- VarBL (Alg. 2) ---------------------------------------------------------
    def gradient_sample(self, x, v, eps_b, eps_o, out=None):
        """Gradient at x + L eps_b, v + eps_b with observations y - R^{1/2} eps_o (eps_b None:
        unperturbed state). Leaves the handle to be linearised again."""
        g = torch.empty(self.n, dtype=torch.float64, device=self.device) if out is None else out
        xx = colmajor(x, self.device)
        vv = None if v is None else colmajor(v, self.device)
        eb = None if eps_b is None else colmajor(eps_b, self.device)
        eo = colmajor(eps_o, self.device)
        _check(self.lib.riot_gradient_sample(self.h, _ptr(xx), _ptr(vv), _ptr(eb), _ptr(eo), _ptr(g)),
               "riot_gradient_sample")
        return g

    def block_lanczos(self, B, g, iters):
        """(lambda, U, dz, dx) of Alg. 2's inner loop from gradient samples B [n x l]."""
        B = self._block(B)
        l = B.shape[1]
        lam = torch.empty(l * iters, dtype=torch.float64, device=self.device)
        U = empty_colmajor(self.n, l * iters, self.device)
        dz = torch.empty(self.n, dtype=torch.float64, device=self.device)
        dx = torch.empty(self.n, dtype=torch.float64, device=self.device)
        _check(self.lib.riot_block_lanczos(self.h, l, int(iters), _ptr(B), _ptr(g), _ptr(lam), _ptr(U),
                                           _ptr(dz), _ptr(dx)), "riot_block_lanczos")
        self._pending = None
        return lam, U, dz, dx

    # -- RIOT-PSAS (observation-space solve) ----------------------------------
    def psas_hess_apply(self, W, out=None):
        """Y = R^{-1/2} G B G^T R^{-1/2} W for observation-space probes W [nobs x m]."""
        W = colmajor(W, self.device)
        if W.dim() == 1:
            W = W.reshape(-1, 1).t().contiguous().t()
        Y = empty_colmajor(self.nobs, W.shape[1], self.device) if out is None else out
        _check(self.lib.riot_psas_hess_apply(self.h, W.shape[1], _ptr(W), _ptr(Y)),
               "riot_psas_hess_apply")
        return Y

    def psas_rhs(self, d, xb_minus_x=None):
        """R^{-1/2} (d - G (x_b - x)) (xb_minus_x None: x = x_b)."""
        rhs = torch.empty(self.nobs, dtype=torch.float64, device=self.device)
        dd = colmajor(d, self.device)
        xx = None if xb_minus_x is None else colmajor(xb_minus_x, self.device)
        _check(self.lib.riot_psas_rhs(self.h, _ptr(dd), _ptr(xx), _ptr(rhs)), "riot_psas_rhs")
        return rhs

    def psas_increment(self, lam, U, rhs, k=None, mode="adaptive"):
        """(dw, dx, mode): the dual increment and dx = B G^T dw (new state x_b + dx)."""
        k = lam.numel() if k is None else int(k)
        dw = torch.empty(self.nobs, dtype=torch.float64, device=self.device)
        dx = torch.empty(self.n, dtype=torch.float64, device=self.device)
        mu = ctypes.c_int32(0)
        _check(self.lib.riot_psas_increment(self.h, k, _ptr(lam), _ptr(U), _ptr(rhs), MODES[mode],
                                            _ptr(dw), _ptr(dx), ctypes.byref(mu)),
               "riot_psas_increment")
        self._pending = None
        return dw, dx, {LRA: "lra", LRU: "lru"}[mu.value]

    def posterior_cov(self, lam, V, k=None, mode="adaptive", diag=True, dense=False,
                      want_host=True, out=None):
        k = lam.numel() if k is None else k
        if out is None:
            W = empty_colmajor(self.n, k, self.device)
            coef = torch.empty(k, dtype=torch.float64, device=self.device)
            dg = torch.empty(self.n, dtype=torch.float64, device=self.device) if diag else None
        else:
            W, coef, dg = out
        P = empty_colmajor(self.n, self.n, self.device) if dense else None
        mu = ctypes.c_int32(0)
        _check(self.lib.riot_posterior_cov(self.h, k, _ptr(lam), _ptr(V), MODES[mode], _ptr(W),
                                           _ptr(coef), _ptr(dg), _ptr(P),
                                           ctypes.byref(mu) if want_host else None),
               "riot_posterior_cov")
        return W, coef, dg, P, ({LRA: "lra", LRU: "lru"}.get(mu.value) if want_host else None)

    def cg(self, g, iters, rtol=0.0, record=False):
        dz = torch.empty(self.n, dtype=torch.float64, device=self.device)
        its = empty_colmajor(self.n, max(iters, 1), self.device) if record else None
        used = ctypes.c_int32(0)
        _check(self.lib.riot_cg(self.h, _ptr(g), int(iters), float(rtol), _ptr(dz), _ptr(its),
                                ctypes.byref(used)), "riot_cg")
        return dz, (its[:, : used.value] if record else None), used.value

    def forecast(self, x0, nsteps):
        x0 = colmajor(x0, self.device)
        out = torch.empty(self.n, dtype=torch.float64, device=self.device)
        _check(self.lib.riot_forecast(self.h, _ptr(x0), int(nsteps), _ptr(out)), "riot_forecast")
        return out

    def apply_L(self, X):
        X = colmajor(X, self.device)
        vec = X.dim() == 1
        if vec:
            X = X.reshape(-1, 1).t().contiguous().t()
        Y = empty_colmajor(self.n, X.shape[1], self.device)
        _check(self.lib.riot_apply_L(self.h, X.shape[1], _ptr(X), _ptr(Y)), "riot_apply_L")
        return Y[:, 0] if vec else Y

    def _block(self, X):
        X = colmajor(X, self.device)
        if X.dim() == 1:
            X = X.reshape(-1, 1).t().contiguous().t()
        return X

    def tl_apply(self, X):
        """Z = G X (observations x columns)."""
        X = self._block(X)
        Z = empty_colmajor(max(self.nobs, 1), X.shape[1], self.device)
        _check(self.lib.riot_tl_apply(self.h, X.shape[1], _ptr(X), _ptr(Z)), "riot_tl_apply")
        return Z[: self.nobs]

    def ad_apply(self, Fo):
        """X = G^T Fo."""
        Fo = self._block(Fo)
        X = empty_colmajor(self.n, Fo.shape[1], self.device)
        _check(self.lib.riot_ad_apply(self.h, Fo.shape[1], _ptr(Fo), _ptr(X)), "riot_ad_apply")
        return X

    def gn_apply(self, X, out=None):
        """Y = G^T R^{-1} G X."""
        X = self._block(X)
        Y = empty_colmajor(self.n, X.shape[1], self.device) if out is None else out
        _check(self.lib.riot_gn_apply(self.h, X.shape[1], _ptr(X), _ptr(Y)), "riot_gn_apply")
        return Y

    # -- checkpointed observation map (handles built with ckpt_stride > 0) ----
    def n_checkpoints(self):
        c = self.ckpt_stride
        return (self.nsteps + c - 1) // c + 1 if self.nsteps > 0 else 1

    def ckpt_forward(self, x0):
        """(checkpoints n x (nseg+1), observed values [nobs]) of the window from x0."""
        x0 = colmajor(x0, self.device)
        ck = empty_colmajor(self.n, self.n_checkpoints(), self.device)
        obs = torch.empty(max(self.nobs, 1), dtype=torch.float64, device=self.device)
        _check(self.lib.riot_ckpt_forward(self.h, _ptr(x0), _ptr(ck), _ptr(obs)), "riot_ckpt_forward")
        return ck, obs[: self.nobs]

    def ckpt_tangent(self, ck, dX0):
        """dObs [nobs x m] = G dX0 on the checkpointed trajectory."""
        dX0 = self._block(dX0)
        m = dX0.shape[1]
        dObs = empty_colmajor(max(self.nobs, 1), m, self.device)
        _check(self.lib.riot_ckpt_tangent(self.h, m, _ptr(ck), _ptr(dX0), _ptr(dObs)),
               "riot_ckpt_tangent")
        return dObs[: self.nobs]

    def ckpt_adjoint(self, ck, gObs):
        """gX0 [n x m] = G^T gObs on the checkpointed trajectory."""
        gObs = colmajor(gObs, self.device)
        if gObs.dim() == 1:
            gObs = gObs.reshape(-1, 1).t().contiguous().t()
        m = gObs.shape[1]
        gX0 = empty_colmajor(self.n, m, self.device)
        _check(self.lib.riot_ckpt_adjoint(self.h, m, _ptr(ck), _ptr(gObs), _ptr(gX0)),
               "riot_ckpt_adjoint")
        return gX0

    def philox_normal(self, n, m, seed, stream=0, out=None):
        out = empty_colmajor(n, m, self.device) if out is None else out
        assert out.shape == (n, m)
        _check(self.lib.riot_philox_normal(self.h, n, m, ctypes.c_uint64(seed), ctypes.c_uint64(stream),
                                           _ptr(out)), "riot_philox_normal")
        return out


def gaussian_taps(ell, sigma_b):
    """Half-kernel taps of the library's Gaussian square root of B (riot_gaussian_taps)."""
    lib = load_library()
    w = lib.riot_gaussian_taps(float(ell), float(sigma_b), 0, None)
    if w < 0:
        raise RiotError(-1, "riot_gaussian_taps")
    taps = np.empty(w + 1)
    lib.riot_gaussian_taps(float(ell), float(sigma_b), w + 1, taps.ctypes.data_as(ctypes.c_void_p))
    return taps


def exp_corr_sqrt(n, ell):
    """Library square root of the periodic 1-D exponential correlation (riot_exp_corr_sqrt)."""
    L1 = np.empty((int(n), int(n)))
    _check(load_library().riot_exp_corr_sqrt(int(n), float(ell), L1.ctypes.data_as(ctypes.c_void_p)),
           "riot_exp_corr_sqrt")
    return L1


class RiotBatch:
    """Many independent inner-loop problems run together (C ABI riot_batch_*).

    problems: sequence of dicts with keys n, nsteps, dt, forcing, obs_step, obs_idx, y,
    rinv, taps, m. The batch owns packed device buffers; `x`, `grad`, `lam`, `V`, `dz`,
    `dx`, `d` are torch views of them (problem j's slices via vec/lam_of/V_of). All calls
    run on the batch's own stream (non-default, so that the pipeline can be captured).
    """

    def __init__(self, problems, prec=FP64, device="cuda"):
        self.lib = load_library()
        self.device = torch.device(device)
        self.stream = torch.cuda.Stream(device=self.device)
        self.P = len(problems)
        descs = (_Desc * self.P)()
        self._keep = []
        self.n, self.m, self.nsteps, self.nobs = [], [], [], []
        P = lambda a, c: a.ctypes.data_as(ctypes.POINTER(c))  # noqa: E731
        for j, pr in enumerate(problems):
            arrs = [np.ascontiguousarray(pr["obs_step"], dtype=np.int32),
                    np.ascontiguousarray(pr["obs_idx"], dtype=np.int32),
                    np.ascontiguousarray(pr["y"], dtype=np.float64),
                    np.ascontiguousarray(pr["rinv"], dtype=np.float64),
                    np.ascontiguousarray(pr["taps"], dtype=np.float64)]
            self._keep.append(arrs)
            d = descs[j]
            d.n, d.nsteps, d.dt, d.forcing = int(pr["n"]), int(pr["nsteps"]), float(pr["dt"]), float(pr["forcing"])
            d.nobs = int(arrs[0].size)
            d.obs_step, d.obs_idx = P(arrs[0], ctypes.c_int32), P(arrs[1], ctypes.c_int32)
            d.y, d.rinv = P(arrs[2], ctypes.c_double), P(arrs[3], ctypes.c_double)
            d.l_halfwidth, d.l_taps = int(arrs[4].size - 1), P(arrs[4], ctypes.c_double)
            d.m_max, d.prec, d.elems_per_lane = int(pr["m"]), int(prec), 8
            self.n.append(d.n), self.m.append(d.m_max), self.nsteps.append(d.nsteps)
            self.nobs.append(d.nobs)
        nbytes = self.lib.riot_batch_workspace_bytes(self.P, descs)
        if nbytes == 0:
            raise RiotError(-1, "riot_batch_workspace_bytes")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        b = ctypes.c_void_p()
        _check(self.lib.riot_batch_init(self.P, descs, ctypes.c_void_p(aligned), ctypes.c_size_t(nbytes),
                                        ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(b)),
               "riot_batch_init")
        self.b = b
        io = _BatchIO()
        _check(self.lib.riot_batch_buffers(self.b, ctypes.byref(io)), "riot_batch_buffers")
        self.off_n = np.concatenate([[0], np.cumsum(self.n)]).astype(np.int64)
        self.off_m = np.concatenate([[0], np.cumsum(self.m)]).astype(np.int64)
        self.off_nm = np.concatenate([[0], np.cumsum(np.asarray(self.n) * np.asarray(self.m))]).astype(np.int64)
        self.off_obs = np.concatenate([[0], np.cumsum(np.maximum(self.nobs, 1))]).astype(np.int64)

        def view(ptr, count):
            off = ptr - base
            return self.workspace[off: off + 8 * count].view(torch.float64)
        tn, tm, tnm = int(self.off_n[-1]), int(self.off_m[-1]), int(self.off_nm[-1])
        self.x, self.grad = view(io.x, tn), view(io.grad, tn)
        self.lam, self.V = view(io.lambda_, tm), view(io.V, tnm)
        self.dz, self.dx = view(io.dz, tn), view(io.dx, tn)
        self.d = view(io.d, int(self.off_obs[-1]))

    def close(self):
        if getattr(self, "b", None):
            self.lib.riot_batch_free(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # packed slices of problem j
    def vec(self, j, t):
        return t[int(self.off_n[j]): int(self.off_n[j + 1])]

    def lam_of(self, j):
        return self.lam[int(self.off_m[j]): int(self.off_m[j + 1])]

    def V_of(self, j):
        return self.V[int(self.off_nm[j]): int(self.off_nm[j + 1])].view(self.m[j], self.n[j]).t()

    def set_x(self, xs):
        with torch.cuda.stream(self.stream):
            for j, x in enumerate(xs):
                self.vec(j, self.x).copy_(torch.as_tensor(x, dtype=torch.float64))

    def run(self, seed=0):
        _check(self.lib.riot_batch_run(self.b, ctypes.c_uint64(seed)), "riot_batch_run")

    def set_layout(self, workgroups, wave_max_threads):
        _check(self.lib.riot_batch_set_layout(self.b, int(workgroups), int(wave_max_threads)),
               "riot_batch_set_layout")

    def autotune(self):
        wg, wv, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_float()
        _check(self.lib.riot_batch_autotune(self.b, ctypes.byref(wg), ctypes.byref(wv), ctypes.byref(ms)),
               "riot_batch_autotune")
        return wg.value, wv.value, ms.value

    def capture(self, seed=0):
        _check(self.lib.riot_batch_capture(self.b, ctypes.c_uint64(seed)), "riot_batch_capture")

    def replay(self):
        _check(self.lib.riot_batch_replay(self.b), "riot_batch_replay")

    def profile(self):
        """(ms, load balance, tiles) of one instrumented probe-product launch."""
        ms, bf, nt = ctypes.c_float(), ctypes.c_double(), ctypes.c_int32()
        _check(self.lib.riot_batch_profile(self.b, ctypes.byref(ms), ctypes.byref(bf), ctypes.byref(nt)),
               "riot_batch_profile")
        return ms.value, bf.value, nt.value

    def problem(self, j):
        """A Riot bound to problem j's handle inside the batch (same stream and workspace)."""
        h = ctypes.c_void_p()
        _check(self.lib.riot_batch_problem(self.b, int(j), ctypes.byref(h)), "riot_batch_problem")
        return Riot._bind(self.lib, h, self.n[j], self.nsteps[j], self.m[j], self.nobs[j], self.device,
                          self.stream, self)


def _aligned_workspace(nbytes, device):
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    return ws, (ws.data_ptr() + 255) // 256 * 256


def _cols(t, rows, device):
    t = colmajor(t, device)
    if t.dim() == 1:
        t = t.reshape(-1, 1).t().contiguous().t()
    assert t.shape[0] == rows
    return t


class Sketch:
    """Alg. 3 after the probe products, for any operator (C ABI riot_sketch_*)."""

    def __init__(self, n, m_max, device="cuda"):
        self.lib = load_library()
        self.n, self.m_max, self.device = int(n), int(m_max), torch.device(device)
        nb = self.lib.riot_sketch_workspace_bytes(self.n, self.m_max)
        if nb == 0:
            raise RiotError(-1, "riot_sketch_workspace_bytes")
        self.workspace, base = _aligned_workspace(nb, self.device)
        self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        _check(self.lib.riot_sketch_init(self.n, self.m_max, ctypes.c_void_p(base), ctypes.c_size_t(nb),
                                         ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
               "riot_sketch_init")
        self.h = h

    def __del__(self):
        try:
            if getattr(self, "h", None):
                self.lib.riot_sketch_free(self.h)
                self.h = None
        except Exception:
            pass

    def eig(self, Omega, Y, want_info=True):
        Om, Yc = _cols(Omega, self.n, self.device), _cols(Y, self.n, self.device)
        m = Om.shape[1]
        lam = torch.empty(m, dtype=torch.float64, device=self.device)
        V = empty_colmajor(self.n, m, self.device)
        info = _RsvdInfo()
        _check(self.lib.riot_sketch_eig(self.h, m, _ptr(Om), _ptr(Yc), _ptr(lam), _ptr(V),
                                        ctypes.byref(info) if want_info else None), "riot_sketch_eig")
        return lam, V, (RsvdInfo(info.chol_shifts, info.qr_passes, info.k_asym, info.orth_err, info.kappa_est,
                         info.resid_est)
                        if want_info else None)

    def increment(self, lam, V, g, k=None, mode="adaptive"):
        k = V.shape[1] if k is None else int(k)
        dz = torch.empty(self.n, dtype=torch.float64, device=self.device)
        dofs, mu = ctypes.c_double(), ctypes.c_int32()
        _check(self.lib.riot_sketch_increment(self.h, k, _ptr(lam), _ptr(V), _ptr(colmajor(g, self.device)),
                                              MODES[mode], _ptr(dz), ctypes.byref(dofs), ctypes.byref(mu)),
               "riot_sketch_increment")
        return dz, dofs.value, {LRA: "lra", LRU: "lru"}[mu.value]


    def residual(self, Q, AQ):
        """||A Q - Q Q^T A Q||_F / ||A Q||_F (riot_sketch_residual)."""
        Qc, AQc = _cols(Q, self.n, self.device), _cols(AQ, self.n, self.device)
        rho = ctypes.c_double()
        _check(self.lib.riot_sketch_residual(self.h, Qc.shape[1], _ptr(Qc), _ptr(AQc),
                                             ctypes.byref(rho)), "riot_sketch_residual")
        return rho.value


def sketch_eig_noalloc(Omega, Y, want_info=True, lam=None, V=None):
    """riot_sketch_eig_noalloc: Sketch.eig without a handle or workspace (the library's static
    scratch on the current device). Returns (lam, V, info) like Sketch.eig."""
    lib = load_library()
    Yc = colmajor(Y)
    n = Yc.shape[0]
    Om = _cols(Omega, n, Yc.device)
    Yc = _cols(Yc, n, Yc.device)
    m = Om.shape[1]
    lam = torch.empty(m, dtype=torch.float64, device=Yc.device) if lam is None else lam
    V = empty_colmajor(n, m, Yc.device) if V is None else V
    info = _RsvdInfo()
    stream = torch.cuda.current_stream(Yc.device)
    _check(lib.riot_sketch_eig_noalloc(n, m, _ptr(Om), _ptr(Yc), _ptr(lam), _ptr(V),
                                       ctypes.c_void_p(stream.cuda_stream),
                                       ctypes.byref(info) if want_info else None),
           "riot_sketch_eig_noalloc")
    return lam, V, (RsvdInfo(info.chol_shifts, info.qr_passes, info.k_asym, info.orth_err, info.kappa_est,
                         info.resid_est)
                    if want_info else None)


class ProposalNet:
    """Learned sketch proposal: periodic 1-D conv net, its training and inference kernels
    (C ABI riot_net_*). Inputs x: (batch, in_channels, n) float64 (or (batch, n) with one
    input channel); outputs N: (batch, k, n) float32."""

    def __init__(self, n, k=64, channels=64, layers=4, width=9, batch_max=32, segments=1,
                 in_channels=1, device="cuda"):
        self.lib = load_library()
        d = _NetDesc()
        d.n, d.layers, d.channels, d.k, d.width, d.batch_max, d.segments, d.in_channels = (
            int(n), int(layers), int(channels), int(k), int(width), int(batch_max), int(segments),
            int(in_channels))
        self.n, self.k, self.channels, self.layers, self.width = d.n, d.k, d.channels, d.layers, d.width
        self.segments, self.in_channels = d.segments, d.in_channels
        self.batch_max, self.device = d.batch_max, torch.device(device)
        nb = self.lib.riot_net_workspace_bytes(ctypes.byref(d))
        if nb == 0:
            raise RiotError(-1, "riot_net_workspace_bytes")
        self.workspace, base = _aligned_workspace(nb, self.device)
        self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        _check(self.lib.riot_net_init(ctypes.byref(d), ctypes.c_void_p(base), ctypes.c_size_t(nb),
                                      ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
               "riot_net_init")
        self.h = h
        self.nparams = int(self.lib.riot_net_param_count(self.h))
        self.step = 0

    def __del__(self):
        try:
            if getattr(self, "h", None):
                self.lib.riot_net_free(self.h)
                self.h = None
        except Exception:
            pass

    def layer_shapes(self):
        """[(cout, cin, width)] per layer, in the flat parameter order."""
        out, cin = [], self.in_channels
        for li in range(self.layers):
            cout = self.k // self.segments if li == self.layers - 1 else self.channels
            out.append((cout, cin, self.width))
            cin = cout
        return out

    @staticmethod
    def _f64(t):
        assert t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
        return ctypes.c_void_p(t.data_ptr())

    @staticmethod
    def _f32(t):
        assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()
        return ctypes.c_void_p(t.data_ptr())

    def _flat(self, t):
        if t is None:
            return None
        t = torch.as_tensor(t, dtype=torch.float32).to(self.device).contiguous()
        assert t.numel() == self.nparams
        return t

    def set_params(self, flat=None, grads=None):
        """Parameters (a new start: Adam's step count restarts) and/or gradients."""
        p, g = self._flat(flat), self._flat(grads)
        _check(self.lib.riot_net_set_params(self.h, None if p is None else self._f32(p),
                                            None if g is None else self._f32(g)),
               "riot_net_set_params")
        if p is not None:
            self.step = 0

    def params(self):
        p = torch.empty(self.nparams, dtype=torch.float32, device=self.device)
        g = torch.empty(self.nparams, dtype=torch.float32, device=self.device)
        _check(self.lib.riot_net_get_params(self.h, self._f32(p), self._f32(g)), "riot_net_get_params")
        return p, g

    def _states(self, x):
        x = torch.as_tensor(x, dtype=torch.float64).to(self.device)
        x = x.reshape(-1, self.in_channels, self.n).contiguous()
        assert 1 <= x.shape[0] <= self.batch_max
        return x

    def forward(self, x):
        x = self._states(x)
        N = torch.empty((x.shape[0], self.k, self.n), dtype=torch.float32, device=self.device)
        _check(self.lib.riot_net_forward(self.h, x.shape[0], self._f64(x), self._f32(N), None, 0),
               "riot_net_forward")
        return N

    def propose(self, x, Omega):
        """The network's k columns for one state x into Omega[:, :k] (FP64, column-major)."""
        x = self._states(x)
        assert x.shape[0] == 1 and Omega.stride(0) == 1 and Omega.shape[1] >= self.k
        _check(self.lib.riot_net_forward(self.h, 1, self._f64(x), None, ctypes.c_void_p(Omega.data_ptr()),
                                         Omega.stride(1)), "riot_net_forward")
        return Omega

    def backward(self, gN):
        gN = gN.to(torch.float32).contiguous()
        _check(self.lib.riot_net_backward(self.h, gN.shape[0], self._f32(gN)), "riot_net_backward")
        return self.params()[1]

    def capture_loss(self, N, V, w):
        """(loss per sample (numpy), gN) for N (batch, k, n) f32, V (batch, k, n) f64, w (batch, k)."""
        N = N.to(torch.float32).contiguous()
        V = torch.as_tensor(V, dtype=torch.float64).to(self.device).contiguous()
        w = torch.as_tensor(w, dtype=torch.float64).to(self.device).contiguous()
        b = N.shape[0]
        loss = (ctypes.c_double * b)()
        gN = torch.empty_like(N)
        _check(self.lib.riot_net_capture_loss(self.h, b, self._f32(N), self._f64(V), self._f64(w), loss,
                                              self._f32(gN)), "riot_net_capture_loss")
        return np.array(loss[:]), gN

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step += 1
        _check(self.lib.riot_net_adam(self.h, lr, beta1, beta2, eps, self.step), "riot_net_adam")

    def train_step(self, x, V, w, lr):
        """One Adam step on a batch; returns the per-sample losses before the step."""
        x = self._states(x)
        V = torch.as_tensor(V, dtype=torch.float64).to(self.device).contiguous()
        w = torch.as_tensor(w, dtype=torch.float64).to(self.device).contiguous()
        b = x.shape[0]
        loss = (ctypes.c_double * b)()
        self.step += 1
        _check(self.lib.riot_net_train_step(self.h, b, self._f64(x), self._f64(V), self._f64(w), lr, self.step, loss),
               "riot_net_train_step")
        return np.array(loss[:])


class Tracer:
    """Tracer source inversion on a periodic 2-D grid (C ABI riot_tracer_*).

    grid: dict with N, T, dt, u0, u1, v, K, block, ntb. Controls are [ntb][by][bx]
    flattened (ncontrol,), observation vectors follow the caller's observation order.
    """

    def __init__(self, grid, E, obs_t, obs_y, obs_x, y, rinv, L1, sigma, m_max, device="cuda"):
        self.lib = load_library()
        self.device = torch.device(device)
        g = dict(grid)
        self.N, self.T, self.block, self.ntb = int(g["N"]), int(g["T"]), int(g["block"]), int(g["ntb"])
        self.Nb = self.N // self.block
        self.ncontrol = self.ntb * self.Nb * self.Nb
        self.m_max = int(m_max)
        keep = [np.ascontiguousarray(E, dtype=np.float64),
                np.ascontiguousarray(obs_t, dtype=np.int32), np.ascontiguousarray(obs_y, dtype=np.int32),
                np.ascontiguousarray(obs_x, dtype=np.int32), np.ascontiguousarray(y, dtype=np.float64),
                np.ascontiguousarray(rinv, dtype=np.float64), np.ascontiguousarray(L1, dtype=np.float64)]
        self.nobs = int(keep[1].size)
        P = lambda a, c: a.ctypes.data_as(ctypes.POINTER(c))  # noqa: E731
        d = _TracerDesc()
        d.N, d.nsteps, d.dt, d.u0, d.u1, d.v, d.K = (self.N, self.T, float(g["dt"]), float(g["u0"]),
                                                      float(g["u1"]), float(g["v"]), float(g["K"]))
        d.block, d.ntb = self.block, self.ntb
        d.E, d.nobs = P(keep[0], ctypes.c_double), self.nobs
        d.obs_t, d.obs_y, d.obs_x = (P(keep[1], ctypes.c_int32), P(keep[2], ctypes.c_int32),
                                     P(keep[3], ctypes.c_int32))
        d.y, d.rinv, d.L1 = P(keep[4], ctypes.c_double), P(keep[5], ctypes.c_double), P(keep[6], ctypes.c_double)
        d.sigma, d.m_max = float(sigma), self.m_max
        nb = self.lib.riot_tracer_workspace_bytes(ctypes.byref(d))
        if nb == 0:
            raise RiotError(-1, "riot_tracer_workspace_bytes")
        self.workspace_bytes = int(nb)
        self.workspace, base = _aligned_workspace(nb, self.device)
        self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        _check(self.lib.riot_tracer_init(ctypes.byref(d), ctypes.c_void_p(base), ctypes.c_size_t(nb),
                                         ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
               "riot_tracer_init")
        self.h = h
        self.base_version = 0

    def __del__(self):
        try:
            if getattr(self, "h", None):
                self.lib.riot_tracer_free(self.h)
                self.h = None
        except Exception:
            pass

    def forward(self, s):
        """Observed concentrations for controls s; s becomes the derivatives' base."""
        s = colmajor(s, self.device)
        obs = torch.empty(max(self.nobs, 1), dtype=torch.float64, device=self.device)
        _check(self.lib.riot_tracer_forward(self.h, _ptr(s), _ptr(obs)), "riot_tracer_forward")
        self.base_version += 1
        return obs[: self.nobs]

    def _m(self, X, rows):
        X = _cols(X, rows, self.device)
        return X, X.shape[1]

    def tangent(self, dS):
        dS, m = self._m(dS, self.ncontrol)
        out = empty_colmajor(max(self.nobs, 1), m, self.device)
        _check(self.lib.riot_tracer_tangent(self.h, m, _ptr(dS), _ptr(out)), "riot_tracer_tangent")
        return out[: self.nobs]

    def adjoint(self, gObs):
        gObs, m = self._m(gObs, self.nobs)
        out = empty_colmajor(self.ncontrol, m, self.device)
        _check(self.lib.riot_tracer_adjoint(self.h, m, _ptr(gObs), _ptr(out)), "riot_tracer_adjoint")
        return out

    def apply_L(self, Z):
        Z, m = self._m(Z, self.ncontrol)
        out = empty_colmajor(self.ncontrol, m, self.device)
        _check(self.lib.riot_tracer_apply_L(self.h, m, _ptr(Z), _ptr(out)), "riot_tracer_apply_L")
        return out

    def hess_apply(self, W, out=None):
        W, m = self._m(W, self.ncontrol)
        Y = empty_colmajor(self.ncontrol, m, self.device) if out is None else out
        _check(self.lib.riot_tracer_hess_apply(self.h, m, _ptr(W), _ptr(Y)), "riot_tracer_hess_apply")
        return Y

    def gradient(self, v=None, want_cost=True):
        g = torch.empty(self.ncontrol, dtype=torch.float64, device=self.device)
        d = torch.empty(max(self.nobs, 1), dtype=torch.float64, device=self.device)
        J = ctypes.c_double()
        vv = None if v is None else colmajor(v, self.device)
        _check(self.lib.riot_tracer_gradient(self.h, _ptr(vv), _ptr(g), _ptr(d),
                                             ctypes.byref(J) if want_cost else None), "riot_tracer_gradient")
        return g, d[: self.nobs], (J.value if want_cost else None)
