"""Python face of the C ABI: argument marshalling only.

Every numerical step runs inside libfcgle.so (HIP kernels for gfx950).  torch
provides device memory and the current stream.
"""
from __future__ import annotations

import ctypes
import weakref
from typing import Optional, Sequence, Tuple

import numpy as np
import torch

from . import _lib as L

STATE_DTYPE = {"fp64": torch.complex128, "fp32": torch.complex64, "bf16x3": torch.complex64,
               "bf16x6": torch.complex64}
NUM_TILE_CONFIGS = 5  # tile configurations accepted by fcgle_set_tiles (0 .. 4)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


class Plan:
    """A set-up problem: per-axis eigenpairs, f-grids and scratch on one GPU.

    n, alpha, h: per-axis inner points, fractional orders and grid spacings.
    params: (nu, eta, gamma, kappa, zeta).  tau: time step (grids are built for it).
    precision: 'fp64' | 'fp32' | 'bf16x3' | 'bf16x6'.
    """

    def __init__(self, n: Sequence[int], alpha: Sequence[float], h: Sequence[float],
                 params: Sequence[float], tau: float, precision: str = "fp64", fd_order: int = 2,
                 device: Optional[int] = None):
        if not torch.cuda.is_available():
            raise RuntimeError("fcgle.Plan needs a GPU")
        self.lib = L.lib()
        self.n = tuple(int(m) for m in n)
        self.d = len(self.n)
        self.precision = precision
        self.dtype = STATE_DTYPE[precision]
        self.tau = float(tau)
        self.params = tuple(float(p) for p in params)
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        nn = (ctypes.c_int64 * self.d)(*self.n)
        aa = (ctypes.c_double * self.d)(*[float(a) for a in alpha])
        hh = (ctypes.c_double * self.d)(*[float(x) for x in h])
        pp = L.Params(*self.params)
        out = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            L.check(self.lib.fcgle_setup(self.d, nn, aa, hh, ctypes.byref(pp), int(fd_order),
                                         L.PRECISIONS[precision], self.tau, ctypes.byref(out)))
        self.handle = out
        self._state = None  # (weakref to the tensor the library's cached state belongs to, its _version)
        self._sources = []

    # -- lifetime --------------------------------------------------------------------------
    def close(self):
        if getattr(self, "handle", None):
            self.lib.fcgle_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers ---------------------------------------------------------------------------
    def _check_tensor(self, u: torch.Tensor, name: str = "u"):
        if u.dtype != self.dtype:
            raise TypeError(f"{name} must be {self.dtype}, got {u.dtype}")
        if u.device != self.device:
            raise ValueError(f"{name} must live on {self.device}")
        if tuple(u.shape) != self.n:
            raise ValueError(f"{name} has shape {tuple(u.shape)}, expected {self.n}")
        if not u.is_contiguous():
            raise ValueError(f"{name} must be contiguous")

    def empty(self) -> torch.Tensor:
        return torch.empty(self.n, dtype=self.dtype, device=self.device)

    # -- operations ------------------------------------------------------------------------
    def eig(self, mu: int) -> Tuple[np.ndarray, np.ndarray]:
        m = self.n[mu]
        Q = np.empty((m, m))
        lam = np.empty(m)
        L.check(self.lib.fcgle_get_eig(self.handle, mu, Q.ctypes.data_as(L.P_dbl), lam.ctypes.data_as(L.P_dbl)))
        return Q, lam

    def apply_f(self, kind: str, theta: float, u: torch.Tensor, out: Optional[torch.Tensor] = None):
        self._check_tensor(u)
        if out is None:
            out = self.empty()
        self._check_tensor(out, "out")
        L.check(self.lib.fcgle_apply_f(self.handle, L.KINDS[kind], float(theta), _ptr(u), _ptr(out), _stream()))
        return out

    def apply_f_noalloc(self, kind: str, theta: float, u: torch.Tensor, out: torch.Tensor):
        """out = f(theta K) u like apply_f, with no device allocation (fcgle_apply_f_noalloc): the
        library's fixed per-device work space instead of the plan's buffers.  apply_f must have
        run once with the same (kind, theta) on this plan; states up to 16 MiB."""
        self._check_tensor(u)
        self._check_tensor(out, "out")
        L.check(self.lib.fcgle_apply_f_noalloc(self.handle, L.KINDS[kind], float(theta), _ptr(u), _ptr(out),
                                               _stream()))
        return out

    def apply_inv_refined(self, theta: float, v: torch.Tensor, sweeps: int = 1,
                          out: Optional[torch.Tensor] = None, residuals: bool = False):
        """x = (I - theta (nu + i eta) K)^{-1} v to FP64 accuracy: the plan's precision for the
        inverse, `sweeps` refinement sweeps with the residual formed in FP64 (fcgle_apply_inv_refined).
        v and out are complex128 tensors of the plan's shape.  With residuals=True also returns the
        relative residual norms ||v - (I - theta (nu + i eta) K) x_k|| / ||v||, k = 0..sweeps."""
        for t, name in ((v, "v"),) + (((out, "out"),) if out is not None else ()):
            if t.dtype != torch.complex128 or t.device != self.device or tuple(t.shape) != self.n \
                    or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous complex128 tensor of shape {self.n} on {self.device}")
        if out is None:
            out = torch.empty(self.n, dtype=torch.complex128, device=self.device)
        rn = (ctypes.c_double * (sweeps + 1))() if residuals else None
        L.check(self.lib.fcgle_apply_inv_refined(self.handle, float(theta), _ptr(v), _ptr(out), int(sweeps),
                                                 ctypes.cast(rn, L.P_dbl) if rn is not None else None, _stream()))
        return (out, list(rn)) if residuals else out

    def set_source(self, rates: Sequence[complex], tensors: Sequence[torch.Tensor]):
        """s(t) = sum_k exp(rates[k] t) tensors[k]; rates real or complex."""
        for S in tensors:
            self._check_tensor(S, "S")
        self._sources = list(tensors)  # keep alive
        k = len(rates)
        rr = (ctypes.c_double * max(k, 1))(*[complex(r).real for r in rates])
        ri = (ctypes.c_double * max(k, 1))(*[complex(r).imag for r in rates])
        ss = (ctypes.c_void_p * max(k, 1))(*[S.data_ptr() for S in tensors])
        L.check(self.lib.fcgle_set_source(self.handle, k, rr, ri, ss))

    def set_state(self, u: torch.Tensor, u_prev: Optional[torch.Tensor] = None):
        self._check_tensor(u)
        if u_prev is not None:
            self._check_tensor(u_prev, "u_prev")
        L.check(self.lib.fcgle_set_state(self.handle, _ptr(u), _ptr(u_prev), _stream()))
        self._state = (weakref.ref(u), u._version)

    def _sync_state(self, u: torch.Tensor):
        # The library caches the eigenspace state (and the LBDF2 history) of the buffer it last
        # stepped, keyed by its device address.  That address says nothing about the tensor:
        # the caching allocator hands a freed block to the next tensor, and writes through the
        # library do not bump _version.  So the cache is kept only while the caller passes the
        # very tensor object of the last step, not written by torch since.
        st = self._state
        if st is None or st[0]() is not u or st[1] != u._version:
            L.check(self.lib.fcgle_set_state(self.handle, _ptr(u), ctypes.c_void_p(0), _stream()))
        self._state = (weakref.ref(u), u._version)

    def step(self, scheme: str, u: torch.Tensor, t: float) -> torch.Tensor:
        """One step in place from time t.  scheme: 'exp_euler', 'lawson', 'lie', 'lbdf2',
        'strang' (no source term) or 'krogstad'."""
        self._check_tensor(u)
        self._sync_state(u)
        L.check(self.lib.fcgle_step(self.handle, L.SCHEMES[scheme], _ptr(u), float(t), self.tau, _stream()))
        return u

    def run(self, scheme: str, u: torch.Tensor, t0: float, nsteps: int) -> torch.Tensor:
        """nsteps steps in place from t0 (schemes as for step)."""
        self._check_tensor(u)
        self._sync_state(u)
        L.check(self.lib.fcgle_run(self.handle, L.SCHEMES[scheme], _ptr(u), float(t0), self.tau, int(nsteps),
                                   _stream()))
        return u

    def vjp(self, u_n: torch.Tensor, ubar_next: torch.Tensor, t: float, pbar: torch.Tensor,
            ubar_n: Optional[torch.Tensor] = None, scheme: str = "exp_euler") -> torch.Tensor:
        self._check_tensor(u_n, "u_n")
        self._check_tensor(ubar_next, "ubar_next")
        if ubar_n is None:
            ubar_n = self.empty()
        self._check_tensor(ubar_n, "ubar_n")
        if pbar.dtype != torch.float64 or pbar.numel() != 5 or pbar.device != self.device:
            raise ValueError("pbar must be 5 float64 values on the plan's device")
        L.check(self.lib.fcgle_vjp(self.handle, L.SCHEMES[scheme], _ptr(u_n), _ptr(ubar_next), _ptr(ubar_n),
                                   _ptr(pbar), float(t), self.tau, _stream()))
        self._state = None
        return ubar_n

    def vjp_run(self, u_start: torch.Tensor, m: int, ubar: torch.Tensor, pbar: torch.Tensor, t0: float,
                scheme: str = "exp_euler") -> torch.Tensor:
        """Adjoint of m steps from the checkpoint u_start at t0: ubar (cotangent of u_m) is
        replaced in place by the cotangent of u_start; pbar (5 float64 on the device) is added to."""
        self._check_tensor(u_start, "u_start")
        self._check_tensor(ubar, "ubar")
        if pbar.dtype != torch.float64 or pbar.numel() != 5 or pbar.device != self.device:
            raise ValueError("pbar must be 5 float64 values on the plan's device")
        L.check(self.lib.fcgle_vjp_run(self.handle, L.SCHEMES[scheme], _ptr(u_start), int(m), _ptr(ubar),
                                       _ptr(pbar), float(t0), self.tau, _stream()))
        self._state = None
        return ubar

    def check_finite(self, u: torch.Tensor) -> bool:
        self._check_tensor(u)
        rc = self.lib.fcgle_check_finite(self.handle, _ptr(u), _stream())
        if rc == L.ERR_NONFINITE:
            return False
        L.check(rc)
        return True

    def autotune(self, reps: int = 3):
        """Overwrites the library's cached state: the next step starts from the tensor again."""
        L.check(self.lib.fcgle_autotune(self.handle, int(reps), _stream()))
        self._state = None

    def set_tiles(self, axis: int, fwd: bool, cfg: int):
        L.check(self.lib.fcgle_set_tiles(self.handle, int(axis), int(bool(fwd)), int(cfg)))

    def set_fusion(self, prologue: bool = True, epilogue: bool = True, reverse: bool = False,
                   update_in_backward: bool = False, phi1_on_the_fly: bool = False, flows: bool = False):
        """Fuse the nonlinearity into the first / the pointwise epilogue into the last mode
        product; reverse: run forward operators from the last axis to the first;
        update_in_backward: apply the exponential-Euler update in the loads of the first
        backward product instead (even/odd plans, d >= 2); phi1_on_the_fly: that
        update forms phi_1 from separable tables instead of reading the grid (n_1 <= 512);
        flows: fuse the exact nonlinear flows of Strang splitting into the mode products."""
        L.check(self.lib.fcgle_set_fusion(self.handle, (1 if prologue else 0) | (2 if epilogue else 0)
                                          | (4 if reverse else 0) | (8 if update_in_backward else 0)
                                          | (32 if phi1_on_the_fly else 0) | (64 if flows else 0)))

    def set_structure(self, split: bool):
        """True: even/odd half-size mode products (default for fp64/fp32); False: dense."""
        L.check(self.lib.fcgle_set_structure(self.handle, int(bool(split))))

    def set_wide_loads(self, force: bool):
        """True: every N-loader mode product reads through 64-bit element indices (the
        configuration the library picks by itself where 32 rows of the tensor span more
        than 2 GiB); False: that automatic choice."""
        L.check(self.lib.fcgle_set_wide_loads(self.handle, int(bool(force))))

    def describe(self) -> str:
        buf = ctypes.create_string_buffer(1024)
        L.check(self.lib.fcgle_describe(self.handle, buf, 1024))
        return buf.value.decode()

    def timing_enable(self, capacity: int):
        L.check(self.lib.fcgle_timing_enable(self.handle, int(capacity)))

    def timing_read(self, cap: int = 100000):
        """Per-launch records of the mode-product kernels timed since timing_enable:
        a list of (axis, forward, kernel_signature, milliseconds)."""
        ax = (ctypes.c_int * cap)()
        fw = (ctypes.c_int * cap)()
        sg = (ctypes.c_int * cap)()
        ms = (ctypes.c_double * cap)()
        cnt = ctypes.c_int64()
        L.check(self.lib.fcgle_timing_read(self.handle, cap, ax, fw, sg, ms, ctypes.byref(cnt)))
        return [(ax[i], fw[i], sg[i], ms[i]) for i in range(cnt.value)]


class BatchPlan:
    """Independent 2-D problems of uneven sizes advanced together (FP32 MFMA, complex64).

    instances: sequence of (n, alpha, h, params) with n = (n1, n2), alpha/h per axis and
    params = (nu, eta, gamma, kappa, zeta).  tau: shared time step.
    """

    def __init__(self, instances, tau: float, precision: str = "fp32", device: Optional[int] = None):
        if not torch.cuda.is_available():
            raise RuntimeError("fcgle.BatchPlan needs a GPU")
        self.lib = L.lib()
        self.shapes = [tuple(int(m) for m in inst[0]) for inst in instances]
        if any(len(n) != 2 for n in self.shapes):
            raise ValueError("batched instances are 2-D")
        self.count = len(self.shapes)
        self.tau = float(tau)
        self.dtype = STATE_DTYPE[precision]
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        nn = (ctypes.c_int64 * (2 * self.count))(*[m for n in self.shapes for m in n])
        aa = (ctypes.c_double * (2 * self.count))(*[float(a) for inst in instances for a in inst[1]])
        hh = (ctypes.c_double * (2 * self.count))(*[float(x) for inst in instances for x in inst[2]])
        pp = (L.Params * self.count)(*[L.Params(*[float(v) for v in inst[3]]) for inst in instances])
        out = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            L.check(self.lib.fcgle_batch_setup(self.count, nn, aa, hh, pp, L.PRECISIONS[precision], self.tau,
                                               ctypes.byref(out)))
        self.handle = out

    def close(self):
        if getattr(self, "handle", None):
            self.lib.fcgle_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, us, t0: float, nsteps: int, scheme: str = "exp_euler"):
        if len(us) != self.count:
            raise ValueError(f"expected {self.count} state tensors")
        for u, n in zip(us, self.shapes):
            if u.dtype != self.dtype or u.device != self.device or tuple(u.shape) != n or not u.is_contiguous():
                raise ValueError(f"state tensors must be contiguous {self.dtype} of the instance shapes on {self.device}")
        ptrs = (ctypes.c_void_p * self.count)(*[u.data_ptr() for u in us])
        L.check(self.lib.fcgle_batch_run(self.handle, L.SCHEMES[scheme], ptrs, float(t0), self.tau, int(nsteps),
                                         _stream()))
        return us

    def autotune(self, reps: int = 3):
        L.check(self.lib.fcgle_autotune(self.handle, int(reps), _stream()))

    def set_persistent(self, persistent: bool, spin_limit: int = 0):
        """Run as one persistent launch per call (True) or as the graph of grouped launches
        (False); spin_limit bounds each dependency wait of the persistent kernel (0: unchanged)."""
        L.check(self.lib.fcgle_batch_set_persistent(self.handle, int(bool(persistent)), int(spin_limit)))

    def describe(self) -> str:
        buf = ctypes.create_string_buffer(1024)
        L.check(self.lib.fcgle_describe(self.handle, buf, 1024))
        return buf.value.decode()


def decode_signature(sig: int) -> dict:
    """Inverse of the kernel signature of fcgle_timing_read."""
    structure = sig // 4096
    sig %= 4096
    ek = sig % 8
    sig //= 8
    pk = sig % 8
    sig //= 8
    tl = sig % 2
    sig //= 2
    cfg = sig % 8
    prec = sig // 8
    return {"precision": ["fp64", "fp32", "bf16x3", "bf16x6"][prec], "tile_cfg": cfg, "t_loader": bool(tl),
            "structure": ["dense", "even_odd_fwd", "even_odd_bwd", "even_odd_fwd_fused"][structure],
            "prologue": ["none", "nonlinearity", "exp_euler_update", "exp_euler_update_otf", "nonlinear_flow",
                         "?", "?", "?"][pk],
            "epilogue": ["store", "grid", "sep_exp", "exp_euler", "keep_old", "exp_euler_rec", "axpy",
                         "nonlinear_flow"][ek]}


# -- host-only helpers ---------------------------------------------------------------------

def host_fd_weights(alpha: float, n: int, fd_order: int = 2) -> np.ndarray:
    g = np.empty(n)
    L.check(L.lib().fcgle_host_fd_weights(float(alpha), int(n), int(fd_order), g.ctypes.data_as(L.P_dbl)))
    return g


def host_eig(n: int, alpha: float, h: float, fd_order: int = 2):
    Q = np.empty((n, n))
    lam = np.empty(n)
    L.check(L.lib().fcgle_host_eig(int(n), float(alpha), float(h), int(fd_order), Q.ctypes.data_as(L.P_dbl),
                                   lam.ctypes.data_as(L.P_dbl)))
    return Q, lam


def host_fz(kind: str, z: np.ndarray) -> np.ndarray:
    z = np.ascontiguousarray(np.asarray(z, dtype=np.complex128))
    zz = z.view(np.float64).reshape(-1)
    out = np.empty_like(zz)
    L.check(L.lib().fcgle_host_fz(L.KINDS[kind], z.size, zz.ctypes.data_as(L.P_dbl), out.ctypes.data_as(L.P_dbl)))
    return out.view(np.complex128).reshape(z.shape)


# -- differentiable trajectory ---------------------------------------------------------------

class ExpEulerTrajectory(torch.autograd.Function):
    """u(T) after `steps` exponential-Euler steps from u0, differentiable with respect to u0
    and the five parameters (nu, eta, gamma, kappa, zeta).

    Forward: the library's eigenspace steps, with the physical state saved every
    `every` steps (checkpoints).  Backward: for each checkpoint segment, last first, one
    fcgle_vjp_run call recomputes the segment and sweeps the discrete adjoint through it.
    Gradients follow torch's convention for complex inputs of a real loss,
    dL/dRe u + i dL/dIm u.
    """

    @staticmethod
    def forward(ctx, u0, params, problem, steps, every, t0):
        plan = problem.plan_for(tuple(float(p) for p in params.detach().cpu().tolist()))
        u = u0.detach().to(plan.dtype).contiguous().clone()
        plan.set_state(u)
        ckpts = []
        k = 0
        while k < steps:
            m = min(every, steps - k)
            ckpts.append((k, u.clone(), m))
            plan.run("exp_euler", u, t0 + k * plan.tau, m)
            k += m
        ctx.plan = plan
        ctx.ckpts = ckpts
        ctx.t0 = t0
        ctx.params_meta = (params.dtype, params.device)
        ctx.u0_dtype = u0.dtype
        return u

    @staticmethod
    def backward(ctx, grad_u):
        plan = ctx.plan
        ubar = grad_u.detach().to(plan.dtype).contiguous().clone()
        pbar = torch.zeros(5, dtype=torch.float64, device=plan.device)
        for k, uk, m in reversed(ctx.ckpts):
            plan.vjp_run(uk, m, ubar, pbar, ctx.t0 + k * plan.tau)
        dt, dev = ctx.params_meta
        return ubar.to(ctx.u0_dtype), pbar.to(dtype=dt, device=dev), None, None, None, None


class Problem:
    """Grid, orders, time step and precision of a problem whose parameters may vary: keeps
    the plan of the most recent parameter set (setting up a plan costs the FP64
    eigendecompositions and the f-grids).  A plan replaced by one for other parameters is not
    closed here: an autograd graph that ran on it still holds it for its backward pass, and it
    is released with its last reference."""

    def __init__(self, n, alpha, h, tau: float, precision: str = "fp64", fd_order: int = 2):
        self.n, self.alpha, self.h = tuple(n), tuple(alpha), tuple(h)
        self.tau, self.precision, self.fd_order = float(tau), precision, fd_order
        self._plan = None
        self._key = None

    def plan_for(self, params) -> Plan:
        if self._key != params:
            self._plan = None  # dropped, not closed (see the class comment)
            self._plan = Plan(self.n, self.alpha, self.h, params, tau=self.tau, precision=self.precision,
                              fd_order=self.fd_order)
            self._key = params
        return self._plan

    def trajectory(self, u0: torch.Tensor, params: torch.Tensor, steps: int, every: int = 20,
                   t0: float = 0.0) -> torch.Tensor:
        if every < 1:
            raise ValueError("every must be >= 1")
        return ExpEulerTrajectory.apply(u0, params, self, int(steps), int(every), float(t0))

    def close(self):
        if self._plan is not None:
            self._plan.close()
            self._plan = None
            self._key = None
