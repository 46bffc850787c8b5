"""Stochastic L-BFGS outer loop (App. D, Algorithm 2) on the device.

The unknown u lives on Gamma (a Gamma-compact device vector): either c0
itself or the squared slowness u = 1/c0^2 (Sec. 2.4; the preconditioning
the paper keeps, Sec. 4.6).  The estimator g(u, i) is the encoded TR
gradient of Alg. 1 (fwi_gradient) whose encoding is fixed by the iteration
index i, so that the two evaluations of an iteration share it (App. D).
Every vector operation — the two-loop recursion and the history (fwi_lbfgs_*),
axpby, projection, the parametrisation and the grid <-> Gamma copies
(fwi_vec_*, fwi_gamma_*) — runs in the library; this module only sequences
those calls and keeps the scalars (energies, weights) on the host.

    est = EncodedEstimator(handle, c_background, src_signals, observed, seed0=100)
    u0 = est.u_from_c(c_start)
    u_hat, J = slbfgs(est, u0, nu=1.0, h0=h0, n_evals=16, u_min=..., u_max=...)
"""

from __future__ import annotations

import ctypes
import math
from typing import Callable, List, Optional, Tuple

import torch

from . import _lib as L
from .fwi import FwiError, Handle, _check, rademacher


def _ptr(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


class VecOps:
    """The library's vector primitives on tensors of one dtype and device."""

    def __init__(self, device: torch.device, dtype: torch.dtype):
        self.lib = L.load()
        self.device = device
        self.dtype = dtype
        self.prec = 4 if dtype == torch.float32 else 8

    def _st(self):
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def axpby(self, a: float, x: Optional[torch.Tensor], b: float, y: torch.Tensor) -> torch.Tensor:
        """y <- a x + b y (in place)."""
        _check(self.lib.fwi_vec_axpby(y.numel(), float(a), _ptr(x) if x is not None else None, float(b), _ptr(y),
                                      self.prec, self._st()), "fwi_vec_axpby")
        return y

    def copy(self, x: torch.Tensor, y: torch.Tensor) -> torch.Tensor:
        return self.axpby(1.0, x, 0.0, y)

    def clip(self, x: torch.Tensor, lo: float, hi: float) -> torch.Tensor:
        _check(self.lib.fwi_vec_clip(x.numel(), _ptr(x), float(lo), float(hi), self.prec, self._st()), "fwi_vec_clip")
        return x

    def sqslowness(self, mode: int, x: torch.Tensor, out: torch.Tensor, aux: Optional[torch.Tensor] = None):
        _check(self.lib.fwi_vec_sqslowness(x.numel(), int(mode), _ptr(x), _ptr(aux) if aux is not None else None,
                                           _ptr(out), self.prec, self._st()), "fwi_vec_sqslowness")
        return out


class LbfgsHistory:
    """Device L-BFGS history of at most m pairs (fwi_lbfgs_*)."""

    def __init__(self, n: int, m: int, ops: VecOps):
        self.ops = ops
        self._h = ctypes.c_void_p(None)
        _check(ops.lib.fwi_lbfgs_create(int(n), int(m), ops.prec, ops.device.index or 0, ctypes.byref(self._h)),
               "fwi_lbfgs_create")

    def push(self, s: torch.Tensor, y: torch.Tensor) -> None:
        _check(self.ops.lib.fwi_lbfgs_push(self._h, _ptr(s), _ptr(y), self.ops._st()), "fwi_lbfgs_push")

    def apply(self, g: torch.Tensor, r: torch.Tensor, h0: float) -> torch.Tensor:
        """r <- H g."""
        _check(self.ops.lib.fwi_lbfgs_apply(self._h, _ptr(g), _ptr(r), float(h0), self.ops._st()), "fwi_lbfgs_apply")
        return r

    def apply_noalloc(self, g: torch.Tensor, r: torch.Tensor, h0: float) -> torch.Tensor:
        """r <- H g through fwi_lbfgs_apply_noalloc (no device allocation; the
        library's static scratch, shared by every such call on the device)."""
        _check(self.ops.lib.fwi_lbfgs_apply_noalloc(self._h, _ptr(g), _ptr(r), float(h0), self.ops._st()),
               "fwi_lbfgs_apply_noalloc")
        return r

    def count(self) -> int:
        c = ctypes.c_int32()
        _check(self.ops.lib.fwi_lbfgs_count(self._h, ctypes.byref(c)), "fwi_lbfgs_count")
        return int(c.value)

    def close(self) -> None:
        if self._h is not None and self._h.value:
            self.ops.lib.fwi_lbfgs_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class EncodedEstimator:
    """g(u, i) = (D, dD/du on Gamma) of the Rademacher-encoded TR gradient with
    weights SplitMix64(seed0 + i) (Sec. 3.2).  `observed(w)` returns the
    encoded observed data sum_i w_i f_i^delta [nt, n_rec] on the device (the
    caller's data; for synthetic data a forward at the true medium gives it by
    linearity).  Outside Gamma c0 stays c_background.  param = 'sqslowness'
    (u = 1/c0^2) or 'speed' (u = c0)."""

    def __init__(self, handle: Handle, c_background, src_signals, observed: Callable, seed0: int = 0,
                 param: str = "sqslowness"):
        if param not in ("sqslowness", "speed"):
            raise ValueError(param)
        self.h = handle
        self.param = param
        self.seed0 = int(seed0)
        self.observed = observed
        dev, dt = handle.device, handle.dtype
        self.ops = VecOps(dev, dt)
        n = ctypes.c_int64()
        _check(handle._lib.fwi_gamma_size(handle._h, ctypes.byref(n)), "fwi_gamma_size")
        self.n = int(n.value)
        self.c_work = torch.as_tensor(c_background, device=dev, dtype=dt).reshape(handle.shape).contiguous().clone()
        self.src = torch.as_tensor(src_signals, device=dev, dtype=dt).contiguous()
        self.grad = torch.empty((1, *handle.shape), device=dev, dtype=dt)
        self.c_gam = torch.empty(self.n, device=dev, dtype=dt)
        self.g_c = torch.empty(self.n, device=dev, dtype=dt)
        self.evals = 0

    def empty(self) -> torch.Tensor:
        return torch.empty(self.n, device=self.h.device, dtype=self.h.dtype)

    def gather(self, full: torch.Tensor, compact: torch.Tensor) -> torch.Tensor:
        _check(self.h._lib.fwi_gamma_gather(self.h._h, _ptr(full), _ptr(compact), self.ops._st()), "fwi_gamma_gather")
        return compact

    def scatter(self, compact: torch.Tensor, full: torch.Tensor) -> torch.Tensor:
        _check(self.h._lib.fwi_gamma_scatter(self.h._h, _ptr(compact), _ptr(full), self.ops._st()),
               "fwi_gamma_scatter")
        return full

    def u_from_c(self, c_full) -> torch.Tensor:
        """The unknown of a full-grid speed field."""
        c = torch.as_tensor(c_full, device=self.h.device, dtype=self.h.dtype).reshape(self.h.shape).contiguous()
        u = self.gather(c, self.empty())
        return self.ops.sqslowness(0, u, u) if self.param == "sqslowness" else u

    def c_from_u(self, u: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """c0 on Gamma of an unknown vector."""
        out = out if out is not None else self.empty()
        return self.ops.sqslowness(1, u, out) if self.param == "sqslowness" else self.ops.copy(u, out)

    def bounds(self, c_min: float, c_max: float) -> Tuple[float, float]:
        """Bounds on u of the speed bounds (the projection of Alg. 2)."""
        if self.param == "sqslowness":
            return 1.0 / (c_max * c_max), 1.0 / (c_min * c_min)
        return c_min, c_max

    def __call__(self, u: torch.Tensor, i: int, G: torch.Tensor) -> float:
        """Evaluate at u with the encoding of iteration i; G <- dD/du; returns D."""
        w = torch.from_numpy(rademacher(self.seed0 + i, self.h.n_src)).to(self.h.device)
        obs = self.observed(w)
        self.c_from_u(u, self.c_gam)
        self.scatter(self.c_gam, self.c_work)
        mis, _ = self.h.gradient(self.c_work, self.src, w, obs, out=self.grad)
        self.gather(self.grad, self.g_c)
        if self.param == "sqslowness":
            self.ops.sqslowness(2, self.g_c, G, aux=self.c_gam)
        else:
            self.ops.copy(self.g_c, G)
        self.evals += 1
        return float(mis[0])


class _StepBuffers:
    """Device vectors one quasi-Newton step works in."""

    def __init__(self, est: EncodedEstimator):
        self.d, self.trial, self.s, self.y = est.empty(), est.empty(), est.empty(), est.empty()
        self.G_u, self.G_trial, self.r = est.empty(), est.empty(), est.empty()


def quasi_newton_step(est: EncodedEstimator, u: torch.Tensor, i: int, hist: LbfgsHistory, nu: float, h0: float,
                      buf: _StepBuffers) -> float:
    """One stochastic quasi-Newton step of length nu with the encoding of
    iteration i (App. D), in place on u: the direction d = -H G at u, the
    estimator at the trial point u + nu d, the pair (nu d, G_trial - G) pushed
    to the history, the direction corrected by -H G_trial with the updated
    history, u <- u + nu d.  Returns the energy estimate, the smaller of the
    two misfits.  Both estimator calls use encoding i, so the pair is
    consistent."""
    ops = est.ops
    F_u = est(u, i, buf.G_u)
    hist.apply(buf.G_u, buf.d, h0)
    ops.axpby(0.0, None, -1.0, buf.d)                 # d = -H G_u
    ops.copy(u, buf.trial)
    ops.axpby(nu, buf.d, 1.0, buf.trial)              # trial point u + nu d
    F_trial = est(buf.trial, i, buf.G_trial)
    ops.axpby(nu, buf.d, 0.0, buf.s)                  # s = nu d
    ops.copy(buf.G_trial, buf.y)
    ops.axpby(-1.0, buf.G_u, 1.0, buf.y)              # y = G_trial - G_u
    hist.push(buf.s, buf.y)
    hist.apply(buf.G_trial, buf.r, h0)
    ops.axpby(-1.0, buf.r, 1.0, buf.d)                # d = d - H G_trial
    ops.axpby(nu, buf.d, 1.0, u)
    return min(F_u, F_trial)


class IterateAverage:
    """The returned estimate (App. D): the iterate itself until the energy
    estimate first increases, then the w(i)-weighted mean of the iterates of
    the following steps, accumulated on the device."""

    def __init__(self, est: EncodedEstimator, weight: Callable[[int], float]):
        self.ops = est.ops
        self.weight = weight
        self.on = False
        self.total = self.ops.axpby(0.0, None, 0.0, est.empty())
        self.wsum = 0.0
        self.J_last = math.inf
        self.estimate = est.empty()

    def update(self, i: int, u: torch.Tensor, J: float) -> torch.Tensor:
        if self.on:
            wi = self.weight(i)
            self.ops.axpby(wi, u, 1.0, self.total)
            self.wsum += wi
            self.ops.axpby(1.0 / self.wsum, self.total, 0.0, self.estimate)
        else:
            self.on = J > self.J_last
            self.ops.copy(u, self.estimate)
        self.J_last = J
        return self.estimate


def slbfgs(est: EncodedEstimator, u0: torch.Tensor, *, nu: float, n_evals: int, m_h: int = 64, h0: float = 1.0,
           u_min: float = -math.inf, u_max: float = math.inf, weight: Callable[[int], float] = lambda i: float(i) ** 3,
           callback: Optional[Callable] = None) -> Tuple[torch.Tensor, List[float]]:
    """Algorithm 2 without line search: quasi-Newton steps i = 1, 2, ... until
    n_evals estimator calls (two per step) are spent, each followed by the
    projection onto [u_min, u_max] and the iterate averaging.  Returns
    (u_hat, energy estimates J_i); callback(i, u_hat, J_i) after every step."""
    ops = est.ops
    hist = LbfgsHistory(u0.numel(), m_h, ops)
    u = ops.copy(u0, est.empty())
    buf = _StepBuffers(est)
    average = IterateAverage(est, weight)
    u_hat = ops.copy(u, est.empty())
    Js: List[float] = []
    i = 0
    try:
        while 2 * i < n_evals:
            i += 1
            J = quasi_newton_step(est, u, i, hist, nu, h0, buf)
            ops.clip(u, u_min, u_max)
            u_hat = average.update(i, u, J)
            Js.append(J)
            if callback is not None:
                callback(i, u_hat, J)
    finally:
        hist.close()
    return u_hat, Js
