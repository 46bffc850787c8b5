"""Python binding of the C-ABI (argument marshalling only).

Every step of the simulation and of the gradient runs in the HIP kernels of
``libfwi.so``; PyTorch only provides device memory and the current stream.
Functions take and return torch tensors on the handle's device.
"""

from __future__ import annotations

import ctypes
import math
from typing import Optional, Sequence, Tuple

import numpy as np
import torch

from . import _lib as L


class FwiError(RuntimeError):
    def __init__(self, status: int, where: str):
        lib = L.load()
        msg = lib.fwi_status_string(status).decode()
        detail = lib.fwi_last_error().decode()
        super().__init__(f"{where}: {msg} ({detail})")
        self.status = status


def _check(status: int, where: str) -> None:
    if status != L.FWI_OK:
        raise FwiError(status, where)


def db_to_neper(alpha_db: float, y: float) -> float:
    """Absorption prefactor in dB MHz^-y cm^-1 -> Np (rad/s)^-y m^-1 (the unit
    of alpha0 in fwi_set_absorption): 1 dB = ln(10)/20 Np, omega = 2 pi f."""
    return alpha_db * 100.0 * math.log(10.0) / 20.0 / (2.0 * math.pi * 1.0e6) ** y


def rademacher(seed: int, n: int) -> np.ndarray:
    """Rademacher weights from SplitMix64 (host, bit-exact); int8 [n]."""
    lib = L.load()
    out = np.empty(n, dtype=np.int8)
    _check(lib.fwi_rademacher(ctypes.c_uint64(seed & ((1 << 64) - 1)), n,
                              out.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))), "fwi_rademacher")
    return out


def delays(seed: int, n: int, tau_steps: int) -> np.ndarray:
    """Whole-step delays of delayed source encoding (host, bit-exact); int32 [n]."""
    lib = L.load()
    out = np.empty(n, dtype=np.int32)
    _check(lib.fwi_delays(ctypes.c_uint64(seed & ((1 << 64) - 1)), n, int(tau_steps),
                          out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))), "fwi_delays")
    return out


def _params(shape, dx, dt, nt, c_ref, c_min, c_max, rho0, pml, pml_alpha, precision, batch):
    nz, ny, nx = shape
    p = L.FwiParams()
    p.nx, p.ny, p.nz = int(nx), int(ny), int(nz)
    p.dx, p.dt, p.c_ref = float(dx), float(dt), float(c_ref)
    p.c_min, p.c_max, p.rho0 = float(c_min), float(c_max), float(rho0)
    for a in range(3):
        p.pml[a] = int(pml[a])
    p.pml_alpha = float(pml_alpha)
    p.nt, p.precision, p.batch = int(nt), int(precision), int(batch)
    return p


class _Geometry:
    """Keeps the host arrays alive while the C struct points at them."""

    def __init__(self, src_ijk, rec_ijk, gamma, boundary):
        self.src = np.ascontiguousarray(np.asarray(src_ijk, dtype=np.int32).reshape(-1, 3))
        self.rec = np.ascontiguousarray(np.asarray(rec_ijk, dtype=np.int32).reshape(-1, 3))
        self.gamma = np.ascontiguousarray(np.asarray(gamma, dtype=np.uint8))
        self.boundary = np.ascontiguousarray(np.asarray(boundary, dtype=np.uint8))
        g = L.FwiGeometry()
        g.n_src = self.src.shape[0]
        g.src_ijk = self.src.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        g.n_rec = self.rec.shape[0]
        g.rec_ijk = self.rec.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        g.gamma_mask = self.gamma.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        g.boundary_mask = self.boundary.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        self.c = g


def problem_kwargs(prob, precision: Optional[int] = None, nt: Optional[int] = None) -> dict:
    """Handle arguments from a ``synth.Problem``-like object."""
    return dict(shape=prob.shape, dx=prob.dx, dt=prob.dt, nt=nt or prob.nt, c_ref=prob.c_ref,
                c_min=prob.c_min, c_max=prob.c_max, rho0=prob.rho0, pml=prob.pml,
                pml_alpha=prob.pml_alpha, src_ijk=prob.src_ijk, rec_ijk=prob.rec_ijk,
                gamma=prob.gamma, boundary=prob.boundary,
                precision=precision or prob.precision)


def workspace_bytes(**kw) -> int:
    """Device bytes a handle with these arguments allocates (admission query)."""
    lib = L.load()
    batch = kw.pop("batch", 1)
    geo = _Geometry(kw.pop("src_ijk"), kw.pop("rec_ijk"), kw.pop("gamma"), kw.pop("boundary"))
    p = _params(kw["shape"], kw["dx"], kw["dt"], kw["nt"], kw["c_ref"], kw["c_min"], kw["c_max"],
                kw["rho0"], kw["pml"], kw["pml_alpha"], kw.get("precision", 4), batch)
    return int(lib.fwi_workspace_bytes(ctypes.byref(p), ctypes.byref(geo.c)))


class Handle:
    """One configured grid + geometry + workspace on one device."""

    def __init__(self, *, shape, dx, dt, nt, c_ref, c_min, c_max, rho0, pml, pml_alpha,
                 src_ijk, rec_ijk, gamma, boundary, precision=4, batch=1, device=0):
        self._lib = L.load()
        self._h = ctypes.c_void_p(None)
        # constructor arguments (the autotuner builds a short-horizon twin)
        self.kwargs = dict(shape=shape, dx=dx, dt=dt, nt=nt, c_ref=c_ref, c_min=c_min, c_max=c_max, rho0=rho0,
                           pml=pml, pml_alpha=pml_alpha, src_ijk=src_ijk, rec_ijk=rec_ijk, gamma=gamma,
                           boundary=boundary, precision=precision)
        self.shape = tuple(int(s) for s in shape)
        self.nt = int(nt)
        self.precision = int(precision)
        self.batch = int(batch)
        self.device = torch.device("cuda", device)
        self.dtype = torch.float32 if self.precision == 4 else torch.float64
        geo = _Geometry(src_ijk, rec_ijk, gamma, boundary)
        self.n_src = geo.src.shape[0]
        self.n_rec = geo.rec.shape[0]
        p = _params(shape, dx, dt, nt, c_ref, c_min, c_max, rho0, pml, pml_alpha, precision, batch)
        self.n_cells = self.shape[0] * self.shape[1] * self.shape[2]
        self.tape_token = 0   # bumps whenever a call overwrites the saved tape
        self.use_graph = False
        self.tr_final_state = False   # FWI_TR_FINAL_STATE for gradient / backward
        with torch.cuda.device(self.device):
            _check(self._lib.fwi_create(ctypes.byref(p), ctypes.byref(geo.c), int(device),
                                        ctypes.byref(self._h)), "fwi_create")

    @classmethod
    def from_problem(cls, prob, batch=1, precision=None, nt=None, device=0):
        return cls(**problem_kwargs(prob, precision, nt), batch=batch, device=device)

    def close(self):
        if self._h is not None and self._h.value:
            self._lib.fwi_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------
    def _t(self, x, shape_tail, dtype=None, batch=None):
        """x as a contiguous [B', *shape_tail] tensor on the device.  With
        `batch` given, B' must be 1 or batch, and a leading 1 is expanded to
        batch (one array shared by every problem): the kernels index every
        per-problem array by the problem number, so a shorter array would be
        read out of bounds."""
        dtype = dtype or self.dtype
        t = torch.as_tensor(x, device=self.device, dtype=dtype)
        if t.dim() == len(shape_tail):
            t = t.unsqueeze(0)
        if t.dim() != len(shape_tail) + 1 or tuple(t.shape[1:]) != tuple(shape_tail):
            raise ValueError(f"expected [..., {shape_tail}], got {tuple(t.shape)}")
        if batch is not None and t.shape[0] != batch:
            if t.shape[0] != 1:
                raise ValueError(f"leading dimension {t.shape[0]} is neither 1 nor the batch {batch}")
            t = t.expand(batch, *shape_tail)
        return t.contiguous()

    def _stream(self):
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def forward(self, c, src_sig, w, save_tape=False, check=False):
        """Traces [B, nt, n_rec] of the encoded sources sum_i w_i s_i."""
        c = self._t(c, self.shape)
        B = c.shape[0]
        src = self._t(src_sig, (self.nt, self.n_src), batch=B)
        w = self._t(w, (self.n_src,), torch.int8, batch=B)
        tr = torch.empty((B, self.nt, self.n_rec), device=self.device, dtype=self.dtype)
        flags = (L.FWI_SAVE_TAPE if save_tape else 0) | (L.FWI_CHECK_INPUT if check else 0)
        flags |= L.FWI_GRAPH if self.use_graph else 0
        self.tape_token += 1
        _check(self._lib.fwi_forward(self._h, B, c.data_ptr(), src.data_ptr(), w.data_ptr(),
                                     tr.data_ptr(), flags, self._stream()), "fwi_forward")
        return tr

    def gradient(self, c, src_sig, w, obs, check=False, out=None, mean=False,
                 exact=False) -> Tuple[torch.Tensor, torch.Tensor]:
        """(misfit [B] float64, gradient [B, nz, ny, nx]) of the encoded TR gradient.
        check=True validates c against [c_min, c_max] and the result for
        finiteness (both read a device flag back, so the call synchronises).
        mean=True returns the mean of the B gradients as [1, nz, ny, nx]
        (FWI_MEAN: averaged on the device in a fixed order).  exact=True
        returns the exact discrete gradient instead (FWI_EXACT: reverse mode
        over a stored dp/dc0 history on Gamma; B = 1)."""
        c = self._t(c, self.shape)
        B = c.shape[0]
        src = self._t(src_sig, (self.nt, self.n_src), batch=B)
        w = self._t(w, (self.n_src,), torch.int8, batch=B)
        obs = self._t(obs, (self.nt, self.n_rec), batch=B)
        mis = torch.empty((B,), device=self.device, dtype=torch.float64)
        G = 1 if mean else B
        if out is not None:
            if tuple(out.shape) != (G, *self.shape) or out.dtype != self.dtype or not out.is_contiguous():
                raise ValueError(f"out must be a contiguous [{G}, nz, ny, nx] tensor of the handle's dtype")
            grad = out
        else:
            grad = torch.empty((G, *self.shape), device=self.device, dtype=self.dtype)
        flags = (L.FWI_CHECK_INPUT | L.FWI_CHECK_FINITE if check else 0) | (L.FWI_GRAPH if self.use_graph else 0)
        flags |= L.FWI_TR_FINAL_STATE if self.tr_final_state else 0
        flags |= L.FWI_MEAN if mean else 0
        flags |= L.FWI_EXACT if exact else 0
        self.tape_token += 1
        _check(self._lib.fwi_gradient(self._h, B, c.data_ptr(), src.data_ptr(), w.data_ptr(), obs.data_ptr(),
                                      mis.data_ptr(), grad.data_ptr(), flags, self._stream()), "fwi_gradient")
        return mis, grad

    def backward(self, c, residual, check=False, mean=False) -> Tuple[torch.Tensor, torch.Tensor]:
        """(1/2 ||r||^2 [B], (df/dc)^T r on Gamma) using the tape of the last
        forward(save_tape=True) call with the same batch (FwiError with
        FWI_ERR_NO_TAPE otherwise); check and mean as in gradient()."""
        c = self._t(c, self.shape)
        B = c.shape[0]
        r = self._t(residual, (self.nt, self.n_rec), batch=B)
        mis = torch.empty((B,), device=self.device, dtype=torch.float64)
        grad = torch.empty((1 if mean else B, *self.shape), device=self.device, dtype=self.dtype)
        flags = (L.FWI_GRAPH if self.use_graph else 0) | (L.FWI_TR_FINAL_STATE if self.tr_final_state else 0)
        flags |= (L.FWI_CHECK_INPUT | L.FWI_CHECK_FINITE) if check else 0
        flags |= L.FWI_MEAN if mean else 0
        _check(self._lib.fwi_backward(self._h, B, c.data_ptr(), r.data_ptr(), mis.data_ptr(), grad.data_ptr(),
                                      flags, self._stream()), "fwi_backward")
        return mis, grad

    def derivative(self, field, axis: int, sign: int):
        """Staggered spectral derivative (eq. DisPartDevSt) of one field."""
        f = torch.as_tensor(field, device=self.device, dtype=self.dtype).contiguous()
        if tuple(f.shape) != self.shape:
            raise ValueError("field shape mismatch")
        out = torch.empty_like(f)
        _check(self._lib.fwi_derivative(self._h, f.data_ptr(), out.data_ptr(), int(axis), int(sign),
                                        self._stream()), "fwi_derivative")
        return out

    # ------------------------------------------------------------------
    TUNING_FIELDS = ("y_tile_bytes", "zm_tile_bytes", "zp_tile_bytes", "y_plan", "zm_plan", "zp_plan", "x_plan")

    @property
    def tuning(self) -> dict:
        """Launch tuning: tile row segments {'y_tile_bytes', 'zm_tile_bytes',
        'zp_tile_bytes'} (64 or 128) and radix plans {'y_plan', 'zm_plan',
        'zp_plan', 'x_plan'} (0 or 1) of the pass kinds (fwi_tuning)."""
        t = L.FwiTuning()
        _check(self._lib.fwi_get_tuning(self._h, ctypes.byref(t)), "fwi_get_tuning")
        return {f: int(getattr(t, f)) for f in self.TUNING_FIELDS}

    @tuning.setter
    def tuning(self, value: dict) -> None:
        cur = self.tuning
        cur.update(value)
        t = L.FwiTuning(*(int(cur[f]) for f in self.TUNING_FIELDS))
        _check(self._lib.fwi_set_tuning(self._h, ctypes.byref(t)), "fwi_set_tuning")

    def set_absorption(self, alpha0=0.0, y=1.5, field=None, tr_flip=True) -> None:
        """Power-law absorption (Sec. 2.1): alpha0 in Np (rad/s)^-y m^-1, either a
        number or a per-voxel field [nz, ny, nx] (kept on the device by the handle
        for as long as absorption is set); alpha0 = 0 with no field switches it
        off.  tr_flip: the TR simulation switches the sign of tau (Sec. 3.1)."""
        ptr, f = None, None
        if field is not None:
            f = self._t(field, self.shape)[0].contiguous()
            ptr = ctypes.c_void_p(f.data_ptr())
        torch.cuda.synchronize(self.device)
        _check(self._lib.fwi_set_absorption(self._h, float(alpha0), float(y), ptr, 1 if tr_flip else 0),
               "fwi_set_absorption")
        # the library now reads this field (or none): keep it alive; on an
        # error above the previous field stays in use and stays referenced
        self._alpha0_field = f
        self.tape_token += 1

    def set_delays(self, delays=None) -> None:
        """Delayed source encoding (eq. DelaySE): delays [B, n_src] (or [n_src]
        for B = 1) in whole steps, each in [0, nt); None switches delays off.
        The library shifts the injected signals; signals stay unshifted."""
        if delays is None:
            _check(self._lib.fwi_set_delays(self._h, 0, None), "fwi_set_delays")
            return
        d = np.ascontiguousarray(np.asarray(delays, dtype=np.int32))
        if d.ndim == 1:
            d = d[None, :]
        if d.ndim != 2 or d.shape[1] != self.n_src:
            raise ValueError(f"expected delays [B, {self.n_src}], got {d.shape}")
        _check(self._lib.fwi_set_delays(self._h, int(d.shape[0]), d.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))),
               "fwi_set_delays")

    def timing_enable(self, every: int) -> None:
        """Sample every `every`-th time step's pass launches with HIP events."""
        _check(self._lib.fwi_timing_enable(self._h, int(every)), "fwi_timing_enable")

    def timing_read(self) -> dict:
        """{pass name: (sampled launches, total ms, total algorithmic bytes)}; resets."""
        out = {}
        for k, name in enumerate(L.PASS_NAMES):
            n = ctypes.c_int64()
            ms = ctypes.c_double()
            by = ctypes.c_double()
            _check(self._lib.fwi_timing_read(self._h, k, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by)),
                   "fwi_timing_read")
            out[name] = (int(n.value), float(ms.value), float(by.value))
        return out
