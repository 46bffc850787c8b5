"""Grid transfers of the coarse-to-fine scheme (Sec. 2.4, App. C).

* interp_up(coarse, fine, u): Fourier interpolation of a coarse-grid field to
  a finer grid of the same box with Blackman smoothing (fwi_interp_fourier);
  the initialisation of the next level from a coarse solution.
* resample_time(f, ...): band-limited resampling of source and data time
  series to the coarse time step with a Kaiser-windowed low-pass
  (fwi_resample_time); data are scaled by eta^(d-1) (App. C).
* coarse_level(...): the time step, sample count and cut-off of a level
  coarsened by eta in space and time.

The arithmetic runs in the library; this module marshals tensors.
"""

from __future__ import annotations

import ctypes
import math
from typing import Optional

import torch

from . import _lib as L
from .fwi import Handle, _check


def interp_up(coarse: Handle, fine: Handle, u, window: str = "blackman") -> torch.Tensor:
    """Field on the fine handle's grid from `u` on the coarse handle's grid."""
    if window not in ("blackman", "none"):
        raise ValueError(window)
    u = torch.as_tensor(u, device=coarse.device, dtype=coarse.dtype).reshape(coarse.shape).contiguous()
    out = torch.empty(fine.shape, device=fine.device, dtype=fine.dtype)
    st = ctypes.c_void_p(torch.cuda.current_stream(fine.device).cuda_stream)
    _check(L.load().fwi_interp_fourier(coarse._h, fine._h, ctypes.c_void_p(u.data_ptr()),
                                       ctypes.c_void_p(out.data_ptr()), 1 if window == "blackman" else 0, st),
           "fwi_interp_fourier")
    return out


def coarse_cutoff(c_min: float, dx_coarse: float, ppw: float = 3.0) -> float:
    """Highest frequency a grid of spacing dx_coarse carries with ppw points per
    wavelength in the slowest medium (ppw = 3)."""
    return c_min / (ppw * dx_coarse)


def resample_time(f, dt_in: float, dt_out: float, nt_out: int, f_cut: float, beta: float = 8.0,
                  t_window: Optional[float] = None, scale: float = 1.0) -> torch.Tensor:
    """f [nt_in, channels] (device tensor, float or double) resampled to
    [nt_out, channels] at dt_out with a Kaiser-windowed sinc low-pass at
    f_cut.  t_window defaults to 12 output steps."""
    if not torch.is_tensor(f) or not f.is_cuda:
        raise ValueError("f must be a device tensor")
    f = f.contiguous()
    if f.dim() == 1:
        f = f[:, None]
    prec = 4 if f.dtype == torch.float32 else 8
    tw = t_window if t_window is not None else 12.0 * dt_out
    out = torch.empty((nt_out, f.shape[1]), device=f.device, dtype=f.dtype)
    st = ctypes.c_void_p(torch.cuda.current_stream(f.device).cuda_stream)
    _check(L.load().fwi_resample_time(f.shape[0], f.shape[1], ctypes.c_void_p(f.data_ptr()), float(dt_in),
                                      int(nt_out), float(dt_out), float(f_cut), float(beta), float(tw), float(scale),
                                      ctypes.c_void_p(out.data_ptr()), prec, st), "fwi_resample_time")
    return out


def coarse_level(dt_fine: float, nt_fine: int, eta: float) -> tuple:
    """(dt, nt) of a level coarsened by eta in time covering the same duration."""
    dt = dt_fine * eta
    return dt, int(math.ceil(nt_fine * dt_fine / dt))


def data_scale(eta: float, d: int = 3) -> float:
    """Scale of coarse-level data (App. C): eta^(d-1)."""
    return float(eta) ** (d - 1)
