"""Grid transfers of the coarse-to-fine scheme (Sec. 2.4, App. C) — NumPy.

TEST INFRASTRUCTURE, NOT PRODUCT CODE (see oracle/__init__.py).

Fields of the k-space scheme are band-limited interpolants of their samples
(App. C), so a coarse-grid field is carried to a finer grid of the same box
by Fourier interpolation: its DFT is embedded into the finer frequency grid
(zeros elsewhere) and transformed back, scaled by N_fine / N_coarse.  The
coarse grid's Nyquist bin of an even axis has no sign; without a window it
is split in halves over +-N/2 (the band-limited cosine interpolant).  The
smoothing of App. C multiplies by a separable Blackman window over the
coarse band, w(k) = 0.42 + 0.5 cos(pi k / K) + 0.08 cos(2 pi k / K) with
K = N_coarse / 2 the coarse Nyquist index per axis (reading: the paper names
the window only); w(K) = 0 removes the Nyquist bin.

Time series (sources and data) are carried to a coarser time step by
band-limited resampling with a low-pass cut-off, the Kaiser-windowed sinc
(reading of "Fourier interpolation and low-pass filtering with a Kaiser
window"):
    f_out[m] = scale * sum_n f_in[n] * 2 f_c dt_in * sinc(2 f_c (t_m - t_n))
                                     * I0(beta sqrt(1 - (tau / T_w)^2)) / I0(beta)
with tau = t_m - t_n, the window zero for |tau| > T_w, t_m = m dt_out,
t_n = n dt_in.  Data get scale = eta^(d-1) (App. C), sources scale = 1.
"""

from __future__ import annotations

import numpy as np


def blackman_k(k: np.ndarray, K: float) -> np.ndarray:
    """Blackman window over signed frequency indices k, zero beyond |k| = K."""
    a = np.abs(k) / K
    w = 0.42 + 0.5 * np.cos(np.pi * a) + 0.08 * np.cos(2 * np.pi * a)
    return np.where(a <= 1.0, w, 0.0)


def _embed_axis(X: np.ndarray, axis: int, n_f: int) -> np.ndarray:
    """Embed the DFT along `axis` (length n_c) into length n_f >= n_c."""
    n_c = X.shape[axis]
    shape = list(X.shape)
    shape[axis] = n_f
    Y = np.zeros(shape, dtype=np.complex128)
    for i in range(n_c):
        k = i if i < (n_c + 1) // 2 else i - n_c        # signed frequency
        src = np.take(X, i, axis=axis)
        if n_c % 2 == 0 and abs(k) == n_c // 2 and n_f > n_c:
            # Nyquist of an even coarse axis: half to +N/2 and half to -N/2
            for kk in (n_c // 2, -n_c // 2):
                idx = [slice(None)] * X.ndim
                idx[axis] = kk % n_f
                Y[tuple(idx)] += 0.5 * src
        else:
            idx = [slice(None)] * X.ndim
            idx[axis] = k % n_f
            Y[tuple(idx)] += src
    return Y


def interp_up(u_c: np.ndarray, shape_f, window: str = "blackman") -> np.ndarray:
    """Fourier interpolation of u_c onto a grid of shape shape_f covering the
    same box (each fine size >= the coarse one); window 'blackman' or 'none'."""
    u_c = np.asarray(u_c, dtype=np.float64)
    X = np.fft.fftn(u_c)
    if window == "blackman":
        for ax, n in enumerate(u_c.shape):
            k = np.fft.fftfreq(n) * n
            shp = [1] * u_c.ndim
            shp[ax] = n
            X = X * blackman_k(k, n / 2.0).reshape(shp)
    elif window != "none":
        raise ValueError(window)
    for ax, n_f in enumerate(shape_f):
        X = _embed_axis(X, ax, int(n_f))
    scale = float(np.prod(shape_f)) / float(np.prod(u_c.shape))
    return np.real(np.fft.ifftn(X)) * scale


def kaiser_w(tau: np.ndarray, T_w: float, beta: float) -> np.ndarray:
    x = np.clip(1.0 - (np.asarray(tau) / T_w) ** 2, 0.0, None)
    return np.where(np.abs(tau) <= T_w, np.i0(beta * np.sqrt(x)) / np.i0(beta), 0.0)


def resample_time(f: np.ndarray, dt_in: float, dt_out: float, n_out: int, f_cut: float, beta: float,
                  T_w: float, scale: float = 1.0) -> np.ndarray:
    """Kaiser-windowed sinc resampling of f [n_in, channels] to n_out samples
    at dt_out with cut-off f_cut (written as the plain double sum)."""
    f = np.asarray(f, dtype=np.float64)
    n_in = f.shape[0]
    t_in = np.arange(n_in) * dt_in
    out = np.zeros((n_out,) + f.shape[1:])
    for m in range(n_out):
        tau = m * dt_out - t_in
        h = 2 * f_cut * dt_in * np.sinc(2 * f_cut * tau) * kaiser_w(tau, T_w, beta)
        out[m] = scale * np.tensordot(h, f, axes=(0, 0))
    return out


def coarse_cutoff(c_min: float, dx_coarse: float, ppw: float = 3.0) -> float:
    """Highest frequency the coarse grid carries with ppw points per
    wavelength in the slowest medium (reading: ppw = 3)."""
    return c_min / (ppw * dx_coarse)
