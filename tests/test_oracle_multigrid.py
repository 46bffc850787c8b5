"""Pins of the oracle's grid transfers (Sec. 2.4, App. C).

Fourier interpolation reproduces band-limited analytic fields exactly (odd
and even coarse sizes, the even Nyquist bin split into the band-limited
cosine), the Blackman smoothing scales every Fourier mode by its window value
and keeps constants, and the Kaiser-windowed sinc resampling passes a
sinusoid below the cut-off and removes one above it (closed forms).
"""

import numpy as np
import pytest

from oracle import multigrid as mg


def _field(shape, modes):
    axes = [np.arange(n) / n for n in shape]
    X = np.meshgrid(*axes, indexing="ij")
    out = np.full(shape, 1.3)
    for amp, k in modes:
        out = out + amp * np.prod([np.cos(2 * np.pi * kk * X[a] + 0.3 * a) for a, kk in enumerate(k)], axis=0)
    return out


@pytest.mark.parametrize("shape_c,shape_f", [((12, 12, 16), (24, 24, 32)), ((9, 10, 8), (16, 20, 12))])
def test_fourier_interpolation_is_exact_for_band_limited_fields(shape_c, shape_f):
    modes = [(1.0, (2, 0, 1)), (0.5, (1, 3, 2)), (0.2, (3, 1, 0))]   # below every coarse Nyquist
    got = mg.interp_up(_field(shape_c, modes), shape_f, window="none")
    assert np.abs(got - _field(shape_f, modes)).max() < 1e-12


def test_even_nyquist_is_split_into_the_cosine():
    n_c, n_f = 8, 16
    u_c = np.cos(np.pi * np.arange(n_c))[:, None, None] * np.ones((1, 4, 4))      # (-1)^i
    got = mg.interp_up(u_c, (n_f, 4, 4), window="none")
    x = np.arange(n_f) / n_f
    want = np.cos(2 * np.pi * (n_c / 2) * x)[:, None, None] * np.ones((1, 4, 4))
    assert np.abs(got - want).max() < 1e-12


def test_blackman_scales_each_mode_by_its_window_value():
    n_c, n_f = 16, 32
    for k in (0, 1, 3, 6):
        x_c = np.arange(n_c) / n_c
        x_f = np.arange(n_f) / n_f
        u_c = np.cos(2 * np.pi * k * x_c)[None, :, None] * np.ones((4, 1, 4))
        got = mg.interp_up(u_c, (4, n_f, 4), window="blackman")
        w = 0.42 + 0.5 * np.cos(np.pi * k / (n_c / 2)) + 0.08 * np.cos(2 * np.pi * k / (n_c / 2))
        want = w * np.cos(2 * np.pi * k * x_f)[None, :, None] * np.ones((4, 1, 4))
        assert np.abs(got - want).max() < 1e-12, k
    assert mg.blackman_k(np.array([8.0]), 8.0)[0] == pytest.approx(0.0, abs=1e-15)   # Nyquist removed


def test_windowed_sinc_resampling_passes_band_and_stops_above_cutoff():
    n_in, dt_in, dt_out, n_out = 400, 1.0, 2.0, 200
    t = np.arange(n_in) * dt_in
    tm = np.arange(n_out) * dt_out
    inner = (tm > 30) & (tm < n_in * dt_in - 30)
    for f0, passes in ((0.02, True), (0.05, True), (0.1, True), (0.3, False), (0.4, False)):
        out = mg.resample_time(np.cos(2 * np.pi * f0 * t)[:, None], dt_in, dt_out, n_out, f_cut=0.2, beta=8.0,
                               T_w=24.0)[:, 0]
        if passes:
            assert np.abs(out[inner] - np.cos(2 * np.pi * f0 * tm[inner])).max() < 1e-4, f0
        else:
            assert np.abs(out[inner]).max() < 1e-4, f0
    # scaling and linearity across channels
    f = np.stack([np.sin(2 * np.pi * 0.03 * t), np.cos(2 * np.pi * 0.07 * t)], axis=1)
    a = mg.resample_time(f, dt_in, dt_out, n_out, 0.2, 8.0, 24.0, scale=4.0)
    b = mg.resample_time(f, dt_in, dt_out, n_out, 0.2, 8.0, 24.0)
    assert np.allclose(a, 4.0 * b, rtol=1e-14, atol=0)
    assert mg.kaiser_w(np.array([0.0]), 24.0, 8.0)[0] == 1.0
    assert mg.kaiser_w(np.array([24.5]), 24.0, 8.0)[0] == 0.0
