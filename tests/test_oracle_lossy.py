"""Pins of the lossy FP64 oracle (power-law absorption, Sec. 2.1) against
facts that do not come from the oracle: the lossless scheme it must reduce
to, the power law alpha0 omega^y and the dispersion that the fractional
Laplacian model implies (Kramers-Kronig pair of the power law), the inverse
decay of the time-reversed (gain) step, central finite differences of the
discrete misfit, and the order in alpha0 of what the Alg. 1 form omits.
"""

import math

import numpy as np
import pytest

from oracle import kspace as ks
from oracle import lossy as lo
from synth import configs as sc


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def _small(periodic=False):
    prob = sc.make_small(shape=(12, 14, 16), periodic=periodic, pml=2, nt=36, n_src=2, n_rec=6, layer=2)
    return prob, ks.scheme_for(prob), prob.src_signals(), np.array([1.0, -1.0])


def test_db_conversion():
    # 1 dB = ln(10) / 20 Np; at 1 MHz (omega = 2 pi 1e6) alpha0 omega^y gives
    # back the dB figure per cm
    a0 = lo.db_to_neper(0.75, 1.5)
    assert abs(a0 * (2 * math.pi * 1e6) ** 1.5 / 100.0 - 0.75 * math.log(10) / 20) < 1e-15


def test_zero_absorption_is_the_lossless_scheme():
    # Sec. 2.1: L = 0 gives eq. PreDenRel without loss; the lossy step must
    # then be the lossless one, to the last bit
    prob, sch, S, w = _small()
    los = lo.Lossy(sch, 0.0, 1.5)
    t0 = ks.forward(sch, prob.c_true, prob.src_ijk, S, w, prob.rec_ijk, prob.nt)["traces"]
    t1 = lo.forward(los, prob.c_true, prob.src_ijk, S, w, prob.rec_ijk, prob.nt)["traces"]
    assert np.array_equal(t0, t1)
    D0, G0, _ = ks.tr_gradient(sch, prob.c_eval, prob.src_ijk, S, w, prob.rec_ijk, t0 * 0.9, prob.gamma,
                               prob.boundary, prob.nt)
    D1, G1, _ = lo.tr_gradient(los, prob.c_eval, prob.src_ijk, S, w, prob.rec_ijk, t0 * 0.9, prob.gamma,
                               prob.boundary, prob.nt)
    assert D0 == D1 and np.array_equal(G0, G1)


def _wave(los, c0, m, sign=1.0):
    lam = lo.wave_eigenvalue(lo.mode_matrix(los, c0, m, sign))
    dt = los.sch.dt
    k = 2 * math.pi * m / (los.sch.shape[2] * los.sch.dx)
    omega = math.atan2(lam.imag, lam.real) / dt
    return lam, k, omega


@pytest.mark.parametrize("y", [0.6, 1.5])
def test_plane_wave_decays_with_the_power_law(y):
    # Sec. 2.1: the tau term of L gives the absorption alpha(omega) =
    # alpha0 omega^y (temporal decay alpha0 c0 omega^y); small dt so that the
    # time discretisation of the loss term stays below the tolerance
    dx, c0 = 0.5e-3, 1500.0
    sch = ks.Scheme((2, 2, 64), dx, 0.05 * dx / c0, c0, 1000.0)
    los = lo.Lossy(sch, lo.db_to_neper(0.75, y), y)
    for m in (4, 8, 16):
        lam, k, omega = _wave(los, c0, m)
        gamma = -math.log(abs(lam)) / sch.dt
        assert abs(gamma / (los.alpha0[0, 0, 0] * c0 * omega ** y) - 1.0) < 0.02


@pytest.mark.parametrize("y", [0.6, 1.5])
def test_phase_speed_follows_the_dispersion_relation(y):
    # Sec. 2.1: the eta term gives 1/c(omega) = 1/c0 + alpha0 tan(pi y/2)
    # omega^{y-1} to first order (the Kramers-Kronig partner of the power law)
    dx, c0 = 0.5e-3, 1500.0
    sch = ks.Scheme((2, 2, 64), dx, 0.05 * dx / c0, c0, 1000.0)
    los = lo.Lossy(sch, lo.db_to_neper(0.75, y), y)
    a0 = los.alpha0[0, 0, 0]
    for m in (4, 8, 16):
        _, k, omega = _wave(los, c0, m)
        want = -c0 * c0 * a0 * math.tan(math.pi * y / 2) * omega ** (y - 1)
        assert abs((omega / k - c0) / want - 1.0) < 0.06


def test_flipped_tau_inverts_the_decay():
    # Sec. 3.1: time reversal in absorbing media switches the sign of the
    # absorption; per step the gain of the flipped step undoes the loss
    dx, c0 = 0.5e-3, 1500.0
    sch = ks.Scheme((2, 2, 64), dx, 0.3 * dx / c0, c0, 1000.0)
    los = lo.Lossy(sch, lo.db_to_neper(0.75, 1.5), 1.5)
    for m in (4, 8, 16):
        lp, _, _ = _wave(los, c0, m, 1.0)
        lm, _, _ = _wave(los, c0, m, -1.0)
        assert abs(lp) < 1.0 < abs(lm)
        assert abs(math.log(abs(lp)) + math.log(abs(lm))) < 0.01 * abs(math.log(abs(lp)))


def test_exact_lossy_gradient_matches_central_finite_differences():
    # App. A: with absorption dD/dc0 gains the terms of dL/dc0; the reverse-
    # mode gradient of the discrete lossy loop must match central differences
    prob, sch, S, w = _small()
    los = lo.Lossy(sch, 20 * lo.db_to_neper(0.75, 1.5), 1.5)
    obs = lo.forward(los, prob.c_true, prob.src_ijk, S, w, prob.rec_ijk, prob.nt)["traces"]
    _, G, _ = lo.exact_adjoint_gradient(los, prob.c_eval, prob.src_ijk, S, w, prob.rec_ijk, obs, prob.nt)
    gi = np.argwhere(prob.gamma)
    rng = np.random.default_rng(9)
    h = 1e-3
    for t in rng.choice(len(gi), size=3, replace=False):
        iz, iy, ix = gi[t]
        cp = prob.c_eval.copy()
        cm = prob.c_eval.copy()
        cp[iz, iy, ix] += h
        cm[iz, iy, ix] -= h
        Dp = ks.misfit_and_adjoint_source(
            lo.forward(los, cp, prob.src_ijk, S, w, prob.rec_ijk, prob.nt)["traces"], obs)[0]
        Dm = ks.misfit_and_adjoint_source(
            lo.forward(los, cm, prob.src_ijk, S, w, prob.rec_ijk, prob.nt)["traces"], obs)[0]
        fd = (Dp - Dm) / (2 * h)
        assert abs(fd - G[iz, iy, ix]) <= 1e-6 * abs(G[iz, iy, ix])


def test_alg1_form_omits_a_first_order_term_in_alpha0():
    # Without PML the lossless Alg. 1 formula is the exact gradient (pinned in
    # the lossless file); with absorption it leaves out the dL/dc0 terms, an
    # error that must vanish linearly with alpha0
    prob, sch, S, w = _small(periodic=True)
    g = prob.gamma.astype(bool)
    errs = []
    for mul in (1.0, 4.0):
        los = lo.Lossy(sch, mul * lo.db_to_neper(0.75, 1.5), 1.5)
        obs = lo.forward(los, prob.c_true, prob.src_ijk, S, w, prob.rec_ijk, prob.nt)["traces"]
        _, Gx, _ = lo.exact_adjoint_gradient(los, prob.c_eval, prob.src_ijk, S, w, prob.rec_ijk, obs, prob.nt)
        _, Gf, _ = lo.full_gradient(los, prob.c_eval, prob.src_ijk, S, w, prob.rec_ijk, obs, prob.gamma,
                                    prob.nt)
        errs.append(rel(Gf[g], Gx[g]))
    assert errs[0] < 5e-3
    assert 3.0 < errs[1] / errs[0] < 5.0
