"""Plain FP64 oracle of the lossy model: power-law absorption and dispersion.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Slow on purpose: every
fractional Laplacian is a full complex 3D FFT, a multiplication and a full
inverse FFT.

What is computed (Sec. 2.1, eq. PreDenRel and the definition of L; Sec. 3.1 on
time reversal in absorbing media; App. A, the c0-derivative of L):

  p = c0^2 (rho - L rho),
  L = tau d/dt (-lap)^{y/2 - 1} + eta (-lap)^{(y+1)/2 - 1},
  tau = -2 alpha0 c0^{y-1},   eta = 2 alpha0 c0^y tan(pi y / 2).

Readings of the paper used here (where it is silent or loose):

* Discretisation: after the split-density update of a step,
  p = c0^2 (s + tau A[d] - eta B[s]) with s = sum_xi rho_xi,
  d = rho0 sum_xi d-_xi v_xi (the velocity divergence that drives the density
  update), A = F^-1 |k|^{y-2} F and B = F^-1 |k|^{y-1} F, both multipliers set
  to 0 at k = 0.  Mass conservation gives d rho/dt = -rho0 div v, so the tau
  term of -L rho becomes +tau (-lap)^{y/2-1} (rho0 div v): hence + tau A[d].
  Sources, adjoint injection and the Dirichlet imposition act on the split
  densities before s is formed (as in the lossless step).
* alpha0 is in Np (rad/s)^-y m^-1, a scalar or one value per voxel;
  0 < y < 2 and y != 1 (tan(pi y / 2) is infinite at y = 1).
* Time reversal flips the sign of tau (absorption becomes gain) and keeps
  eta; the TR simulation starts from the tape-only state with d = 0 in its
  first equation of state.
* The adjoint simulation is the same lossy solver (tau not flipped) with the
  reversed running-sum residual injected, as in Alg. 1.
* Gradient.  The exact discrete gradient (``exact_adjoint_gradient``)
  differentiates the discrete equation of state at a fixed state:
  (2 / c0) p + c0^2 (tau' A[d] - eta' B[s]) with tau' = -2 alpha0 (y - 1)
  c0^{y-2} and eta' = 2 alpha0 y c0^{y-1} tan(pi y / 2), the c0-derivatives
  of tau and eta (App. A prints dL/dc0 with other powers of c0 and without
  the tan factor; the finite-difference pin decides for the derivatives of
  the printed tau and eta).  The Alg. 1 form (``tr_gradient``,
  ``full_gradient``) keeps the lossless formula
  G = sum_j 2 / c0^3 p_adj^(j) (p^(j) - 2 p^(j+1) + p^(j+2)) with the lossy
  adjoint and TR fields, i.e. it leaves out the dL/dc0 terms: against the
  exact gradient this costs an error proportional to alpha0 (0.1 % at
  0.75 dB MHz^-1.5 cm^-1, pinned).
"""

from __future__ import annotations

import math
from typing import List, Optional

import numpy as np
import scipy.fft as sfft

from .kspace import (Scheme, State, _WORKERS, _idx, misfit_and_adjoint_source, source_scale)

NEPER_PER_DB = 1.0 / (20.0 * math.log10(math.e))


def db_to_neper(alpha_db: float, y: float) -> float:
    """alpha in dB MHz^-y cm^-1 -> alpha0 in Np (rad/s)^-y m^-1."""
    return 100.0 * alpha_db * NEPER_PER_DB / (2.0 * math.pi * 1.0e6) ** y


class Lossy:
    """The absorption operators on one grid (Sec. 2.1)."""

    def __init__(self, sch: Scheme, alpha0, y: float):
        if not (0.0 < y < 2.0) or y == 1.0:
            raise ValueError("power-law exponent y must lie in (0, 2) and differ from 1")
        self.sch = sch
        self.alpha0 = np.broadcast_to(np.asarray(alpha0, dtype=np.float64), sch.shape)
        self.y = float(y)
        kb = sch.kb
        kmag = np.sqrt(kb[0] ** 2 + kb[1] ** 2 + kb[2] ** 2)
        nz = kmag > 0
        self.mult_d = np.zeros(sch.shape)          # |k|^{y-2}, 0 at k = 0
        self.mult_s = np.zeros(sch.shape)          # |k|^{y-1}, 0 at k = 0
        self.mult_d[nz] = kmag[nz] ** (y - 2.0)
        self.mult_s[nz] = kmag[nz] ** (y - 1.0)
        self.tan = math.tan(math.pi * y / 2.0)

    def frac(self, g: np.ndarray, mult: np.ndarray) -> np.ndarray:
        out = sfft.ifftn(mult * sfft.fftn(g, workers=_WORKERS), workers=_WORKERS)
        return out.real

    def coefficients(self, c0: np.ndarray):
        """tau, eta and their c0-derivatives per voxel."""
        a, y = self.alpha0, self.y
        tau = -2.0 * a * c0 ** (y - 1.0)
        eta = 2.0 * a * c0 ** y * self.tan
        dtau = -2.0 * a * (y - 1.0) * c0 ** (y - 2.0)
        deta = 2.0 * a * y * c0 ** (y - 1.0) * self.tan
        return tau, eta, dtau, deta

    def eos(self, c0: np.ndarray, s: np.ndarray, d: np.ndarray, tau_sign: float = 1.0):
        """p = c0^2 (s + tau_sign tau A[d] - eta B[s]); returns (p, A[d], B[s])."""
        tau, eta, _, _ = self.coefficients(c0)
        A = self.frac(d, self.mult_d)
        B = self.frac(s, self.mult_s)
        return c0 * c0 * (s + tau_sign * tau * A - eta * B), A, B


def step(los: Lossy, st: State, c0: np.ndarray, inject=None, dirichlet=None, tau_sign: float = 1.0):
    """One lossy iteration in place; returns (A[d], B[s]) of its equation of state."""
    sch = los.sch
    dt, rho0 = sch.dt, sch.rho0
    p_hat = sfft.fftn(st.p, workers=_WORKERS)
    for a in range(3):      # momentum conservation, eq. MonCon
        ls = sch.lam_s[a]
        st.v[a] = ls * (ls * st.v[a] - (dt / rho0) * sch.d_plus(st.p, a, p_hat))
    div = [sch.d_minus(st.v[a], a) for a in range(3)]
    for a in range(3):      # mass conservation, eq. MassCon
        lm = sch.lam[a]
        st.rho[a] = lm * (lm * st.rho[a] - dt * rho0 * div[a])
    if inject is not None:
        idx, vals = inject
        for a in range(3):
            np.add.at(st.rho[a], idx, vals)
    if dirichlet is not None:
        idx, vals = dirichlet
        for a in range(3):
            st.rho[a][idx] = vals
    s = st.rho[0] + st.rho[1] + st.rho[2]
    d = rho0 * (div[0] + div[1] + div[2])
    st.p, A, B = los.eos(c0, s, d, tau_sign)    # eq. PreDenRel with L
    return A, B


def forward(los: Lossy, c0, src_ijk, src_sig, w, rec_ijk, nt, boundary=None, keep_history=None):
    """Lossy forward simulation; traces [nt, n_rec], tape [nt, |dGamma|] or
    None, and (keep_history) p^n on the mask's voxels, row 0 = p^0 = 0."""
    sch = los.sch
    c0 = np.asarray(c0, dtype=np.float64)
    src_idx, rec_idx = _idx(src_ijk), _idx(rec_ijk)
    sig = source_scale(sch, c0, src_ijk)
    w = np.asarray(w, dtype=np.float64)
    src_sig = np.asarray(src_sig, dtype=np.float64)
    b_idx = np.nonzero(boundary) if boundary is not None else None
    h_idx = np.nonzero(keep_history) if keep_history is not None else None
    st = State.zeros(sch.shape)
    traces = np.zeros((nt, len(rec_idx[0])))
    tape = np.zeros((nt, len(b_idx[0]))) if b_idx is not None else None
    hist = np.zeros((nt + 1, len(h_idx[0]))) if h_idx is not None else None
    for n in range(nt):
        step(los, st, c0, inject=(src_idx, sig * w * src_sig[n]))
        traces[n] = st.p[rec_idx]
        if tape is not None:
            tape[n] = st.p[b_idx]
        if hist is not None:
            hist[n + 1] = st.p[h_idx]
    return dict(traces=traces, tape=tape, history=hist)


def _adjoint_run(los, c0, rec_idx, a, g_idx, ring_of):
    """Adjoint iterations j = 0..N-1 with
    G += 2 / c0^3 p_adj (p^(j) - 2 p^(j+1) + p^(j+2))."""
    adj = State.zeros(los.sch.shape)
    G = np.zeros(len(g_idx[0]))
    pref = 2.0 / (c0[g_idx] ** 3)
    for j in range(a.shape[0]):
        step(los, adj, c0, inject=(rec_idx, a[j] / 3.0))
        G += pref * adj.p[g_idx] * (ring_of(j) - 2.0 * ring_of(j + 1) + ring_of(j + 2))
    return G


def tr_gradient(los: Lossy, c0, src_ijk, src_sig, w, rec_ijk, obs, gamma, boundary, nt,
                residual=None, fwd=None, flip_tau=True):
    """Lossy TR gradient in the form of Alg. 1: forward with boundary tape,
    residual and reversed running sum, TR (tau flipped unless ``flip_tau`` is
    False, Dirichlet on dGamma, zero interior start) one step ahead of the
    adjoint, ring of p_tr on Gamma.  Returns (D, G on the full grid (zero outside Gamma), forward traces)."""
    sch = los.sch
    c0 = np.asarray(c0, dtype=np.float64)
    c0sq = c0 * c0
    if fwd is None:
        fwd = forward(los, c0, src_ijk, src_sig, w, rec_ijk, nt, boundary=boundary)
    traces, tape = fwd["traces"], fwd["tape"]
    if residual is None:
        D, _, a = misfit_and_adjoint_source(traces, obs)
    else:
        r = np.asarray(residual, dtype=np.float64)
        D = 0.5 * float(np.sum(r * r))
        a = np.cumsum(r[::-1], axis=0)
    b_idx = np.nonzero(boundary)
    g_idx = np.nonzero(gamma)
    rec_idx = _idx(rec_ijk)
    scale_b = 1.0 / (3.0 * c0sq[b_idx])
    sgn = -1.0 if flip_tau else 1.0

    tr = State.zeros(sch.shape)
    for ax in range(3):
        tr.rho[ax][b_idx] = tape[nt - 1] * scale_b
    s0 = tr.rho[0] + tr.rho[1] + tr.rho[2]
    tr.p, _, _ = los.eos(c0, s0, np.zeros(sch.shape), tau_sign=sgn)
    ring = {0: tr.p[g_idx].copy()}
    zero_g = np.zeros(len(g_idx[0]))

    def tr_step(k):
        step(los, tr, c0, dirichlet=(b_idx, tape[nt - 1 - k] * scale_b), tau_sign=sgn)
        return tr.p[g_idx].copy()

    if nt >= 2:
        ring[1] = tr_step(1)

    def ring_of(k):
        if k not in ring:
            ring[k] = tr_step(k) if k <= nt - 1 else zero_g
        return ring[k]

    G = _adjoint_run(los, c0, rec_idx, a, g_idx, ring_of)
    out = np.zeros(sch.shape)
    out[g_idx] = G
    return D, out, traces


def full_gradient(los: Lossy, c0, src_ijk, src_sig, w, rec_ijk, obs, gamma, nt, residual=None):
    """The same formula with the stored forward history of p on Gamma."""
    sch = los.sch
    c0 = np.asarray(c0, dtype=np.float64)
    fwd = forward(los, c0, src_ijk, src_sig, w, rec_ijk, nt, keep_history=gamma)
    hist = fwd["history"]
    if residual is None:
        D, _, a = misfit_and_adjoint_source(fwd["traces"], obs)
    else:
        r = np.asarray(residual, dtype=np.float64)
        D = 0.5 * float(np.sum(r * r))
        a = np.cumsum(r[::-1], axis=0)
    g_idx = np.nonzero(gamma)
    zero_g = np.zeros(len(g_idx[0]))

    def ring_of(k):           # p_tr^(k) = p^{N-k} of the forward run
        return hist[nt - k] if k <= nt else zero_g

    G = _adjoint_run(los, c0, _idx(rec_ijk), a, g_idx, ring_of)
    out = np.zeros(sch.shape)
    out[g_idx] = G
    return D, out, fwd["traces"]


def exact_adjoint_gradient(los: Lossy, c0, src_ijk, src_sig, w, rec_ijk, obs, nt, residual=None):
    """dD/dc0 of the lossy forward loop by the literal transpose of every
    discrete operation (reverse mode, PML included).  The fractional
    operators A and B are real, even multipliers, hence symmetric.  As in the
    lossless case the c0 of the source scaling is held fixed."""
    sch = los.sch
    c0 = np.asarray(c0, dtype=np.float64)
    src_idx, rec_idx = _idx(src_ijk), _idx(rec_ijk)
    sig = source_scale(sch, c0, src_ijk)
    w = np.asarray(w, dtype=np.float64)
    src_sig = np.asarray(src_sig, dtype=np.float64)
    tau, eta, dtau, deta = los.coefficients(c0)
    Q = c0 * c0
    st = State.zeros(sch.shape)
    dpdc: List[np.ndarray] = []
    traces = np.zeros((nt, len(rec_idx[0])))
    for n in range(nt):
        A, B = step(los, st, c0, inject=(src_idx, sig * w * src_sig[n]))
        traces[n] = st.p[rec_idx]
        dpdc.append(2.0 / c0 * st.p + Q * (dtau * A - deta * B))
    r = traces - obs if residual is None else np.asarray(residual, dtype=np.float64)
    D = 0.5 * float(np.sum(r * r))
    dt, rho0 = sch.dt, sch.rho0
    vb = [np.zeros(sch.shape) for _ in range(3)]
    rb = [np.zeros(sch.shape) for _ in range(3)]
    pb = np.zeros(sch.shape)
    cb = np.zeros(sch.shape)
    for n in range(nt - 1, -1, -1):
        np.add.at(pb, rec_idx, r[n])                          # loss term, M^T r^n
        cb += pb * dpdc[n]
        sb = Q * pb - los.frac(eta * Q * pb, los.mult_s)      # p = Q (s + tau A[d] - eta B[s])
        db = los.frac(tau * Q * pb, los.mult_d)
        pb = np.zeros(sch.shape)
        ub = [rho0 * db for _ in range(3)]                    # d = rho0 sum u_a
        for a in range(3):
            rb[a] = rb[a] + sb                                # s = sum rho_a
            t = sch.lam[a] * rb[a]                            # rho update transposed
            ub[a] = ub[a] - dt * rho0 * t
            rb[a] = sch.lam[a] * t
            vb[a] = vb[a] + sch.d_minus_T(ub[a], a)           # u_a = d-_a v_a
        for a in range(3):                                    # velocity update transposed
            t = sch.lam_s[a] * vb[a]
            pb = pb - (dt / rho0) * sch.d_plus_T(t, a)
            vb[a] = sch.lam_s[a] * t
    return D, cb, traces


def mode_matrix(los: Lossy, c0: float, m: int, tau_sign: float = 1.0) -> np.ndarray:
    """6 x 6 real matrix of one lossy step acting on the plane wave of x-mode
    m (k = 2 pi m / (nx dx)) in a homogeneous periodic box (no PML): state
    (v_x, s, p), each as its cos / sin (k x) components.  Obtained by running
    the step on the six basis states and projecting back onto the mode."""
    sch = los.sch
    nz, ny, nx = sch.shape
    x = np.arange(nx) * sch.dx
    k = 2.0 * math.pi * m / (nx * sch.dx)
    cs = np.broadcast_to(np.cos(k * x), sch.shape)
    sn = np.broadcast_to(np.sin(k * x), sch.shape)
    c0f = np.full(sch.shape, float(c0))

    def proj(g):
        return np.array([np.sum(g * cs), np.sum(g * sn)]) / np.sum(cs * cs)

    cols = []
    for b in range(6):
        st = State.zeros(sch.shape)
        base = np.array(cs if b % 2 == 0 else sn)
        if b < 2:
            st.v[0] = base
        elif b < 4:
            for a in range(3):
                st.rho[a] = base / 3.0
        else:
            st.p = base
        step(los, st, c0f, tau_sign=tau_sign)
        cols.append(np.concatenate([proj(st.v[0]), proj(st.rho[0] + st.rho[1] + st.rho[2]), proj(st.p)]))
    return np.array(cols).T


def wave_eigenvalue(M: np.ndarray) -> complex:
    """The eigenvalue of the travelling wave: largest modulus, positive phase."""
    ev = np.linalg.eigvals(M)
    ev = ev[np.imag(ev) > 0]
    return complex(ev[np.argmax(np.abs(ev))])
