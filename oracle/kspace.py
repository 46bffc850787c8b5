"""Plain FP64 oracle: k-space PSTD acoustics, TR gradient, exact adjoint.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Slow on purpose: every
spectral derivative is a full complex 3D FFT, a multiplication and a full
complex inverse FFT, exactly as eq. DisPartDev / DisPartDevSt define it.

Notation follows the paper (App. B):  p pressure, v_xi particle velocity,
rho_xi split density, c0 sound speed, rho0 ambient density, kappa the k-space
operator, Lambda_xi / Lambda^s_xi the PML multipliers on the normal /
staggered grid, M the sensor operator, S the source operator, g^n the
boundary-layer pressure, q the time-reversed residual.

Readings of the paper used here (where it is silent or loose):

* sinc is the unnormalised sin(x)/x, kappa(0) = 1 (the form for which the
  correction is exact in a homogeneous medium, App. B).
* Arrays are [z, y, x]; the PML lies inside the grid; Lambda = exp(-alpha
  dt / 2) with alpha = pml_alpha * (c_ref / dx) * (d / P)^4, d the distance
  in cells into a PML of P cells (normal grid at integer positions, staggered
  grid at half-integer positions).
* The forward loop runs N iterations n = 0..N-1 (Alg. 1 writes 0..N_t) and
  records f^n = M p^{n+1}, g^n = p^{n+1}(dGamma).
* The mass source is added as 2 dt s / (3 dx c0) to each split density
  (App. B: divide by c0, scale by 2 / (3 dx)); c0 taken at the source voxel.
* Adjoint source: the reversed running sum a^j = sum_{i<=j} r^{N-1-i} of the
  residual r^n = f^n - f^delta_n (Alg. 1 "cumsum"), injected as a^j / 3 into
  each split density at the receiver voxels; gradient prefactor 2 / c0^3.
  These are the exact discrete scalings; the paper's own constants
  (2 dt / (3 dx c0) and 2 / (dt c0^3)) differ from them by one global positive
  factor 2 / (dx c_w), which the paper says it omits.  Finite-difference and
  dot-product tests pin this choice.
* Time reversal: rho_xi(dGamma) <- g / (3 c0^2) per split component, TR step
  k = 1..N-1 imposes g^{N-1-k}; p_tr^(k) = 0 for k >= N.  Adjoint iteration j
  pairs with p_tr^(j), p_tr^(j+1), p_tr^(j+2) (Alg. 1 ring p_rec^-, 0, +).
* Misfit D = 1/2 sum_n sum_r (r^n_r)^2, no dt weight.
"""

from __future__ import annotations

import dataclasses
import os
from typing import List, Optional

import numpy as np
import scipy.fft as sfft

_WORKERS = max(1, min(16, os.cpu_count() or 1))

_MASK64 = (1 << 64) - 1


# --------------------------------------------------------------------------
# SplitMix64 and Rademacher weights (Sec. 3.2: w_i = +-1 with equal probability)
# --------------------------------------------------------------------------

def splitmix64(seed: int, i: int) -> int:
    """i-th output (0-based) of SplitMix64 seeded with ``seed``.

    SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): the state advances by the
    golden-ratio increment 0x9e3779b97f4a7c15 and each output is the state
    passed through the variant-13 finaliser of Stafford's MurmurHash3 mix.
    """
    z = (seed + (i + 1) * 0x9E3779B97F4A7C15) & _MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
    return z ^ (z >> 31)


def rademacher(seed: int, n: int) -> np.ndarray:
    """Rademacher weights (Sec. 3.2, App. E): +1 if the top bit of the i-th
    SplitMix64 output is 0, else -1.  int8 [n]."""
    w = np.empty(n, dtype=np.int8)
    for i in range(n):
        w[i] = -1 if (splitmix64(seed, i) >> 63) else 1
    return w


def delays(seed: int, n: int, tau_steps: int) -> np.ndarray:
    """Delayed source encoding (Sec. 3.2, eq. DelaySE): d_i ~ U[0,1) is the
    uniform (top 53 bits / 2^53) of SplitMix64 output n + i of ``seed``;
    the delay in whole steps is floor(d_i tau_steps + 1/2)."""
    out = np.empty(n, dtype=np.int32)
    for i in range(n):
        d = (splitmix64(seed, n + i) >> 11) / float(1 << 53)
        out[i] = int(np.floor(d * tau_steps + 0.5))
    return out


def delayed_signals(src_sig, delay_steps, nt_total: int) -> np.ndarray:
    """Delayed encoded sources (Sec. 3.2, eq. DelaySE): source i emits
    s_i(t - d_i tau), i.e. its samples start delay_steps[i] steps late.
    Returns [nt_total, n_src]: zero before each source's delay and after its
    own samples run out."""
    src = np.asarray(src_sig, dtype=np.float64)
    nt, ns = src.shape
    out = np.zeros((nt_total, ns))
    for i in range(ns):
        d = int(delay_steps[i])
        for n in range(d, nt_total):
            if n - d < nt:
                out[n, i] = src[n - d, i]
    return out


# --------------------------------------------------------------------------
# discretisation (App. B)
# --------------------------------------------------------------------------

def wavenumbers(n: int, dx: float) -> np.ndarray:
    """Discrete wavevector k_xi = 2 pi * fftfreq(n, dx)."""
    return 2.0 * np.pi * np.fft.fftfreq(n, d=dx)


def sinc_unnormalised(x: np.ndarray) -> np.ndarray:
    out = np.ones_like(x)
    nz = x != 0
    out[nz] = np.sin(x[nz]) / x[nz]
    return out


def pml_profile(n: int, size: int, dx: float, dt: float, c_ref: float, alpha: float,
                staggered: bool) -> np.ndarray:
    """Lambda = exp(-a dt / 2), a = alpha (c_ref/dx) (d/P)^4 (see module doc)."""
    if size == 0:
        return np.ones(n)
    s = np.arange(n, dtype=np.float64) + (0.5 if staggered else 0.0)
    d = np.maximum(0.0, np.maximum(size - s, s - (n - 1 - size)))
    a = alpha * (c_ref / dx) * (d / size) ** 4
    return np.exp(-a * dt / 2.0)


class Scheme:
    """Operators of the k-space scheme on one grid (App. B)."""

    def __init__(self, shape, dx, dt, c_ref, rho0, pml=(0, 0, 0), pml_alpha=2.0):
        self.shape = tuple(int(s) for s in shape)
        nz, ny, nx = self.shape
        self.dx, self.dt, self.c_ref, self.rho0 = float(dx), float(dt), float(c_ref), float(rho0)
        self.pml = tuple(int(p) for p in pml)          # (px, py, pz)
        k1 = [wavenumbers(nx, dx), wavenumbers(ny, dx), wavenumbers(nz, dx)]
        kb = [k1[0][None, None, :], k1[1][None, :, None], k1[2][:, None, None]]
        kmag = np.sqrt(kb[0] ** 2 + kb[1] ** 2 + kb[2] ** 2)
        # eq. DisPartDev: kappa = sinc(c_ref dt |k| / 2)
        self.kappa = sinc_unnormalised(c_ref * dt * kmag / 2.0)
        self.kb = kb
        # eq. DisPartDevSt: i k_xi kappa exp(+- i k_xi dxi / 2)
        self.m_plus = [1j * kb[a] * self.kappa * np.exp(+1j * kb[a] * dx / 2.0) for a in range(3)]
        self.m_minus = [1j * kb[a] * self.kappa * np.exp(-1j * kb[a] * dx / 2.0) for a in range(3)]
        lens = [nx, ny, nz]
        shp = [(1, 1, nx), (1, ny, 1), (nz, 1, 1)]
        self.lam = [pml_profile(lens[a], self.pml[a], dx, dt, c_ref, pml_alpha, False).reshape(shp[a])
                    for a in range(3)]
        self.lam_s = [pml_profile(lens[a], self.pml[a], dx, dt, c_ref, pml_alpha, True).reshape(shp[a])
                      for a in range(3)]

    # spectral derivative: Re F^-1 { m F g }
    def apply(self, g: np.ndarray, m: np.ndarray, g_hat: Optional[np.ndarray] = None) -> np.ndarray:
        if g_hat is None:
            g_hat = sfft.fftn(g, workers=_WORKERS)
        out = sfft.ifftn(m * g_hat, workers=_WORKERS)
        scale = np.abs(out).max() if out.size else 0.0
        assert np.abs(out.imag).max() <= 1e-10 * max(scale, 1e-300), "multiplier not Hermitian"
        return out.real

    def d_plus(self, g, axis, g_hat=None):
        return self.apply(g, self.m_plus[axis], g_hat)

    def d_minus(self, g, axis, g_hat=None):
        return self.apply(g, self.m_minus[axis], g_hat)

    # literal transposes (kernel reflected <=> multiplier conjugated)
    def d_plus_T(self, g, axis):
        return self.apply(g, np.conj(self.m_plus[axis]))

    def d_minus_T(self, g, axis):
        return self.apply(g, np.conj(self.m_minus[axis]))


@dataclasses.dataclass
class State:
    v: List[np.ndarray]
    rho: List[np.ndarray]
    p: np.ndarray

    @staticmethod
    def zeros(shape):
        return State([np.zeros(shape) for _ in range(3)], [np.zeros(shape) for _ in range(3)],
                     np.zeros(shape))

    def copy(self):
        return State([a.copy() for a in self.v], [a.copy() for a in self.rho], self.p.copy())


def _idx(ijk: np.ndarray):
    """[n,3] (ix,iy,iz) -> fancy index tuple (iz, iy, ix)."""
    ijk = np.asarray(ijk)
    return (ijk[:, 2], ijk[:, 1], ijk[:, 0])


def step(sch: Scheme, st: State, c0sq: np.ndarray, inject=None, dirichlet=None) -> None:
    """One iteration of the Alg. 1 loop body, in place.

    inject:    (index tuple, values)  added to every rho_xi at those voxels
    dirichlet: (index tuple, values)  assigned to every rho_xi at those voxels
    """
    dt, rho0 = sch.dt, sch.rho0
    p_hat = sfft.fftn(st.p, workers=_WORKERS)
    for a in range(3):      # momentum conservation, eq. MonCon
        ls = sch.lam_s[a]
        st.v[a] = ls * (ls * st.v[a] - (dt / rho0) * sch.d_plus(st.p, a, p_hat))
    for a in range(3):      # mass conservation, eq. MassCon
        lm = sch.lam[a]
        st.rho[a] = lm * (lm * st.rho[a] - dt * rho0 * sch.d_minus(st.v[a], a))
    if inject is not None:
        idx, vals = inject
        for a in range(3):
            np.add.at(st.rho[a], idx, vals)
    if dirichlet is not None:
        idx, vals = dirichlet
        for a in range(3):
            st.rho[a][idx] = vals
    st.p = c0sq * (st.rho[0] + st.rho[1] + st.rho[2])   # eq. PreDenRel


def velocity_half_step(sch: Scheme, st: State) -> List[np.ndarray]:
    """v^{n+1/2} from (v^{n-1/2}, p^n) without modifying the state."""
    p_hat = sfft.fftn(st.p, workers=_WORKERS)
    out = []
    for a in range(3):
        ls = sch.lam_s[a]
        out.append(ls * (ls * st.v[a] - (sch.dt / sch.rho0) * sch.d_plus(st.p, a, p_hat)))
    return out


# --------------------------------------------------------------------------
# forward simulation (Alg. 1, forward iteration)
# --------------------------------------------------------------------------

def scheme_for(prob) -> Scheme:
    return Scheme(prob.shape, prob.dx, prob.dt, prob.c_ref, prob.rho0, prob.pml, prob.pml_alpha)


def source_scale(sch: Scheme, c0: np.ndarray, src_ijk) -> np.ndarray:
    """2 dt / (3 dx c0) at the source voxels (App. B mass-source conversion)."""
    return 2.0 * sch.dt / (3.0 * sch.dx * c0[_idx(src_ijk)])


def forward(sch: Scheme, c0, src_ijk, src_sig, w, rec_ijk, nt, boundary=None,
            keep_history=None, return_state=False):
    """Forward simulation with encoded sources s_hat_i(t_n) = w_i s_i(t_n).

    Returns dict(traces [nt, n_rec], tape [nt, |dGamma|] or None,
    history [nt+1, |H|] of p on the voxels of mask ``keep_history`` (row 0 is
    p^0 = 0), rho_sum history for the exact adjoint, final state).
    """
    c0 = np.asarray(c0, dtype=np.float64)
    c0sq = c0 * c0
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
        step(sch, st, c0sq, inject=(src_idx, sig * w * src_sig[n]))
        traces[n] = st.p[rec_idx]                 # f^n = M p
        if tape is not None:
            tape[n] = st.p[b_idx]                 # g^n = p(dGamma)
        if hist is not None:
            hist[n + 1] = st.p[h_idx]
    out = dict(traces=traces, tape=tape, history=hist)
    if return_state:
        out["state"] = st
    return out


def misfit_and_adjoint_source(traces, obs):
    """Alg. 1 setup: r^n = f^n - f^delta_n, D = 1/2 ||r||^2, and the reversed
    running sum a^j = sum_{i<=j} r^{N-1-i} (time-reversed residual, then
    cumsum)."""
    r = np.asarray(traces, dtype=np.float64) - np.asarray(obs, dtype=np.float64)
    D = 0.5 * float(np.sum(r * r))
    a = np.cumsum(r[::-1], axis=0)
    return D, r, a


# --------------------------------------------------------------------------
# TR gradient (Alg. 1) and its two reference gradients
# --------------------------------------------------------------------------

def tr_gradient(sch: Scheme, c0, src_ijk, src_sig, w, rec_ijk, obs, gamma, boundary, nt,
                tr_init="zero", reinject_sources=False, residual=None, fwd=None):
    """Time-reversal speed-of-sound gradient (Alg. 1, Sec. 3.1).

    Forward run with boundary tape; residual / misfit / cumsum; TR state from
    the tape (zero interior, or the final forward state when
    ``tr_init='final_state'``); one TR pre-step; then N lock-stepped
    iterations of the adjoint (injection a^j/3) and the TR (Dirichlet on
    dGamma) with the gradient accumulated on Gamma.

    ``residual`` replaces f - f^delta (autograd backward: the incoming
    gradient of the traces); then ``obs`` is ignored and D = 1/2 ||r||^2.
    ``reinject_sources`` subtracts the sources in reverse order during TR
    (makes TR exact in a PML-free box; used only by the pins).
    Returns (D, G) with G on the full grid, zero outside Gamma, plus the
    forward traces.
    """
    c0 = np.asarray(c0, dtype=np.float64)
    c0sq = c0 * c0
    if fwd is None:
        fwd = forward(sch, c0, src_ijk, src_sig, w, rec_ijk, nt, boundary=boundary,
                      return_state=(tr_init == "final_state"))
    traces, tape = fwd["traces"], fwd["tape"]
    if residual is None:
        D, r, a = misfit_and_adjoint_source(traces, obs)
    else:
        r = np.asarray(residual, dtype=np.float64)
        D = 0.5 * float(np.sum(r * r))
        a = np.cumsum(r[::-1], axis=0)
    b_idx = np.nonzero(boundary)
    g_idx = np.nonzero(gamma)
    rec_idx = _idx(rec_ijk)
    src_idx = _idx(src_ijk)
    sig = source_scale(sch, c0, src_ijk)
    w = np.asarray(w, dtype=np.float64)
    src_sig = np.asarray(src_sig, dtype=np.float64)
    scale_b = 1.0 / (3.0 * c0sq[b_idx])                  # g / (3 c0(dGamma)^2)

    # TR initial state (Alg. 1 setup)
    if tr_init == "zero":
        tr = State.zeros(sch.shape)
    elif tr_init == "final_state":
        fin = fwd["state"]
        v_next = velocity_half_step(sch, fin)             # v^{N+1/2}
        tr = State([-v for v in v_next], [r_.copy() for r_ in fin.rho], fin.p.copy())
    else:
        raise ValueError(tr_init)
    for ax in range(3):
        tr.rho[ax][b_idx] = tape[nt - 1] * scale_b
    tr.p = c0sq * (tr.rho[0] + tr.rho[1] + tr.rho[2])

    def tr_step(k):
        inj = None
        if reinject_sources:
            inj = (src_idx, -sig * w * src_sig[nt - k])
        step(sch, tr, c0sq, inject=inj, dirichlet=(b_idx, tape[nt - 1 - k] * scale_b))
        return tr.p[g_idx].copy()

    ring = {0: tr.p[g_idx].copy()}
    if nt >= 2:
        ring[1] = tr_step(1)                              # advance TR by one step
    zero_g = np.zeros(len(g_idx[0]))
    adj = State.zeros(sch.shape)
    G = np.zeros(len(g_idx[0]))
    pref = 2.0 / (c0[g_idx] ** 3)
    for j in range(nt):
        step(sch, adj, c0sq, inject=(rec_idx, a[j] / 3.0))
        k = j + 2
        ring[k] = tr_step(k) if k <= nt - 1 else zero_g
        pm, p0, pp = ring[j], ring.get(j + 1, zero_g), ring[k]
        G += pref * adj.p[g_idx] * (pm - 2.0 * p0 + pp)
        ring.pop(j)
    out = np.zeros(sch.shape)
    out[g_idx] = G
    return D, out, traces


def full_gradient(sch: Scheme, c0, src_ijk, src_sig, w, rec_ijk, obs, gamma, nt, residual=None):
    """Same gradient formula with the stored forward history p^n on Gamma in
    place of the TR re-simulation (the 'full' column of Table TRGrad)."""
    c0 = np.asarray(c0, dtype=np.float64)
    c0sq = c0 * c0
    fwd = forward(sch, c0, src_ijk, src_sig, w, rec_ijk, nt, keep_history=gamma)
    hist = fwd["history"]                     # hist[n] = p^n on Gamma, n = 0..N
    if residual is None:
        D, r, a = misfit_and_adjoint_source(fwd["traces"], obs)
    else:
        r = np.asarray(residual, dtype=np.float64)
        D = 0.5 * float(np.sum(r * r))
        a = np.cumsum(r[::-1], axis=0)
    g_idx = np.nonzero(gamma)
    rec_idx = _idx(rec_ijk)
    zero_g = np.zeros(len(g_idx[0]))

    def ph(n):
        return hist[n] if n >= 0 else zero_g

    adj = State.zeros(sch.shape)
    G = np.zeros(len(g_idx[0]))
    pref = 2.0 / (c0[g_idx] ** 3)
    for j in range(nt):
        step(sch, adj, c0sq, inject=(rec_idx, a[j] / 3.0))
        G += pref * adj.p[g_idx] * (ph(nt - j) - 2.0 * ph(nt - 1 - j) + ph(nt - 2 - j))
    out = np.zeros(sch.shape)
    out[g_idx] = G
    return D, out, fwd["traces"]


def exact_adjoint_gradient(sch: Scheme, c0, src_ijk, src_sig, w, rec_ijk, obs, nt, residual=None):
    """dD/dc0 by the literal transpose of every discrete operation of the
    forward loop (reverse-mode differentiation of Alg. 1's forward iteration,
    PML included).  D depends on c0 through the equation of state
    p = c0^2 sum rho_xi; the c0 in the source scaling (source voxels only) is
    held fixed, so the result is exact on every voxel without a source.
    """
    c0 = np.asarray(c0, dtype=np.float64)
    Q = c0 * c0
    src_idx, rec_idx = _idx(src_ijk), _idx(rec_ijk)
    sig = source_scale(sch, c0, src_ijk)
    w = np.asarray(w, dtype=np.float64)
    src_sig = np.asarray(src_sig, dtype=np.float64)
    st = State.zeros(sch.shape)
    rho_sum = []
    traces = np.zeros((nt, len(rec_idx[0])))
    for n in range(nt):
        step(sch, st, Q, inject=(src_idx, sig * w * src_sig[n]))
        traces[n] = st.p[rec_idx]
        rho_sum.append(st.rho[0] + st.rho[1] + st.rho[2])
    r = traces - obs if residual is None else np.asarray(residual, dtype=np.float64)
    D = 0.5 * float(np.sum(r * r))
    dt, rho0 = sch.dt, sch.rho0
    vb = [np.zeros(sch.shape) for _ in range(3)]
    rb = [np.zeros(sch.shape) for _ in range(3)]
    pb = np.zeros(sch.shape)
    Qb = np.zeros(sch.shape)
    for n in range(nt - 1, -1, -1):
        np.add.at(pb, rec_idx, r[n])                       # loss term, M^T r^n
        Qb += pb * rho_sum[n]                              # p = Q sum rho
        for a in range(3):
            rb[a] = rb[a] + Q * pb
        pb = np.zeros(sch.shape)
        for a in range(3):                                 # rho update transposed
            t = sch.lam[a] * rb[a]
            vb[a] = vb[a] - dt * rho0 * sch.d_minus_T(t, a)
            rb[a] = sch.lam[a] * t
        for a in range(3):                                 # velocity update transposed
            t = sch.lam_s[a] * vb[a]
            pb = pb - (dt / rho0) * sch.d_plus_T(t, a)
            vb[a] = sch.lam_s[a] * t
    return D, 2.0 * c0 * Qb, traces


def tangent_linear_traces(sch: Scheme, c0, dc, src_ijk, src_sig, w, rec_ijk, nt):
    """Directional derivative of the traces along dc (dc = 0 at source
    voxels): forward-mode differentiation of the forward iteration."""
    c0 = np.asarray(c0, dtype=np.float64)
    Q = c0 * c0
    dQ = 2.0 * c0 * np.asarray(dc, dtype=np.float64)
    src_idx, rec_idx = _idx(src_ijk), _idx(rec_ijk)
    sig = source_scale(sch, c0, src_ijk)
    w = np.asarray(w, dtype=np.float64)
    src_sig = np.asarray(src_sig, dtype=np.float64)
    st = State.zeros(sch.shape)
    dst = State.zeros(sch.shape)
    dtr = np.zeros((nt, len(rec_idx[0])))
    dt, rho0 = sch.dt, sch.rho0
    for n in range(nt):
        for a in range(3):
            ls = sch.lam_s[a]
            dst.v[a] = ls * (ls * dst.v[a] - (dt / rho0) * sch.d_plus(dst.p, a))
        for a in range(3):
            lm = sch.lam[a]
            dst.rho[a] = lm * (lm * dst.rho[a] - dt * rho0 * sch.d_minus(dst.v[a], a))
        step(sch, st, Q, inject=(src_idx, sig * w * src_sig[n]))
        rs = st.rho[0] + st.rho[1] + st.rho[2]
        dst.p = dQ * rs + Q * (dst.rho[0] + dst.rho[1] + dst.rho[2])
        dtr[n] = dst.p[rec_idx]
    return dtr


# --------------------------------------------------------------------------
# brute force
# --------------------------------------------------------------------------

def _dft_matrix(n: int, sign: float) -> np.ndarray:
    j = np.arange(n)
    return np.exp(sign * 2j * np.pi * np.outer(j, j) / n)


def brute_force_dft3(g: np.ndarray, inverse: bool = False) -> np.ndarray:
    """3D DFT by its definition, one O(N^2) sum per axis (no FFT)."""
    sign = 1.0 if inverse else -1.0
    out = np.asarray(g, dtype=np.complex128)
    for ax in range(3):
        F = _dft_matrix(out.shape[ax], sign)
        out = np.moveaxis(np.tensordot(F, np.moveaxis(out, ax, 0), axes=(1, 0)), 0, ax)
    if inverse:
        out = out / out.size
    return out
