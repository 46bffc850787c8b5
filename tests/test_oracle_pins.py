"""Pins of the FP64 oracle against facts that do not come from the oracle.

Each test names the passage of arXiv 2102.00755 (or the mathematical fact)
it relies on.  Tiny grids keep the whole file to well under a minute.
"""

import math

import numpy as np
import pytest

import oracle
from oracle import kspace as ks
from synth import configs as sc


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


# ---------------------------------------------------------------- T0 config arithmetic
def test_config_time_step_and_data_size():
    # Sec. 4.1: dt = cfl dx / c_max = 83.3 ns at 0.5 mm, cfl 0.3, c_max 1800 m/s
    assert abs(sc.time_step(0.5e-3) - 83.3e-9) < 0.05e-9
    # Sec. 4.1: 1024 x 1024 x 3912 single-precision samples = 15.28 GiB
    assert round(1024 * 1024 * 3912 * 4 / 2 ** 30, 2) == 15.28


# ---------------------------------------------------------------- SplitMix64 / Rademacher
def test_splitmix64_published_outputs():
    # First outputs of SplitMix64 seeded with 0, as printed by the public
    # reference implementation of Steele, Lea & Flood's generator.
    got = [ks.splitmix64(0, i) for i in range(3)]
    assert got == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_rademacher_is_top_bit_rule_and_balanced():
    w = oracle.rademacher(1005, 4096)
    assert w.dtype == np.int8 and set(np.unique(w).tolist()) == {-1, 1}
    assert abs(float(w.mean())) < 0.06          # E[w] = 0 (Sec. 3.2), 4096 draws
    for i in (0, 1, 17):
        assert w[i] == (-1 if ks.splitmix64(1005, i) >> 63 else 1)


# ---------------------------------------------------------------- T1 brute-force DFT
@pytest.mark.parametrize("shape", [(6, 5, 8), (7, 4, 6), (8, 8, 8)])
def test_fft_matches_brute_force_dft(shape):
    rng = np.random.default_rng(1)
    g = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    import scipy.fft as sfft
    assert rel(sfft.fftn(g), oracle.brute_force_dft3(g)) < 1e-13
    assert rel(sfft.ifftn(g), oracle.brute_force_dft3(g, inverse=True)) < 1e-13


@pytest.mark.parametrize("shape", [(6, 5, 8), (7, 4, 6), (8, 8, 8)])
def test_staggered_derivative_vs_brute_force(shape):
    # eq. DisPartDevSt evaluated with explicit DFT sums instead of FFTs
    sch = ks.Scheme(shape, 0.5e-3, 8e-8, 1800.0, 1000.0)
    rng = np.random.default_rng(2)
    g = rng.standard_normal(shape)
    for a in range(3):
        for m, fn in ((sch.m_plus[a], sch.d_plus), (sch.m_minus[a], sch.d_minus)):
            ref = oracle.brute_force_dft3(m * oracle.brute_force_dft3(g), inverse=True)
            assert np.abs(ref.imag).max() < 1e-12 * np.abs(ref).max()
            assert rel(fn(g, a), ref.real) < 1e-12


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_staggered_derivative_single_mode_closed_form(axis):
    # For g = sin(k0 xi + phi), eq. DisPartDevSt gives
    # d+- g = k0 kappa(k0) cos(k0 (xi +- dxi/2) + phi), kappa = sin(u)/u,
    # u = c_ref dt k0 / 2.
    shape = (12, 10, 16)
    dx, dt, cref = 0.5e-3, 8e-8, 1800.0
    sch = ks.Scheme(shape, dx, dt, cref, 1000.0)
    n = shape[::-1][axis]
    k0 = 2 * math.pi * 3 / (n * dx)
    coord = np.arange(n) * dx
    phi = 0.3
    u = cref * dt * k0 / 2
    kap = math.sin(u) / u
    bshape = [1, 1, 1]
    bshape[2 - axis] = n
    g = np.broadcast_to(np.sin(k0 * coord + phi).reshape(bshape), shape).copy()
    for sgn, fn in ((+1, sch.d_plus), (-1, sch.d_minus)):
        want = k0 * kap * np.cos(k0 * (coord + sgn * dx / 2) + phi)
        want = np.broadcast_to(want.reshape(bshape), shape)
        assert rel(fn(g, axis), want) < 1e-12


# ---------------------------------------------------------------- T2 homogeneous single mode
def test_single_mode_evolves_exactly_as_cosine():
    # App. B: the k-space correction makes time stepping exact in a
    # homogeneous medium with c = c_ref.  For the standing wave started with
    # v^{-1/2} = (dt / 2 rho0) d+ p^0 the discrete field is p^0 cos(n c dt |k|).
    shape = (8, 10, 12)
    dx, c = 0.5e-3, 1500.0
    dt = 0.3 * dx / c
    sch = ks.Scheme(shape, dx, dt, c, 1000.0)
    nz, ny, nx = shape
    kx, ky, kz = 2 * math.pi * 2 / (nx * dx), 2 * math.pi * 3 / (ny * dx), 2 * math.pi * 1 / (nz * dx)
    z, y, x = np.meshgrid(np.arange(nz) * dx, np.arange(ny) * dx, np.arange(nx) * dx, indexing="ij")
    p0 = np.cos(kx * x + ky * y + kz * z)
    c0sq = np.full(shape, c * c)
    st = ks.State.zeros(shape)
    st.p = p0.copy()
    for a in range(3):
        st.rho[a] = p0 / (3 * c * c)
        st.v[a] = (dt / (2 * sch.rho0)) * sch.d_plus(p0, a)
    theta = c * dt * math.sqrt(kx * kx + ky * ky + kz * kz)
    err = 0.0
    for n in range(1, 1001):
        ks.step(sch, st, c0sq)
        err = max(err, float(np.abs(st.p - p0 * math.cos(n * theta)).max()))
    assert err < 1e-10


# ---------------------------------------------------------------- T3 Green's function
def test_homogeneous_greens_function():
    # Sec. 2.1 eq. WaveSecondOrder with s = dm/dt: a point mass source of
    # strength M(t) = 2 dx^2 s(t) / c0 (App. B conversion, summed over the
    # three split densities) radiates p(r, t) = M'(t - r/c) / (4 pi r).
    # Left-point injection delays the recorded sample f^n to t = (n + 1/2) dt.
    shape = (64, 64, 64)
    dx, c = 0.5e-3, 1500.0
    dt = 0.3 * dx / c
    sch = ks.Scheme(shape, dx, dt, c, 1000.0, pml=(10, 10, 10), pml_alpha=2.0)
    # 0.25 MHz = 12 points per wavelength; the remaining error (about 1 %)
    # is second order in omega dt (it falls 2.2x from 0.375 to 0.25 MHz).
    f0 = 0.25e6
    nt = 160
    src = np.array([[32, 32, 32]], dtype=np.int32)
    rec = np.array([[32 + 10, 32, 32], [32, 32 - 12, 32], [32, 32, 32 + 14],
                    [32 + 7, 32 + 7, 32], [32 - 6, 32 + 6, 32 - 6]], dtype=np.int32)
    sig = sc.toneburst(nt, dt, f0)[:, None]
    c0 = np.full(shape, c)
    out = ks.forward(sch, c0, src, sig, np.ones(1), rec, nt)
    tb = 3 / f0
    w, W = 2 * math.pi * f0, 2 * math.pi / tb

    def ds(t):
        t = np.asarray(t)
        v = w * np.cos(w * t) * 0.5 * (1 - np.cos(W * t)) + np.sin(w * t) * 0.5 * W * np.sin(W * t)
        return np.where((t >= 0) & (t <= tb), v, 0.0)

    t = (np.arange(nt) + 0.5) * dt
    for j, r_ in enumerate(rec):
        r = math.dist(r_.tolist(), src[0].tolist()) * dx
        want = dx * dx * ds(t - r / c) / (2 * math.pi * r * c)
        assert rel(out["traces"][:, j], want) < 1.5e-2


# ---------------------------------------------------------------- T4 reversibility
def test_scheme_is_exactly_reversible_without_pml():
    # Sec. 3.1 (time-reversal symmetry): without PML the leapfrog scheme run
    # backwards from (rho^N, -v^{N+1/2}) with the sources removed in reverse
    # order retraces p^N ... p^1.
    prob = sc.make_small(shape=(12, 14, 16), periodic=True, nt=40, n_src=2, n_rec=4)
    sch = ks.scheme_for(prob)
    full = np.ones(prob.shape, dtype=np.uint8)
    fwd = ks.forward(sch, prob.c_true, prob.src_ijk, prob.src_signals(), np.ones(2),
                     prob.rec_ijk, prob.nt, keep_history=full, return_state=True)
    hist = fwd["history"]
    fin = fwd["state"]
    vn = ks.velocity_half_step(sch, fin)
    st = ks.State([-v for v in vn], [r.copy() for r in fin.rho], fin.p.copy())
    c0sq = prob.c_true ** 2
    sig = ks.source_scale(sch, prob.c_true, prob.src_ijk)
    src_idx = ks._idx(prob.src_ijk)
    S = prob.src_signals()
    scale = float(np.abs(hist).max())
    for k in range(1, prob.nt):
        ks.step(sch, st, c0sq, inject=(src_idx, -sig * S[prob.nt - k]))
        assert float(np.abs(st.p.ravel() - hist[prob.nt - k]).max()) < 1e-12 * scale


# ---------------------------------------------------------------- T5 encoding
def test_forward_is_linear_in_encoded_sources():
    # Sec. 3.2: M A^-1 (sum_i w_i s_i) = sum_i w_i M A^-1 s_i
    prob = sc.make_small(shape=(12, 14, 16), nt=30, n_src=3, n_rec=6)
    sch = ks.scheme_for(prob)
    S = prob.src_signals() * np.array([1.0, 0.7, -1.3])
    w = oracle.rademacher(11, 3).astype(np.float64)
    enc = ks.forward(sch, prob.c_true, prob.src_ijk, S, w, prob.rec_ijk, prob.nt)["traces"]
    acc = np.zeros_like(enc)
    for i in range(3):
        e = np.zeros(3)
        e[i] = 1.0
        acc += w[i] * ks.forward(sch, prob.c_true, prob.src_ijk, S, e, prob.rec_ijk, prob.nt)["traces"]
    assert rel(enc, acc) < 1e-12


def test_encoded_gradient_averaged_over_all_signs_is_the_full_sum():
    # App. E: g_E = grad J + sum_{i != j} w_i w_j X_ij; averaging over all 2^ns
    # Rademacher patterns cancels every cross-talk term exactly.
    prob = sc.make_small(shape=(12, 14, 16), nt=30, n_src=3, n_rec=6, layer=2)
    sch = ks.scheme_for(prob)
    S = prob.src_signals()
    obs_i = [ks.forward(sch, prob.c_true, prob.src_ijk, S, np.eye(3)[i], prob.rec_ijk,
                        prob.nt)["traces"] for i in range(3)]
    grads = []
    for i in range(3):
        _, G, _ = ks.tr_gradient(sch, prob.c_eval, prob.src_ijk, S, np.eye(3)[i], prob.rec_ijk,
                                 obs_i[i], prob.gamma, prob.boundary, prob.nt)
        grads.append(G)
    want = sum(grads)
    acc = np.zeros(prob.shape)
    for bits in range(8):
        w = np.array([1.0 if (bits >> i) & 1 else -1.0 for i in range(3)])
        obs = sum(w[i] * obs_i[i] for i in range(3))
        _, G, _ = ks.tr_gradient(sch, prob.c_eval, prob.src_ijk, S, w, prob.rec_ijk, obs,
                                 prob.gamma, prob.boundary, prob.nt)
        acc += G / 8.0
    assert rel(acc, want) < 1e-11


# ---------------------------------------------------------------- T6/T7 exact adjoint
def _small_pml():
    prob = sc.make_small(shape=(12, 14, 16), pml=2, nt=36, n_src=2, n_rec=6, layer=2)
    sch = ks.scheme_for(prob)
    S = prob.src_signals()
    w = np.array([1.0, -1.0])
    obs = ks.forward(sch, prob.c_true, prob.src_ijk, S, w, prob.rec_ijk, prob.nt)["traces"]
    return prob, sch, S, w, obs


def test_dot_product_tangent_vs_transpose():
    # <J dc, r> = <dc, J^T r> for the linearised forward map c0 -> traces
    prob, sch, S, w, obs = _small_pml()
    rng = np.random.default_rng(5)
    dc = rng.standard_normal(prob.shape) * prob.gamma
    r = rng.standard_normal((prob.nt, prob.n_rec))
    jdc = ks.tangent_linear_traces(sch, prob.c_eval, dc, prob.src_ijk, S, w, prob.rec_ijk, prob.nt)
    _, jtr, _ = ks.exact_adjoint_gradient(sch, prob.c_eval, prob.src_ijk, S, w, prob.rec_ijk,
                                          None, prob.nt, residual=r)
    lhs = float(np.sum(jdc * r))
    rhs = float(np.sum(dc * jtr))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), abs(rhs))


def test_exact_adjoint_matches_central_finite_differences():
    # Sec. 2.3: the adjoint-state gradient is dD/dc0 (eq. FWI with D = 1/2||f - f^delta||^2)
    prob, sch, S, w, obs = _small_pml()
    _, G, _ = ks.exact_adjoint_gradient(sch, prob.c_eval, prob.src_ijk, S, w, prob.rec_ijk, obs,
                                        prob.nt)
    gi = np.argwhere(prob.gamma)
    rng = np.random.default_rng(9)
    h = 1e-3
    for t in rng.choice(len(gi), size=4, replace=False):
        iz, iy, ix = gi[t]
        cp = prob.c_eval.copy()
        cm = prob.c_eval.copy()
        cp[iz, iy, ix] += h
        cm[iz, iy, ix] -= h
        Dp = ks.misfit_and_adjoint_source(
            ks.forward(sch, cp, prob.src_ijk, S, w, prob.rec_ijk, prob.nt)["traces"], obs)[0]
        Dm = ks.misfit_and_adjoint_source(
            ks.forward(sch, cm, prob.src_ijk, S, w, prob.rec_ijk, prob.nt)["traces"], obs)[0]
        fd = (Dp - Dm) / (2 * h)
        assert abs(fd - G[iz, iy, ix]) <= 1e-6 * abs(G[iz, iy, ix]) + 1e-30


def test_stored_history_gradient_equals_exact_adjoint_without_pml():
    # eq. Gradc0 discretised as in Alg. 1 (2/c0^3 times the second time
    # difference of p against the adjoint field) is the exact discrete
    # gradient when there is no PML.
    prob = sc.make_small(shape=(12, 14, 16), periodic=True, nt=36, n_src=2, n_rec=6, layer=2)
    sch = ks.scheme_for(prob)
    S = prob.src_signals()
    w = np.array([1.0, -1.0])
    obs = ks.forward(sch, prob.c_true, prob.src_ijk, S, w, prob.rec_ijk, prob.nt)["traces"]
    D1, Gx, _ = ks.exact_adjoint_gradient(sch, prob.c_eval, prob.src_ijk, S, w, prob.rec_ijk, obs,
                                          prob.nt)
    D2, Gf, _ = ks.full_gradient(sch, prob.c_eval, prob.src_ijk, S, w, prob.rec_ijk, obs,
                                 prob.gamma, prob.nt)
    g = prob.gamma.astype(bool)
    assert abs(D1 - D2) <= 1e-13 * D1
    assert rel(Gf[g], Gx[g]) < 1e-11


def test_tr_gradient_is_exact_when_time_reversal_is_exact():
    # Sec. 3.1: p_tr(t) = p(T - t) when the re-simulation is exact; without
    # PML, started from the final state with the sources removed in reverse,
    # the TR gradient of Alg. 1 equals the stored-history gradient.
    prob = sc.make_small(shape=(12, 14, 16), periodic=True, nt=36, n_src=2, n_rec=6, layer=2)
    sch = ks.scheme_for(prob)
    S = prob.src_signals()
    w = np.array([1.0, -1.0])
    obs = ks.forward(sch, prob.c_true, prob.src_ijk, S, w, prob.rec_ijk, prob.nt)["traces"]
    _, Gf, _ = ks.full_gradient(sch, prob.c_eval, prob.src_ijk, S, w, prob.rec_ijk, obs,
                                prob.gamma, prob.nt)
    _, Gt, _ = ks.tr_gradient(sch, prob.c_eval, prob.src_ijk, S, w, prob.rec_ijk, obs,
                              prob.gamma, prob.boundary, prob.nt, tr_init="final_state",
                              reinject_sources=True)
    g = prob.gamma.astype(bool)
    assert rel(Gt[g], Gf[g]) < 1e-10


def test_pml_absorbs_outgoing_waves():
    # App. B: the PML damps outgoing waves.  After a pulse has left the
    # interior, the field energy falls by orders of magnitude; without PML
    # (periodic box) it does not.
    shape = (32, 32, 32)
    dx = 0.5e-3
    c = 1500.0
    dt = 0.3 * dx / 1800.0
    nt = 260
    src = np.array([[16, 16, 16]], dtype=np.int32)
    rec = np.array([[18, 16, 16]], dtype=np.int32)
    sig = sc.toneburst(nt, dt, 1.0e6)[:, None]
    c0 = np.full(shape, c)
    energy = {}
    for P in (0, 4, 8):
        sch = ks.Scheme(shape, dx, dt, 1800.0, 1000.0, pml=(P, P, P))
        out = ks.forward(sch, c0, src, sig, np.ones(1), rec, nt, return_state=True)
        energy[P] = float(np.sum(out["state"].p ** 2))
        peak = float(np.max(np.abs(out["traces"])))
        energy[(P, "peak")] = peak
    assert energy[8] < 1e-3 * energy[0]
    assert energy[8] < 0.5 * energy[4]          # a thicker layer absorbs more


def test_tr_gradient_error_falls_with_boundary_layer_thickness():
    # Sec. 4.2 / Table TRGrad: the TR gradient's error against the stored
    # full-field gradient falls fast as the imposed boundary layer thickens
    # (the paper: 22.8 % -> 5.6 % -> 0.90 % for 1 / 2 / 4 voxels).
    errs = []
    for layer in (1, 2, 4):
        prob = sc.make_small(shape=(32, 32, 32), pml=4, nt=150, n_src=2, n_rec=12, layer=layer)
        sch = ks.scheme_for(prob)
        S = prob.src_signals()
        w = np.array([1.0, -1.0])
        obs = ks.forward(sch, prob.c_true, prob.src_ijk, S, w, prob.rec_ijk, prob.nt)["traces"]
        _, Gf, _ = ks.full_gradient(sch, prob.c_eval, prob.src_ijk, S, w, prob.rec_ijk, obs,
                                    prob.gamma, prob.nt)
        _, Gt, _ = ks.tr_gradient(sch, prob.c_eval, prob.src_ijk, S, w, prob.rec_ijk, obs,
                                  prob.gamma, prob.boundary, prob.nt)
        g = prob.gamma.astype(bool)
        errs.append(rel(Gt[g], Gf[g]))
    assert errs[0] > 1.5 * errs[1] > 1.5 * 1.5 * errs[2]


# ---------------------------------------------------------------- delayed source encoding
def test_delayed_encoding_removes_cross_talk():
    # App. E: g_E^tau = grad J + sum_{i != j} w_i w_j X_ij, and X_ij vanishes
    # as the delay between sources i and j outgrows the time the field needs
    # to leave the medium.  Two sources on a 16^3 grid with PML: the gap
    # between the encoded gradient and the sum of the single-source gradients
    # falls monotonically with the delay (0, 160, 240 steps).
    prob = sc.make_small(shape=(16, 16, 16), pml=4, nt=480, n_src=2, n_rec=8, layer=2)
    sch = ks.scheme_for(prob)
    T1 = 240
    base = sc.toneburst(T1, prob.dt, 1.0e6)
    w = np.array([1.0, -1.0])
    g = prob.gamma.astype(bool)

    def gap(delay):
        S = np.zeros((prob.nt, 2))
        S[:T1, 0] = base
        S[delay:delay + T1, 1] = base
        f_i = [ks.forward(sch, prob.c_true, prob.src_ijk, S, np.eye(2)[i], prob.rec_ijk, prob.nt)["traces"]
               for i in range(2)]

        def grad(weights, obs):
            return ks.exact_adjoint_gradient(sch, prob.c_eval, prob.src_ijk, S, weights, prob.rec_ijk, obs,
                                             prob.nt)[1]

        single = grad(np.eye(2)[0], f_i[0]) + grad(np.eye(2)[1], f_i[1])
        enc = grad(w, w[0] * f_i[0] + w[1] * f_i[1])
        return rel(enc[g], single[g])

    e0, e1, e2 = gap(0), gap(160), gap(240)
    assert e0 > e1 > e2
    assert e2 < 1e-2 and e0 > 20 * e2


def test_uniform_delay_shifts_traces_exactly():
    # eq. DelaySE with one delay d for every source: the scheme is the same
    # operation at every step and starts from zero, so the traces are the
    # undelayed traces d steps later, bit for bit, and zero before
    prob = sc.make_small(shape=(16, 16, 16), pml=4, nt=40, n_src=2, n_rec=8, layer=2)
    sch = ks.scheme_for(prob)
    S = prob.src_signals()
    w = ks.rademacher(prob.enc_seed, prob.n_src)
    d = 7
    f0 = ks.forward(sch, prob.c_true, prob.src_ijk, S, w, prob.rec_ijk, prob.nt)["traces"]
    Sd = ks.delayed_signals(S, [d] * prob.n_src, prob.nt + d)
    f1 = ks.forward(sch, prob.c_true, prob.src_ijk, Sd, w, prob.rec_ijk, prob.nt + d)["traces"]
    assert np.all(f1[:d] == 0)
    assert np.array_equal(f1[d:], f0)


def test_per_source_delays_superpose():
    # linearity and time invariance: the delayed encoded traces are the sum of
    # each source's own traces shifted by its delay and weighted by w_i
    prob = sc.make_small(shape=(16, 16, 16), pml=4, nt=30, n_src=3, n_rec=8, layer=2)
    sch = ks.scheme_for(prob)
    S = prob.src_signals()
    w = np.array([1, -1, 1], dtype=np.int8)
    d = [0, 5, 11]
    N = prob.nt + 11
    enc = ks.forward(sch, prob.c_true, prob.src_ijk, ks.delayed_signals(S, d, N), w, prob.rec_ijk, N)["traces"]
    want = np.zeros_like(enc)
    Sp = np.zeros((N, 3))
    Sp[:prob.nt] = S
    for i in range(3):
        e = np.zeros(3)
        e[i] = 1.0
        fi = ks.forward(sch, prob.c_true, prob.src_ijk, Sp[:N - d[i]], e, prob.rec_ijk, N - d[i])["traces"]
        want[d[i]:] += w[i] * fi
    assert rel(enc, want) < 1e-12
