"""GPU parity: the HIP path through the C-ABI against the FP64 oracle.

Sizes span several tiles with a ragged tail (the half spectrum along x has
nx/2 + 1 columns; axis tiles are 8 (FP32) / 4 (FP64) columns wide) and the
radices 2, 3, 4, 5, 7, 8.  Tolerances: FP64 builds at round-off level; FP32
rel l2 <= 1e-4 on traces and <= 1e-3 on gradients.
"""

import numpy as np
import pytest
import torch

import oracle
from oracle import kspace as ks
from synth import make_small
from synth.configs import random_traces

pytestmark = pytest.mark.gpu


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def handle(prob, precision, batch=1):
    from paper_2102_00755_amd.fwi import Handle
    return Handle.from_problem(prob, batch=batch, precision=precision)


SHAPES = [(16, 24, 32), (24, 40, 48), (24, 56, 112)]


@pytest.mark.parametrize("precision,tol", [(8, 1e-12), (4, 2e-6)])
@pytest.mark.parametrize("shape", SHAPES)
def test_derivative_matches_oracle(shape, precision, tol):
    print(f"derivative shape={shape} precision={precision}", flush=True)
    prob = make_small(shape=shape, nt=4, precision=precision)
    h = handle(prob, precision)
    sch = ks.scheme_for(prob)
    rng = np.random.default_rng(3)
    g = rng.standard_normal(shape)
    for axis in range(3):
        for sign in (+1, -1):
            got = h.derivative(torch.from_numpy(g), axis, sign).cpu().numpy()
            want = sch.d_plus(g, axis) if sign > 0 else sch.d_minus(g, axis)
            assert rel(got, want) < tol, (axis, sign, rel(got, want))
    h.close()


# every FFT length added for larger and PML-padded grids (192, 240, 320, 384,
# 480, 512) on every axis it can take: x (as nx/2), y and z
LONG_SHAPES = [(16, 192, 480), (320, 16, 768), (16, 480, 1024), (512, 16, 640), (240, 384, 16)]


@pytest.mark.parametrize("precision,tol", [(8, 1e-12), (4, 2e-6)])
@pytest.mark.parametrize("shape", LONG_SHAPES)
def test_derivative_long_lengths_match_oracle(shape, precision, tol):
    print(f"derivative shape={shape} precision={precision}", flush=True)
    prob = make_small(shape=shape, nt=2, precision=precision, r_transducer=5.0, r_gamma=3.0)
    h = handle(prob, precision)
    sch = ks.scheme_for(prob)
    rng = np.random.default_rng(4)
    g = rng.standard_normal(shape)
    for axis in range(3):
        for sign in (+1, -1):
            got = h.derivative(torch.from_numpy(g), axis, sign).cpu().numpy()
            want = sch.d_plus(g, axis) if sign > 0 else sch.d_minus(g, axis)
            assert rel(got, want) < tol, (axis, sign, rel(got, want))
    h.close()


def test_long_length_gradient_matches_oracle():
    # a TR gradient whose x passes run at nx/2 = 240 and y passes at 192
    shape = (24, 192, 480)
    prob = make_small(shape=shape, nt=24, n_src=2, n_rec=12, layer=2, precision=8, r_transducer=8.0,
                      r_gamma=5.0)
    print(f"gradient shape={shape}", flush=True)
    sch = ks.scheme_for(prob)
    w, S = _inputs(prob)
    obs = random_traces(prob.nt, prob.n_rec, seed=5, scale=1e-3)
    D, G, _ = ks.tr_gradient(sch, prob.c_eval, prob.src_ijk, S, w, prob.rec_ijk, obs, prob.gamma, prob.boundary,
                             prob.nt)
    traces = ks.forward(sch, prob.c_eval, prob.src_ijk, S, w, prob.rec_ijk, prob.nt)["traces"]
    h = handle(prob, 8)
    got_tr = h.forward(torch.from_numpy(prob.c_eval), torch.from_numpy(S), torch.from_numpy(w))[0].cpu().numpy()
    assert rel(got_tr, traces) < 1e-10
    mis, grad = h.gradient(torch.from_numpy(prob.c_eval), torch.from_numpy(S), torch.from_numpy(w),
                           torch.from_numpy(obs))
    g = prob.gamma.astype(bool)
    assert abs(float(mis[0]) - D) <= 1e-10 * D
    assert rel(grad[0].cpu().numpy()[g], G[g]) < 1e-9
    h.close()


@pytest.mark.parametrize("precision,ttol,gtol", [(8, 1e-10, 1e-9), (4, 1e-4, 1e-3)])
@pytest.mark.parametrize("shape", [(32, 32, 64), (32, 96, 448)])
def test_radix_plan_1_matches_oracle(shape, precision, ttol, gtol):
    # every pass kind with radix plan 1, on lengths whose two plans differ:
    # 32 (8*4 / 4*8), 96 (3*8*4 / 3*4*8) and nx/2 = 224 (the full-size x length)
    print(f"radix plan 1 shape={shape} precision={precision}", flush=True)
    prob = make_small(shape=shape, nt=30, n_src=2, n_rec=12, layer=2, precision=precision)
    w, S = _inputs(prob)
    sch = ks.scheme_for(prob)
    obs = random_traces(prob.nt, prob.n_rec, seed=6, scale=1e-3)   # a residual large against rounding
    traces = ks.forward(sch, prob.c_eval, prob.src_ijk, S, w, prob.rec_ijk, prob.nt)["traces"]
    D, G, _ = ks.tr_gradient(sch, prob.c_eval, prob.src_ijk, S, w, prob.rec_ijk, obs, prob.gamma,
                             prob.boundary, prob.nt)
    h = handle(prob, precision)
    h.tuning = {"y_plan": 1, "zm_plan": 1, "zp_plan": 1, "x_plan": 1}
    got_tr = h.forward(torch.from_numpy(prob.c_eval), torch.from_numpy(S), torch.from_numpy(w))[0].cpu().numpy()
    assert rel(got_tr, traces) < ttol
    mis, grad = h.gradient(torch.from_numpy(prob.c_eval), torch.from_numpy(S), torch.from_numpy(w),
                           torch.from_numpy(obs))
    assert abs(float(mis[0]) - D) <= ttol * D
    gmask = prob.gamma.astype(bool)
    assert rel(grad[0].cpu().numpy()[gmask], G[gmask]) < gtol
    h.close()


def _inputs(prob, seed=0):
    w = oracle.rademacher(prob.enc_seed, prob.n_src)
    S = prob.src_signals()
    return w, S


@pytest.mark.parametrize("precision,tol", [(8, 1e-10), (4, 1e-4)])
@pytest.mark.parametrize("shape", SHAPES[:2])
def test_forward_matches_oracle(shape, precision, tol):
    print(f"forward shape={shape} precision={precision}", flush=True)
    prob = make_small(shape=shape, nt=60, n_src=3, n_rec=12, precision=precision)
    w, S = _inputs(prob)
    sch = ks.scheme_for(prob)
    want = ks.forward(sch, prob.c_true, prob.src_ijk, S, w, prob.rec_ijk, prob.nt)["traces"]
    h = handle(prob, precision)
    got = h.forward(torch.from_numpy(prob.c_true), torch.from_numpy(S), torch.from_numpy(w))
    got = got[0].cpu().numpy()
    assert rel(got, want) < tol, rel(got, want)
    h.close()


@pytest.mark.parametrize("precision,ttol,gtol", [(8, 1e-10, 1e-9), (4, 1e-4, 1e-3)])
@pytest.mark.parametrize("shape", SHAPES[:2])
def test_tr_gradient_matches_oracle(shape, precision, ttol, gtol):
    print(f"gradient shape={shape} precision={precision}", flush=True)
    prob = make_small(shape=shape, nt=60, n_src=3, n_rec=12, layer=2, precision=precision)
    w, S = _inputs(prob)
    sch = ks.scheme_for(prob)
    obs = ks.forward(sch, prob.c_true, prob.src_ijk, S, w, prob.rec_ijk, prob.nt)["traces"]
    D, G, _ = ks.tr_gradient(sch, prob.c_eval, prob.src_ijk, S, w, prob.rec_ijk, obs, prob.gamma,
                             prob.boundary, prob.nt)
    h = handle(prob, precision)
    mis, grad = h.gradient(torch.from_numpy(prob.c_eval), torch.from_numpy(S), torch.from_numpy(w),
                           torch.from_numpy(obs))
    assert abs(float(mis[0]) - D) <= ttol * D
    gmask = prob.gamma.astype(bool)
    got = grad[0].cpu().numpy()
    assert np.all(got[~gmask] == 0)
    assert rel(got[gmask], G[gmask]) < gtol, rel(got[gmask], G[gmask])
    h.close()


@pytest.mark.parametrize("precision,tol", [(8, 1e-9), (4, 1e-3)])
def test_backward_matches_oracle(precision, tol):
    shape = SHAPES[1]
    prob = make_small(shape=shape, nt=50, n_src=2, n_rec=12, layer=2, precision=precision)
    w, S = _inputs(prob)
    sch = ks.scheme_for(prob)
    r = random_traces(prob.nt, prob.n_rec, seed=11, scale=1e-3)
    D, G, _ = ks.tr_gradient(sch, prob.c_eval, prob.src_ijk, S, w, prob.rec_ijk, None, prob.gamma,
                             prob.boundary, prob.nt, residual=r)
    h = handle(prob, precision)
    c = torch.from_numpy(prob.c_eval)
    h.forward(c, torch.from_numpy(S), torch.from_numpy(w), save_tape=True)
    mis, grad = h.backward(c, torch.from_numpy(r))
    gmask = prob.gamma.astype(bool)
    assert abs(float(mis[0]) - D) <= 1e-6 * D
    assert rel(grad[0].cpu().numpy()[gmask], G[gmask]) < tol
    h.close()


def test_batched_equals_individual():
    shape = SHAPES[0]
    probs = [make_small(shape=shape, nt=40, n_src=2, n_rec=12, layer=2, seed=s, precision=4)
             for s in (21, 22, 23)]
    base = probs[0]
    h1 = handle(base, 4, batch=1)
    h3 = handle(base, 4, batch=3)
    S = base.src_signals()
    cs, ws, obss = [], [], []
    for i, p in enumerate(probs):
        cs.append(p.c_eval)
        ws.append(oracle.rademacher(100 + i, base.n_src))
        obss.append(random_traces(base.nt, base.n_rec, seed=50 + i, scale=1e-3))
    c = torch.from_numpy(np.stack(cs))
    w = torch.from_numpy(np.stack(ws))
    obs = torch.from_numpy(np.stack(obss))
    Sb = torch.from_numpy(np.stack([S] * 3))
    mb, gb = h3.gradient(c, Sb, w, obs)
    for i in range(3):
        m1, g1 = h1.gradient(c[i], Sb[i], w[i], obs[i])
        assert torch.equal(g1[0].cpu(), gb[i].cpu())
        assert float(m1[0]) == float(mb[i])
    h1.close()
    h3.close()


def test_batched_call_broadcasts_shared_inputs():
    # one unbatched signal / weight / data array with a batched c is shared by
    # every problem (expanded by the binding) and gives what the explicitly
    # repeated arrays give; a leading dimension that is neither 1 nor B is
    # rejected before anything is launched
    shape = SHAPES[0]
    probs = [make_small(shape=shape, nt=30, n_src=2, n_rec=12, layer=2, seed=s, precision=4) for s in (31, 32)]
    base = probs[0]
    h = handle(base, 4, batch=2)
    c = torch.from_numpy(np.stack([p.c_eval for p in probs]))
    S = torch.from_numpy(base.src_signals())
    w = torch.from_numpy(oracle.rademacher(7, base.n_src))
    obs = torch.from_numpy(random_traces(base.nt, base.n_rec, seed=5, scale=1e-3))
    m_sh, g_sh = h.gradient(c, S, w, obs)
    m_ex, g_ex = h.gradient(c, S.expand(2, *S.shape), w.expand(2, *w.shape), obs.expand(2, *obs.shape))
    assert torch.equal(g_sh.cpu(), g_ex.cpu()) and torch.equal(m_sh.cpu(), m_ex.cpu())
    t_sh = h.forward(c, S, w)
    t_ex = h.forward(c, S.expand(2, *S.shape), w.expand(2, *w.shape))
    assert torch.equal(t_sh.cpu(), t_ex.cpu())
    c3 = torch.from_numpy(np.stack([p.c_eval for p in probs] + [base.c_eval]))
    with pytest.raises(ValueError):
        h.gradient(c3[:2], S.expand(3, *S.shape), w, obs)
    with pytest.raises(ValueError):
        h.forward(c3[:2], S, w.expand(3, *w.shape))
    with pytest.raises(ValueError):
        h.backward(c3[:2], obs.expand(3, *obs.shape))
    h.close()


@pytest.mark.parametrize("precision,tol", [(8, 1e-9), (4, 1e-3)])
def test_tr_gradient_from_final_state_matches_oracle(precision, tol):
    # reading 11: TR started from (rho^N, -v^{N+1/2}) instead of the zero interior
    shape = SHAPES[1]
    prob = make_small(shape=shape, nt=50, n_src=3, n_rec=12, layer=2, precision=precision)
    w, S = _inputs(prob)
    sch = ks.scheme_for(prob)
    obs = random_traces(prob.nt, prob.n_rec, seed=5, scale=1e-3)
    D, G, _ = ks.tr_gradient(sch, prob.c_eval, prob.src_ijk, S, w, prob.rec_ijk, obs, prob.gamma,
                             prob.boundary, prob.nt, tr_init="final_state")
    D0, G0, _ = ks.tr_gradient(sch, prob.c_eval, prob.src_ijk, S, w, prob.rec_ijk, obs, prob.gamma,
                               prob.boundary, prob.nt)
    g = prob.gamma.astype(bool)
    assert rel(G0[g], G[g]) > 10 * tol          # the two initialisations differ
    h = handle(prob, precision)
    h.tr_final_state = True
    mis, grad = h.gradient(torch.from_numpy(prob.c_eval), torch.from_numpy(S), torch.from_numpy(w),
                           torch.from_numpy(obs))
    assert abs(float(mis[0]) - D) <= 1e-6 * D
    assert rel(grad[0].cpu().numpy()[g], G[g]) < tol
    h.close()


@pytest.mark.parametrize("nt", [1, 2, 3])
def test_few_time_steps_match_oracle(nt):
    # degenerate horizons of Alg. 1: N = 1 has no TR pre-step and only the
    # adjoint-only iterations, N = 2 no paired iteration, N = 3 one
    print(f"few steps nt={nt}", flush=True)
    prob = make_small(shape=SHAPES[1], nt=nt, n_src=2, n_rec=12, layer=1, precision=8)
    w, _ = _inputs(prob)
    S = random_traces(prob.nt, prob.n_src, seed=15)   # nonzero from the first step
    sch = ks.scheme_for(prob)
    r = random_traces(prob.nt, prob.n_rec, seed=13, scale=1e-3)
    D, G, _ = ks.tr_gradient(sch, prob.c_eval, prob.src_ijk, S, w, prob.rec_ijk, None, prob.gamma,
                             prob.boundary, prob.nt, residual=r)
    h = handle(prob, 8)
    c = torch.from_numpy(prob.c_eval)
    h.forward(c, torch.from_numpy(S), torch.from_numpy(w), save_tape=True)
    mis, grad = h.backward(c, torch.from_numpy(r))
    gmask = prob.gamma.astype(bool)
    assert abs(float(mis[0]) - D) <= 1e-12 * D
    got = grad[0].cpu().numpy()
    if nt == 1:   # p_adj^(0) is the injection alone: zero on Gamma, so G = 0
        assert np.all(G == 0) and np.all(got == 0)
    else:
        assert np.linalg.norm(G[gmask]) > 0
        assert rel(got[gmask], G[gmask]) < 1e-9
    h.close()
