"""GPU parity of the lossy path (power-law absorption, Sec. 2.1; TR with the
absorption sign switched, Sec. 3.1) against the FP64 lossy oracle, through
the C-ABI.  Tolerances as for the lossless path: FP64 at round-off level;
FP32 rel l2 <= 1e-4 on traces and <= 1e-3 on gradients.
"""

import numpy as np
import pytest
import torch

import oracle
from oracle import kspace as ks
from oracle import lossy as lo
from synth import make_small
from synth.configs import random_traces

pytestmark = pytest.mark.gpu

SHAPES = [(16, 24, 32), (24, 40, 48)]
# 15 dB MHz^-1.5 cm^-1: strong enough that the traces differ from the
# lossless ones by percent on these small grids
A_DB = 15.0


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def handle(prob, precision, batch=1):
    from paper_2102_00755_amd.fwi import Handle
    return Handle.from_problem(prob, batch=batch, precision=precision)


def _inputs(prob):
    return oracle.rademacher(prob.enc_seed, prob.n_src), prob.src_signals()


@pytest.mark.parametrize("precision,tol", [(8, 1e-10), (4, 1e-4)])
@pytest.mark.parametrize("shape,y", [(SHAPES[0], 1.5), (SHAPES[1], 0.6)])
def test_lossy_forward_matches_oracle(shape, y, precision, tol):
    print(f"lossy forward shape={shape} y={y} precision={precision}", flush=True)
    prob = make_small(shape=shape, nt=60, n_src=3, n_rec=12, precision=precision)
    w, S = _inputs(prob)
    sch = ks.scheme_for(prob)
    a0 = lo.db_to_neper(A_DB, y)
    want = lo.forward(lo.Lossy(sch, a0, y), prob.c_true, prob.src_ijk, S, w, prob.rec_ijk, prob.nt)["traces"]
    lossless = ks.forward(sch, prob.c_true, prob.src_ijk, S, w, prob.rec_ijk, prob.nt)["traces"]
    assert rel(want, lossless) > 1e-2          # the case exercises the absorption
    h = handle(prob, precision)
    h.set_absorption(a0, y)
    got = h.forward(torch.from_numpy(prob.c_true), torch.from_numpy(S), torch.from_numpy(w))[0].cpu().numpy()
    assert rel(got, want) < tol, rel(got, want)
    h.close()


@pytest.mark.parametrize("precision,ttol,gtol", [(8, 1e-10, 1e-9), (4, 1e-4, 1e-3)])
@pytest.mark.parametrize("shape", SHAPES)
def test_lossy_tr_gradient_matches_oracle(shape, precision, ttol, gtol):
    print(f"lossy gradient shape={shape} precision={precision}", flush=True)
    prob = make_small(shape=shape, nt=60, n_src=3, n_rec=12, layer=2, precision=precision)
    w, S = _inputs(prob)
    sch = ks.scheme_for(prob)
    a0 = lo.db_to_neper(A_DB, 1.5)
    los = lo.Lossy(sch, a0, 1.5)
    obs = lo.forward(los, prob.c_true, prob.src_ijk, S, w, prob.rec_ijk, prob.nt)["traces"]
    D, G, _ = lo.tr_gradient(los, prob.c_eval, prob.src_ijk, S, w, prob.rec_ijk, obs, prob.gamma, prob.boundary,
                             prob.nt)
    h = handle(prob, precision)
    h.set_absorption(a0, 1.5)
    mis, grad = h.gradient(torch.from_numpy(prob.c_eval), torch.from_numpy(S), torch.from_numpy(w),
                           torch.from_numpy(obs))
    assert abs(float(mis[0]) - D) <= ttol * D
    gmask = prob.gamma.astype(bool)
    got = grad[0].cpu().numpy()
    assert np.all(got[~gmask] == 0)
    assert rel(got[gmask], G[gmask]) < gtol, rel(got[gmask], G[gmask])
    h.close()


def test_lossy_gradient_without_flip_and_with_alpha0_field():
    # per-voxel alpha0 (Sec. 2.1 writes alpha0(x)) and the TR without the sign
    # switch, FP64
    shape = SHAPES[0]
    prob = make_small(shape=shape, nt=50, n_src=2, n_rec=12, layer=2, precision=8)
    w, S = _inputs(prob)
    sch = ks.scheme_for(prob)
    rng = np.random.default_rng(17)
    a0f = lo.db_to_neper(A_DB, 1.5) * rng.uniform(0.5, 1.5, size=shape)
    los = lo.Lossy(sch, a0f, 1.5)
    r = random_traces(prob.nt, prob.n_rec, seed=12, scale=1e-3)
    D, G, _ = lo.tr_gradient(los, prob.c_eval, prob.src_ijk, S, w, prob.rec_ijk, None, prob.gamma, prob.boundary,
                             prob.nt, residual=r, flip_tau=False)
    h = handle(prob, 8)
    h.set_absorption(1.0, 1.5, field=torch.from_numpy(a0f), tr_flip=False)
    c = torch.from_numpy(prob.c_eval)
    h.forward(c, torch.from_numpy(S), torch.from_numpy(w), save_tape=True)
    mis, grad = h.backward(c, torch.from_numpy(r))
    gmask = prob.gamma.astype(bool)
    assert abs(float(mis[0]) - D) <= 1e-10 * D
    assert rel(grad[0].cpu().numpy()[gmask], G[gmask]) < 1e-9
    h.close()


def test_uniform_field_equals_scalar_and_off_restores_lossless():
    shape = SHAPES[0]
    prob = make_small(shape=shape, nt=40, n_src=2, n_rec=12, layer=2, precision=4)
    w, S = _inputs(prob)
    c = torch.from_numpy(prob.c_true)
    Sg, wg = torch.from_numpy(S), torch.from_numpy(w)
    a0 = lo.db_to_neper(A_DB, 1.5)
    h = handle(prob, 4)
    plain = h.forward(c, Sg, wg).clone()
    h.set_absorption(a0, 1.5)
    scalar = h.forward(c, Sg, wg).clone()
    h.set_absorption(0.0, 1.5, field=torch.full(prob.shape, a0, dtype=torch.float64))
    field = h.forward(c, Sg, wg).clone()
    h.set_absorption(0.0)
    again = h.forward(c, Sg, wg).clone()
    assert torch.equal(scalar, field)
    assert torch.equal(plain, again)
    assert not torch.equal(plain, scalar)
    h.close()


def test_lossy_batched_equals_individual():
    shape = SHAPES[0]
    probs = [make_small(shape=shape, nt=40, n_src=2, n_rec=12, layer=2, seed=s, precision=4) for s in (31, 32)]
    base = probs[0]
    a0 = lo.db_to_neper(A_DB, 1.5)
    h1 = handle(base, 4, batch=1)
    h2 = handle(base, 4, batch=2)
    for h in (h1, h2):
        h.set_absorption(a0, 1.5)
    S = base.src_signals()
    c = torch.from_numpy(np.stack([p.c_eval for p in probs]))
    w = torch.from_numpy(np.stack([oracle.rademacher(200 + i, base.n_src) for i in range(2)]))
    obs = torch.from_numpy(np.stack([random_traces(base.nt, base.n_rec, seed=60 + i, scale=1e-3)
                                     for i in range(2)]))
    Sb = torch.from_numpy(np.stack([S] * 2))
    mb, gb = h2.gradient(c, Sb, w, obs)
    for i in range(2):
        m1, g1 = h1.gradient(c[i], Sb[i], w[i], obs[i])
        assert torch.equal(g1[0].cpu(), gb[i].cpu())
        assert float(m1[0]) == float(mb[i])
    h1.close()
    h2.close()


def test_absorption_argument_errors():
    from paper_2102_00755_amd.fwi import FwiError
    shape = SHAPES[0]
    prob = make_small(shape=shape, nt=8, n_src=2, n_rec=12, layer=2, precision=4)
    h = handle(prob, 4)
    for a0, y in ((1e-3, 1.0), (1e-3, 2.0), (1e-3, 0.0), (-1.0, 1.5), (float("nan"), 1.5)):
        with pytest.raises(FwiError):
            h.set_absorption(a0, y)
    w, S = _inputs(prob)
    c, Sg, wg = torch.from_numpy(prob.c_true), torch.from_numpy(S), torch.from_numpy(w)
    # a rejected call leaves the previous absorption (and its field) in use
    a0 = lo.db_to_neper(A_DB, 1.5)
    h.set_absorption(0.0, 1.5, field=torch.full(prob.shape, a0, dtype=torch.float64))
    before = h.forward(c, Sg, wg).clone()
    with pytest.raises(FwiError):
        h.set_absorption(0.0, 1.0, field=torch.full(prob.shape, 3 * a0, dtype=torch.float64))
    torch.cuda.empty_cache()
    assert torch.equal(h.forward(c, Sg, wg), before)
    h.set_absorption(a0, 1.5)
    h.tr_final_state = True
    obs = random_traces(prob.nt, prob.n_rec, seed=3, scale=1e-3)
    with pytest.raises(FwiError):
        h.gradient(torch.from_numpy(prob.c_eval), torch.from_numpy(S), torch.from_numpy(w), torch.from_numpy(obs))
    h.close()


@pytest.mark.parametrize("nt", [1, 2, 3])
def test_lossy_few_time_steps_match_oracle(nt):
    print(f"lossy few steps nt={nt}", flush=True)
    prob = make_small(shape=SHAPES[1], nt=nt, n_src=2, n_rec=12, layer=1, precision=8)
    w, _ = _inputs(prob)
    S = random_traces(prob.nt, prob.n_src, seed=15)   # nonzero from the first step
    sch = ks.scheme_for(prob)
    a0 = lo.db_to_neper(A_DB, 1.5)
    los = lo.Lossy(sch, a0, 1.5)
    r = random_traces(prob.nt, prob.n_rec, seed=14, scale=1e-3)
    D, G, _ = lo.tr_gradient(los, prob.c_eval, prob.src_ijk, S, w, prob.rec_ijk, None, prob.gamma, prob.boundary,
                             prob.nt, residual=r)
    h = handle(prob, 8)
    h.set_absorption(a0, 1.5)
    c = torch.from_numpy(prob.c_eval)
    h.forward(c, torch.from_numpy(S), torch.from_numpy(w), save_tape=True)
    mis, grad = h.backward(c, torch.from_numpy(r))
    gmask = prob.gamma.astype(bool)
    assert abs(float(mis[0]) - D) <= 1e-12 * D
    assert np.linalg.norm(G[gmask]) > 0
    assert rel(grad[0].cpu().numpy()[gmask], G[gmask]) < 1e-9
    h.close()


def test_lossy_autograd_backward_is_the_lossy_tr_gradient():
    # the differentiable forward (autograd) on a handle with absorption: the
    # backward of 1/2 ||f - f_obs||^2 is the lossy TR gradient of the oracle
    from paper_2102_00755_amd.autograd import simulate
    prob = make_small(shape=SHAPES[0], nt=40, n_src=2, n_rec=12, layer=2, precision=8)
    w, S = _inputs(prob)
    sch = ks.scheme_for(prob)
    a0 = lo.db_to_neper(A_DB, 1.5)
    los = lo.Lossy(sch, a0, 1.5)
    obs = lo.forward(los, prob.c_true, prob.src_ijk, S, w, prob.rec_ijk, prob.nt)["traces"]
    D, G, _ = lo.tr_gradient(los, prob.c_eval, prob.src_ijk, S, w, prob.rec_ijk, obs, prob.gamma, prob.boundary,
                             prob.nt)
    h = handle(prob, 8)
    h.set_absorption(a0, 1.5)
    c = torch.from_numpy(prob.c_eval).to(h.device).requires_grad_(True)
    f = simulate(h, c, torch.from_numpy(S).to(h.device), torch.from_numpy(w).to(h.device))
    loss = 0.5 * ((f - torch.from_numpy(obs).to(h.device)) ** 2).sum()
    loss.backward()
    gmask = prob.gamma.astype(bool)
    assert abs(float(loss.detach()) - D) <= 1e-10 * D
    assert rel(c.grad.cpu().numpy()[gmask], G[gmask]) < 1e-9
    h.close()


def test_lossy_graph_replay_equals_eager():
    # FWI_GRAPH: the lossy step captured once per call and replayed; every
    # replayed call, with eager work in between, equals the eager result bit
    # for bit (batch of two problems)
    prob = make_small(shape=SHAPES[1], nt=40, n_src=2, n_rec=12, layer=2, precision=4)
    h = handle(prob, 4, batch=2)
    h.set_absorption(lo.db_to_neper(A_DB, 1.5), 1.5)
    S = torch.from_numpy(np.stack([prob.src_signals()] * 2))
    w = torch.from_numpy(np.stack([oracle.rademacher(7, 2), oracle.rademacher(8, 2)]))
    c = torch.from_numpy(np.stack([prob.c_eval, prob.c_true]))
    obs = torch.from_numpy(np.stack([random_traces(prob.nt, prob.n_rec, 3, 1e-3),
                                     random_traces(prob.nt, prob.n_rec, 4, 1e-3)]))
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        h.use_graph = False
        tr_e = h.forward(c, S, w).clone()
        m_e, g_e = h.gradient(c, S, w, obs)
        m_e, g_e = m_e.clone(), g_e.clone()
        for rep in range(3):
            h.use_graph = True
            tr_g = h.forward(c, S, w)
            m_g, g_g = h.gradient(c, S, w, obs)
            side.synchronize()
            assert torch.equal(tr_g, tr_e), rep
            assert torch.equal(g_g, g_e), rep
            assert torch.equal(m_g, m_e), rep
            h.use_graph = False            # eager work between the replays
            h.forward(c, S, w)
            side.synchronize()
    h.close()
