"""GPU tests of the stochastic L-BFGS outer loop (App. D, Algorithm 2).

* the library's vector primitives (axpby, clip, squared slowness, Gamma
  gather / scatter, the L-BFGS history and two-loop recursion with ring
  wrap-around) against NumPy and the oracle's two-loop recursion;
* the device SLBFGS against the oracle SLBFGS (both driving their own encoded
  TR gradient) on a small FP64 problem: iterates and energies to 1e-9;
* on the 64^3 single-source workload the energy estimate decreases and the
  speed of sound in Gamma moves towards the true one.
"""

import numpy as np
import pytest
import torch

import oracle
import oracle.slbfgs as osl
from oracle import kspace as ks
from synth import make_config, make_small

pytestmark = pytest.mark.gpu


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("precision", [4, 8])
def test_vector_primitives(precision):
    from paper_2102_00755_amd.slbfgs import LbfgsHistory, VecOps
    dt = torch.float32 if precision == 4 else torch.float64
    tol = 1e-5 if precision == 4 else 1e-12
    dev = torch.device("cuda", 0)
    ops = VecOps(dev, dt)
    rng = np.random.default_rng(2)
    n = 10007                                          # several reduction blocks and a ragged tail
    x = rng.standard_normal(n)
    y = rng.standard_normal(n)
    tx, ty = torch.tensor(x, device=dev, dtype=dt), torch.tensor(y, device=dev, dtype=dt)
    assert rel(ops.axpby(0.5, tx, -2.0, ty.clone()).cpu(), 0.5 * x - 2.0 * y) < tol
    garbage = torch.full((n,), float("nan"), device=dev, dtype=dt)
    assert torch.equal(ops.copy(tx, garbage), tx)     # b = 0 does not read y
    assert rel(ops.clip(tx.clone(), -0.3, 0.7).cpu(), np.clip(x, -0.3, 0.7)) < tol
    c = 1400 + 300 * rng.random(n)
    tc = torch.tensor(c, device=dev, dtype=dt)
    u = ops.sqslowness(0, tc, torch.empty_like(tc))
    assert rel(u.cpu(), 1 / c ** 2) < tol
    assert rel(ops.sqslowness(1, u, torch.empty_like(u)).cpu(), c) < tol
    assert rel(ops.sqslowness(2, tx, torch.empty_like(tx), aux=tc).cpu(), -0.5 * c ** 3 * x) < tol
    # history of m = 4 pairs after 6 pushes (ring wrap) against the oracle
    m, npair = 4, 6
    B = rng.standard_normal((8, 8))
    S = [rng.standard_normal(n) for _ in range(npair)]
    Y = [s + 0.1 * rng.standard_normal(n) for s in S]      # y^T s > 0
    hist = LbfgsHistory(n, m, ops)
    assert hist.count() == 0
    g = rng.standard_normal(n)
    tg = torch.tensor(g, device=dev, dtype=dt)
    r = torch.empty_like(tg)
    assert rel(hist.apply(tg, r, 0.7).cpu(), 0.7 * g) < tol
    for k in range(npair):
        hist.push(torch.tensor(S[k], device=dev, dtype=dt), torch.tensor(Y[k], device=dev, dtype=dt))
        want = osl.two_loop(g, S[max(0, k + 1 - m):k + 1], Y[max(0, k + 1 - m):k + 1], 0.7)
        assert rel(hist.apply(tg, r, 0.7).cpu(), want) < 10 * tol, k
    assert hist.count() == m
    assert rel(hist.apply(tg, tg.clone(), 0.7).cpu(), want) < 10 * tol      # r may alias g
    hist.close()


def test_gamma_gather_scatter():
    from paper_2102_00755_amd.fwi import Handle
    from paper_2102_00755_amd.slbfgs import EncodedEstimator
    prob = make_small(shape=(24, 32, 32), precision=8)
    h = Handle.from_problem(prob, precision=8)
    est = EncodedEstimator(h, prob.c_true, prob.src_signals(), lambda w: None)
    g = prob.gamma.astype(bool)
    assert est.n == int(g.sum())
    rng = np.random.default_rng(3)
    full = rng.standard_normal(prob.shape)
    comp = est.gather(torch.tensor(full, device=h.device), est.empty())
    assert np.array_equal(comp.cpu().numpy(), full[g])           # [z][y][x] order
    base = rng.standard_normal(prob.shape)
    out = est.scatter(comp, torch.tensor(base, device=h.device)).cpu().numpy()
    want = base.copy()
    want[g] = full[g]
    assert np.array_equal(out, want)
    h.close()


def _problem():
    return make_small(shape=(24, 32, 32), nt=48, n_src=2, n_rec=12, layer=2, seed=21, precision=8)


def test_slbfgs_matches_oracle_fp64():
    from paper_2102_00755_amd.fwi import Handle
    from paper_2102_00755_amd.slbfgs import EncodedEstimator, slbfgs
    prob = _problem()
    sch = ks.scheme_for(prob)
    S = prob.src_signals()
    g = prob.gamma.astype(bool)
    seed0 = 40
    c_bg = prob.c_eval.copy()

    def g_oracle(u, i):
        w = oracle.rademacher(seed0 + i, prob.n_src)
        obs = ks.forward(sch, prob.c_true, prob.src_ijk, S, w, prob.rec_ijk, prob.nt)["traces"]
        c = c_bg.copy()
        c[g] = 1.0 / np.sqrt(u)
        D, G, _ = ks.tr_gradient(sch, c, prob.src_ijk, S, w, prob.rec_ijk, obs, prob.gamma, prob.boundary, prob.nt)
        return D, -0.5 * c[g] ** 3 * G[g]

    u0 = 1.0 / c_bg[g] ** 2
    _, G0 = g_oracle(u0, 1)
    h0 = 0.02 * np.abs(u0).max() / np.abs(G0).max()      # first step changes u by about 2 %
    lo, hi = 1.0 / prob.c_max ** 2, 1.0 / prob.c_min ** 2
    u_or, J_or = osl.slbfgs(g_oracle, u0, nu=1.0, n_evals=6, h0=h0, u_min=lo, u_max=hi)

    h = Handle.from_problem(prob, precision=8)
    c_true = torch.from_numpy(prob.c_true).to(h.device)
    Sd = torch.from_numpy(S).to(h.device)
    est = EncodedEstimator(h, c_bg, S, lambda w: h.forward(c_true, Sd, w)[0], seed0=seed0, param="sqslowness")
    print("slbfgs parity", flush=True)
    u_gpu, J_gpu = slbfgs(est, est.u_from_c(c_bg), nu=1.0, n_evals=6, h0=h0, u_min=lo, u_max=hi)
    assert est.evals == 6 and len(J_gpu) == 3
    assert rel(J_gpu, J_or) < 1e-9
    assert rel(u_gpu.cpu().numpy(), u_or) < 1e-9
    assert rel(u_or, u0) > 1e-4                         # the iteration moved
    h.close()


def test_slbfgs_decreases_energy_on_single_source_workload():
    # 64^3, 160 FP64 steps, one source, 8 mm sphere at 1560 m/s in water
    from paper_2102_00755_amd.fwi import Handle
    from paper_2102_00755_amd.slbfgs import EncodedEstimator, slbfgs
    prob = make_config("tiny")
    h = Handle.from_problem(prob, precision=8)
    g = prob.gamma.astype(bool)
    c_true = torch.from_numpy(prob.c_true).to(h.device)
    Sd = torch.from_numpy(prob.src_signals()).to(h.device)
    est = EncodedEstimator(h, prob.c_eval, prob.src_signals(), lambda w: h.forward(c_true, Sd, w)[0], seed0=1)
    u0 = est.u_from_c(prob.c_eval)
    G = est.empty()
    est(u0, 1, G)
    h0 = 0.01 * float(u0.abs().max()) / float(G.abs().max())
    err0 = rel(prob.c_eval[g], prob.c_true[g])
    errs = []
    u_hat, J = slbfgs(est, u0, nu=1.0, n_evals=12, h0=h0, u_min=1 / prob.c_max ** 2, u_max=1 / prob.c_min ** 2,
                      callback=lambda i, uh, Ji: errs.append(rel(1 / np.sqrt(uh.cpu().numpy()), prob.c_true[g])))
    print("energies", J, "errors", err0, errs, flush=True)
    assert J[-1] < 0.5 * J[0]
    assert errs[-1] < err0
    h.close()
