"""GPU parity of the exact discrete gradient (FWI_EXACT): reverse-mode
differentiation of every operation of the forward iteration (App. B; PML
included), with absorption the dL/dc0 terms of App. A, against the oracle's
literal transpose of each step (oracle.kspace.exact_adjoint_gradient,
oracle.lossy.exact_adjoint_gradient), which central finite differences pin
on the CPU.  Tolerances: FP64 misfit <= 1e-10, gradient on Gamma <= 1e-9;
FP32 misfit <= 1e-4, gradient <= 1e-3.
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

A_DB = 15.0


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _problem(shape, precision):
    return make_small(shape=shape, nt=48, n_src=3, n_rec=12, layer=2, precision=precision)


@pytest.mark.parametrize("precision,ttol,gtol", [(8, 1e-10, 1e-9), (4, 1e-4, 1e-3)])
@pytest.mark.parametrize("shape", [(16, 24, 32), (24, 40, 48)])
def test_exact_gradient_lossless_matches_oracle(shape, precision, ttol, gtol):
    from paper_2102_00755_amd.fwi import Handle
    print(f"exact lossless shape={shape} precision={precision}", flush=True)
    prob = _problem(shape, precision)
    w = oracle.rademacher(prob.enc_seed, prob.n_src)
    S = prob.src_signals()
    sch = ks.scheme_for(prob)
    obs = random_traces(prob.nt, prob.n_rec, seed=21, scale=1e-3)
    D, G, _ = ks.exact_adjoint_gradient(sch, prob.c_eval, prob.src_ijk, S, w, prob.rec_ijk, obs, prob.nt)
    h = Handle.from_problem(prob, precision=precision)
    mis, grad = h.gradient(torch.from_numpy(prob.c_eval), torch.from_numpy(S), torch.from_numpy(w),
                           torch.from_numpy(obs), exact=True)
    g = prob.gamma.astype(bool)
    got = grad[0].cpu().numpy()
    assert abs(float(mis[0]) - D) <= ttol * D
    assert np.all(got[~g] == 0)
    assert rel(got[g], G[g]) < gtol, rel(got[g], G[g])
    h.close()


@pytest.mark.parametrize("precision,ttol,gtol", [(8, 1e-10, 1e-9), (4, 1e-4, 1e-3)])
@pytest.mark.parametrize("shape,y,field", [((16, 24, 32), 1.5, False), ((24, 40, 48), 0.6, True)])
def test_exact_gradient_lossy_matches_oracle(shape, y, field, precision, ttol, gtol):
    # absorption 15 dB MHz^-y cm^-1, uniform or a seeded per-voxel field
    # x U[0.5, 1.5]: the gradient carries (2/c0) p + c0^2 (tau' A[d] - eta' B[s])
    from paper_2102_00755_amd.fwi import Handle
    print(f"exact lossy shape={shape} y={y} field={field} precision={precision}", flush=True)
    prob = _problem(shape, precision)
    w = oracle.rademacher(prob.enc_seed, prob.n_src)
    S = prob.src_signals()
    sch = ks.scheme_for(prob)
    a0 = lo.db_to_neper(A_DB, y)
    a0f = a0 * np.random.default_rng(22).uniform(0.5, 1.5, size=shape) if field else a0
    los = lo.Lossy(sch, a0f, y)
    obs = random_traces(prob.nt, prob.n_rec, seed=23, scale=1e-3)
    D, G, _ = lo.exact_adjoint_gradient(los, prob.c_eval, prob.src_ijk, S, w, prob.rec_ijk, obs, prob.nt)
    # the absorption matters on this case: the lossless exact gradient differs
    _, G_no, _ = ks.exact_adjoint_gradient(sch, prob.c_eval, prob.src_ijk, S, w, prob.rec_ijk, obs, prob.nt)
    g = prob.gamma.astype(bool)
    assert rel(G_no[g], G[g]) > 1e-2
    h = Handle.from_problem(prob, precision=precision)
    if field:
        dt = torch.float32 if precision == 4 else torch.float64
        fld = torch.from_numpy(np.asarray(a0f)).to(h.device, dt)
        h.set_absorption(0.0, y, field=fld)
    else:
        h.set_absorption(a0, y)
    mis, grad = h.gradient(torch.from_numpy(prob.c_eval), torch.from_numpy(S), torch.from_numpy(w),
                           torch.from_numpy(obs), exact=True)
    got = grad[0].cpu().numpy()
    assert abs(float(mis[0]) - D) <= ttol * D
    assert np.all(got[~g] == 0)
    assert rel(got[g], G[g]) < gtol, rel(got[g], G[g])
    h.close()


def test_exact_gradient_rejects_batches_and_graphs():
    from paper_2102_00755_amd import _lib as L
    from paper_2102_00755_amd.fwi import FwiError, Handle
    prob = make_small(shape=(16, 24, 32), nt=8, precision=4)
    h = Handle.from_problem(prob, batch=2, precision=4)
    S = torch.from_numpy(prob.src_signals())
    w = torch.from_numpy(oracle.rademacher(prob.enc_seed, prob.n_src))
    c = torch.from_numpy(np.stack([prob.c_eval] * 2))
    obs = torch.from_numpy(random_traces(prob.nt, prob.n_rec, seed=3, scale=1e-3))
    with pytest.raises(FwiError) as e:
        h.gradient(c, S, w, obs, exact=True)
    assert e.value.status == L.FWI_ERR_INVALID_ARG
    with pytest.raises(FwiError) as e:
        h.gradient(c, S, w, obs, exact=True, mean=True)
    assert e.value.status == L.FWI_ERR_INVALID_ARG
    mis, grad = h.gradient(c[:1], S, w, obs, exact=True)       # B = 1 on a batch-2 handle
    assert torch.isfinite(grad).all() and float(mis[0]) > 0
    h.close()
