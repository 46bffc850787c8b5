"""GPU parity with a different PML thickness on each axis, one of them zero.

The density passes keep the three split densities only on the x-lines inside
a y or z PML slab and the undamped sum (plus rho_x on the x-PML voxels)
elsewhere, and the inverse y pass writes d-_y v_y + d-_z v_z instead of the
two spectra on the latter lines.  Which lines and voxels are which follows
from the per-axis thickness, so these cases move the boundaries between the
two storages: an odd thickness (x-PML voxel pairs that straddle the PML
edge), thicknesses that differ between axes, and an axis without PML (no
slab lines, or no x-PML voxels).  Forward traces, TR gradient, lossy TR
gradient, exact gradient and the final-state TR start against the oracle.
Tolerances: FP64 traces <= 1e-10, gradients <= 1e-9; FP32 traces <= 1e-4,
gradients <= 1e-3.
"""

import dataclasses

import numpy as np
import pytest
import torch

import oracle
from oracle import kspace as ks
from oracle import lossy as lo
from synth import make_small
from synth.configs import random_traces

pytestmark = pytest.mark.gpu

SHAPE = (24, 40, 48)   # (nz, ny, nx)
PMLS = [(3, 5, 0), (0, 2, 4), (5, 0, 3)]   # (px, py, pz)


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _problem(pml, precision, nt=48):
    prob = make_small(shape=SHAPE, nt=nt, n_src=3, n_rec=12, layer=2, precision=precision)
    return dataclasses.replace(prob, pml=tuple(pml))


def _handle(prob, precision):
    from paper_2102_00755_amd.fwi import Handle
    return Handle.from_problem(prob, precision=precision)


@pytest.mark.parametrize("precision,ttol,gtol", [(8, 1e-10, 1e-9), (4, 1e-4, 1e-3)])
@pytest.mark.parametrize("pml", PMLS)
def test_forward_and_tr_gradient_with_uneven_pml(pml, precision, ttol, gtol):
    print(f"uneven pml={pml} precision={precision}", flush=True)
    prob = _problem(pml, precision)
    w = oracle.rademacher(prob.enc_seed, prob.n_src)
    S = prob.src_signals()
    sch = ks.scheme_for(prob)
    want = ks.forward(sch, prob.c_true, prob.src_ijk, S, w, prob.rec_ijk, prob.nt)["traces"]
    obs = random_traces(prob.nt, prob.n_rec, seed=31, scale=1e-3)
    D, G, _ = ks.tr_gradient(sch, prob.c_eval, prob.src_ijk, S, w, prob.rec_ijk, obs, prob.gamma,
                             prob.boundary, prob.nt)
    h = _handle(prob, precision)
    got = h.forward(torch.from_numpy(prob.c_true), torch.from_numpy(S), torch.from_numpy(w))[0].cpu().numpy()
    assert rel(got, want) < ttol, rel(got, want)
    mis, grad = h.gradient(torch.from_numpy(prob.c_eval), torch.from_numpy(S), torch.from_numpy(w),
                           torch.from_numpy(obs))
    g = prob.gamma.astype(bool)
    gg = grad[0].cpu().numpy()
    assert abs(float(mis[0]) - D) <= ttol * D
    assert np.all(gg[~g] == 0)
    assert rel(gg[g], G[g]) < gtol, rel(gg[g], G[g])
    h.close()


@pytest.mark.parametrize("precision,ttol,gtol", [(8, 1e-10, 1e-9), (4, 1e-4, 1e-3)])
@pytest.mark.parametrize("pml", PMLS[:2])
def test_lossy_tr_gradient_with_uneven_pml(pml, precision, ttol, gtol):
    print(f"uneven pml lossy={pml} precision={precision}", flush=True)
    prob = _problem(pml, precision)
    w = oracle.rademacher(prob.enc_seed, prob.n_src)
    S = prob.src_signals()
    sch = ks.scheme_for(prob)
    a0 = lo.db_to_neper(15.0, 1.5)
    los = lo.Lossy(sch, a0, 1.5)
    obs = random_traces(prob.nt, prob.n_rec, seed=32, scale=1e-3)
    D, G, _ = lo.tr_gradient(los, prob.c_eval, prob.src_ijk, S, w, prob.rec_ijk, obs, prob.gamma,
                             prob.boundary, prob.nt)
    h = _handle(prob, precision)
    h.set_absorption(a0, 1.5)
    mis, grad = h.gradient(torch.from_numpy(prob.c_eval), torch.from_numpy(S), torch.from_numpy(w),
                           torch.from_numpy(obs))
    g = prob.gamma.astype(bool)
    gg = grad[0].cpu().numpy()
    assert abs(float(mis[0]) - D) <= ttol * D
    assert np.all(gg[~g] == 0)
    assert rel(gg[g], G[g]) < gtol, rel(gg[g], G[g])
    h.close()


@pytest.mark.parametrize("pml", PMLS[1:])
def test_exact_and_final_state_gradients_with_uneven_pml(pml):
    # FP64: the exact discrete gradient (forward history of dp/dc0 on Gamma) and
    # the TR gradient started from the final forward state (the stored
    # densities are reused as they are)
    print(f"uneven pml exact/final-state={pml}", flush=True)
    prob = _problem(pml, 8)
    w = oracle.rademacher(prob.enc_seed, prob.n_src)
    S = prob.src_signals()
    sch = ks.scheme_for(prob)
    obs = random_traces(prob.nt, prob.n_rec, seed=33, scale=1e-3)
    D, G, _ = ks.exact_adjoint_gradient(sch, prob.c_eval, prob.src_ijk, S, w, prob.rec_ijk, obs, prob.nt)
    Df, Gf, _ = ks.tr_gradient(sch, prob.c_eval, prob.src_ijk, S, w, prob.rec_ijk, obs, prob.gamma,
                               prob.boundary, prob.nt, tr_init="final_state")
    h = _handle(prob, 8)
    g = prob.gamma.astype(bool)
    mis, grad = h.gradient(torch.from_numpy(prob.c_eval), torch.from_numpy(S), torch.from_numpy(w),
                           torch.from_numpy(obs), exact=True)
    assert abs(float(mis[0]) - D) <= 1e-10 * D
    assert rel(grad[0].cpu().numpy()[g], G[g]) < 1e-9
    h.tr_final_state = True
    mis, grad = h.gradient(torch.from_numpy(prob.c_eval), torch.from_numpy(S), torch.from_numpy(w),
                           torch.from_numpy(obs))
    assert abs(float(mis[0]) - Df) <= 1e-10 * Df
    assert rel(grad[0].cpu().numpy()[g], Gf[g]) < 1e-9
    h.close()
