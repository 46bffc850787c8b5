"""Write the stored oracle results used by the GPU parity tests.

Calls only the FP64 oracle (oracle/) and the seeded input generators
(synth/); nothing here touches the HIP path.  Run from the repository root:

    python tests/golden/make_golden.py c128        # 128^3, 600 steps (~15 min)
    python tests/golden/make_golden.py fullgrid    # 448x448x224, 40 steps (~30 min)
    python tests/golden/make_golden.py lossyfull   # the same with absorption (~60 min)

Each case stores, rounded to FP32, the oracle forward traces at c_true and
the TR gradient on Gamma at c_eval with its misfit:
  c128      against the observed data f(c_true) (Alg. 1 as a whole);
  fullgrid  from a stored seeded residual r (the backward of the traces):
            over 40 steps f(c_eval) - f(c_true) is too small against FP32
            rounding of the traces to test the gradient through it;
  lossyfull the fullgrid case with power-law absorption (oracle.lossy,
            LOSSY_DB dB MHz^-y cm^-1, y = LOSSY_Y, TR with the sign of tau
            switched).
"""

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import kspace as ks  # noqa: E402
from oracle import lossy as lo  # noqa: E402
from synth import make_config, make_small, random_traces  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
LOSSY_DB = 15.0
LOSSY_Y = 1.5


def fullgrid_problem():
    """Full-size grid and PML with a compact geometry: Gamma a ball of 7
    cells in the centre with a 3-cell boundary layer, 4 sources and 64
    receivers on a sphere of 10 cells, so that within 40 steps the forward,
    adjoint and TR fields all cross Gamma."""
    return make_small(shape=(224, 448, 448), pml=20, nt=40, n_src=4, n_rec=64, layer=3, seed=11,
                      precision=4, r_transducer=10.0, r_gamma=7.0)


def fullgrid_residual(prob):
    """Seeded residual [nt, n_rec], rounded to FP32 (both sides use these
    exact values)."""
    return random_traces(prob.nt, prob.n_rec, seed=12, scale=0.1).astype(np.float32)


def problem(case):
    if case == "c128":
        return make_config("c128")
    if case in ("fullgrid", "lossyfull"):
        return fullgrid_problem()
    raise ValueError(case)


def run(case):
    t0 = time.time()
    prob = problem(case)
    sch = ks.scheme_for(prob)
    w = ks.rademacher(prob.enc_seed, prob.n_src)
    S = prob.src_signals()
    extra = {}
    if case == "lossyfull":
        los = lo.Lossy(sch, lo.db_to_neper(LOSSY_DB, LOSSY_Y), LOSSY_Y)
        obs = lo.forward(los, prob.c_true, prob.src_ijk, S, w, prob.rec_ijk, prob.nt)["traces"]
        print(f"{case}: forward done {time.time() - t0:.0f} s", flush=True)
        r = fullgrid_residual(prob)
        D, G, _ = lo.tr_gradient(los, prob.c_eval, prob.src_ijk, S, w, prob.rec_ijk, None, prob.gamma,
                                 prob.boundary, prob.nt, residual=r.astype(np.float64))
        extra.update(residual=r, alpha_db=np.float64(LOSSY_DB), y=np.float64(LOSSY_Y))
    else:
        obs = ks.forward(sch, prob.c_true, prob.src_ijk, S, w, prob.rec_ijk, prob.nt)["traces"]
        print(f"{case}: forward done {time.time() - t0:.0f} s", flush=True)
        if case == "fullgrid":
            r = fullgrid_residual(prob)
            D, G, _ = ks.tr_gradient(sch, prob.c_eval, prob.src_ijk, S, w, prob.rec_ijk, None, prob.gamma,
                                     prob.boundary, prob.nt, residual=r.astype(np.float64))
            extra["residual"] = r
        else:
            D, G, _ = ks.tr_gradient(sch, prob.c_eval, prob.src_ijk, S, w, prob.rec_ijk, obs, prob.gamma,
                                     prob.boundary, prob.nt)
    print(f"{case}: gradient done {time.time() - t0:.0f} s, D = {D:.6e}", flush=True)
    g = prob.gamma.astype(bool)
    np.savez_compressed(os.path.join(HERE, f"{case}_oracle.npz"),
                        traces_true=obs.astype(np.float32), misfit=np.float64(D),
                        grad_gamma=G[g].astype(np.float32), w=w,
                        note=np.array(f"oracle FP64 results for synth case {case}, rounded to FP32"), **extra)


if __name__ == "__main__":
    for c in sys.argv[1:] or ["c128", "fullgrid", "lossyfull"]:
        run(c)
