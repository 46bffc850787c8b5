"""Write the stored oracle results used by the GPU parity tests.

Calls only the FP64 oracle (oracle/) and the seeded input generators
(synth/); nothing here touches the HIP path.  Run from the repository root:

    python tests/golden/make_golden.py c128        # 128^3, 600 steps (~15 min)
    python tests/golden/make_golden.py fullgrid    # 448x448x224, 40 steps (~30 min)
    python tests/golden/make_golden.py lossyfull   # the same with absorption (~60 min)
    python tests/golden/make_golden.py fullcfg     # the full-size workload, 600 steps (~5 h)
    python tests/golden/make_golden.py batch0 batch1              # 128^3 batch problems 0, 1 (~15 min each)
    python tests/golden/make_golden.py serve96 serve160 serve224  # serving levels (~20 min)

Each case stores, rounded to FP32, the oracle forward traces at c_true and
the TR gradient on Gamma at c_eval with its misfit:
  c128      against the observed data f(c_true) (Alg. 1 as a whole);
  fullgrid  from a stored seeded residual r (the backward of the traces):
            over 40 steps f(c_eval) - f(c_true) is too small against FP32
            rounding of the traces to test the gradient through it;
  lossyfull the fullgrid case with power-law absorption (oracle.lossy,
            LOSSY_DB dB MHz^-y cm^-1, y = LOSSY_Y, TR with the sign of tau
            switched);
  fullcfg   the full-size measurement workload itself (32 encoded emitters,
            1024 receivers, the 4.95 M-voxel Gamma with its 8-voxel layer,
            60 inclusions) on a horizon of FULLCFG_NT steps.  Within that
            horizon no wave scattered inside Gamma has returned to the bowl,
            so f(c_eval) - f(c_true) would be zero to FP32 rounding; the
            observed data are instead half the oracle traces at c_eval plus
            seeded noise (fullcfg_obs), stored, so the residual is large
            against trace rounding and reaches every receiver.  The forward
            traces stored are those at c_eval (the same run the gradient
            uses).
  batch0/1  problems 0 and 1 of the batched workload (128^3, 600 steps,
            phantom seeds 300/301, encoding seeds 1300/1301), as c128;
  serve96   the serving levels: 96^3 @ 1 mm over its full 300 steps,
  serve160  160^3 @ 0.75 mm and 224x224x112 @ 0.5 mm truncated to
  serve224  SERVE_NT[name] steps, with observed data built as for fullcfg.
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


FULLCFG_NT = 600
SERVE_NT = {"serve96": 300, "serve160": 150, "serve224": 150}
# cases whose observed data are built from the oracle traces at c_eval
SYNTH_OBS_CASES = ("fullcfg", "serve96", "serve160", "serve224")


def fullcfg_obs(traces_eval):
    """Observed data of the fullcfg and serving cases from the oracle traces at
    c_eval: 0.5 f + seeded Gaussian noise of 0.1 times the RMS of f, in FP32."""
    f = np.asarray(traces_eval, dtype=np.float64)
    rms = float(np.sqrt(np.mean(f * f)))
    noise = random_traces(f.shape[0], f.shape[1], seed=14, scale=0.1 * rms)
    return (0.5 * f + noise).astype(np.float32)


def problem(case):
    if case == "c128":
        return make_config("c128")
    if case in ("fullgrid", "lossyfull"):
        return fullgrid_problem()
    if case == "fullcfg":
        return make_config("full", nt=FULLCFG_NT)
    if case in ("batch0", "batch1"):
        return make_config("batch", index=int(case[-1]))
    if case in SERVE_NT:
        return make_config(case, nt=SERVE_NT[case])
    raise ValueError(case)


def run(case):
    t0 = time.time()
    prob = problem(case)
    sch = ks.scheme_for(prob)
    w = ks.rademacher(prob.enc_seed, prob.n_src)
    S = prob.src_signals()
    extra = {}
    if case in SYNTH_OBS_CASES:
        fwd = ks.forward(sch, prob.c_eval, prob.src_ijk, S, w, prob.rec_ijk, prob.nt, boundary=prob.boundary)
        f_eval = fwd["traces"]
        print(f"{case}: forward done {time.time() - t0:.0f} s", flush=True)
        obs32 = fullcfg_obs(f_eval)
        D, G, _ = ks.tr_gradient(sch, prob.c_eval, prob.src_ijk, S, w, prob.rec_ijk, obs32.astype(np.float64),
                                 prob.gamma, prob.boundary, prob.nt, fwd=fwd)
        print(f"{case}: gradient done {time.time() - t0:.0f} s, D = {D:.6e}", flush=True)
        g = prob.gamma.astype(bool)
        np.savez_compressed(os.path.join(HERE, f"{case}_oracle.npz"),
                            traces_eval=f_eval.astype(np.float32), obs=obs32, misfit=np.float64(D),
                            grad_gamma=G[g].astype(np.float32), w=w,
                            note=np.array(f"oracle FP64 results for synth case {case} ({prob.nt} steps), "
                                          f"rounded to FP32"))
        return
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
