"""Throughput and latency of the batched and served forms.

    python -m paper_2102_00755_amd.bench_forms batched [--batch 16] [--nt 600]
    python -m paper_2102_00755_amd.bench_forms serve [--requests 200] [--seconds-scale 1]
    python -m paper_2102_00755_amd.bench_forms lbfgs [--n 4954176] [--m 64]
    python -m paper_2102_00755_amd.bench_forms multigrid
    python -m paper_2102_00755_amd.bench_forms lossy [--steps 2] [--nt 2200]
    python -m paper_2102_00755_amd.bench_forms latency [--steps 20]
    python -m paper_2102_00755_amd.bench_forms exact [--nt 200]

batched : 16 independent Rademacher-encoded TR gradients on 128^3 (phantom
          seeds 300..315, encoding seeds 1300..1315), run (a) one after
          another on a batch-1 handle and (b) in one batch-16 handle whose
          passes cover all problems per launch, with the time step captured in
          a hipGraph, each handle with the autotuner's tile widths; reports
          Mcell-steps/s and per-solve latency of both.
serve   : Poisson-arriving forward / gradient requests (50/50) over the grid
          levels 96^3 @ 1.0 mm (300 steps), 160^3 @ 0.75 mm (600) and
          224x224x112 @ 0.5 mm (1200), admitted by HBM footprint, waiting
          requests of one level and kind grouped into batched calls of up to
          --serve-batch; the arrival rate is set to each of --loads times the
          measured single-stream capacity (default 0.8 and 2.0); each level
          uses the autotuner's tile widths; reports p50/p99 latency,
          Mcell-steps/s and the mean requests per call against the same
          requests solved one at a time.
lbfgs   : the SLBFGS two-loop recursion (64 pairs) and pair push at |Gamma| of
          the full workload, with their algorithmic bandwidth.
multigrid: grid transfers between the 1 mm and 0.5 mm levels of the full box.
exact   : the exact discrete gradient (FWI_EXACT) against the TR gradient on the
          full workload (--nt, default 200 steps), without and with absorption.
latency : p50 / p99 of repeated plain encoded TR gradients (one at a time, each
          synchronised): --steps solves of the full workload and 5x as many
          of the 128^3 workload.
lossy   : the encoded TR gradient of the full workload (448x448x224, 2200
          steps) with power-law absorption (0.75 dB MHz^-1.5 cm^-1, y = 1.5,
          TR with the sign of tau switched) against the same gradient without
          absorption on the same handle.
Prints one JSON line per run.  Inputs are synthetic (synth/).
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import tempfile
import time

import numpy as np
import torch

from . import autotune, fwi
from .serving import Level, Server


def _gradient_inputs(prob, dev, dtype):
    w = torch.from_numpy(fwi.rademacher(prob.enc_seed, prob.n_src))
    S = torch.from_numpy(prob.src_signals()).to(dtype)
    return (torch.from_numpy(prob.c_eval).to(dtype), torch.from_numpy(prob.c_true).to(dtype), S, w)


def batched(args) -> dict:
    from synth import make_config
    B = args.batch
    probs = [make_config("batch", index=i, nt=args.nt) for i in range(B)]
    base = probs[0]
    # one geometry for the batch: all emitters of the bowl, per-problem weights
    # select each problem's encoded subset (zero for the others)
    emitters = base.meta["all_emitters"]
    n_all = emitters.shape[0]
    kw = fwi.problem_kwargs(base)
    kw["src_ijk"] = emitters
    dev = torch.device("cuda", 0)
    dtype = torch.float32
    c_eval = torch.stack([torch.from_numpy(p.c_eval) for p in probs]).to(dev, dtype)
    c_true = torch.stack([torch.from_numpy(p.c_true) for p in probs]).to(dev, dtype)
    W = torch.zeros((B, n_all), dtype=torch.int8)
    for i, p in enumerate(probs):
        W[i, p.meta["emitter_index"]] = torch.from_numpy(fwi.rademacher(p.enc_seed, p.n_src))
    W = W.to(dev)
    S = torch.from_numpy(np.repeat(base.pulse[:, None], n_all, axis=1)).to(dev, dtype)
    S = S.unsqueeze(0).expand(B, -1, -1).contiguous()
    side = torch.cuda.Stream(device=dev)
    out = {}
    cache = os.path.join(tempfile.mkdtemp(), "tuning.json")
    with torch.cuda.stream(side):
        hb = fwi.Handle(**kw, batch=B)
        out["tuning_batched"] = autotune.apply(hb, cache=cache)   # tile widths measured for this grid
        hb.use_graph = True
        obs = hb.forward(c_true, S, W)
        side.synchronize()
        hb.gradient(c_eval, S, W, obs)        # warm-up
        side.synchronize()
        t0 = time.perf_counter()
        mis_b, g_b = hb.gradient(c_eval, S, W, obs)
        side.synchronize()
        t_b = time.perf_counter() - t0
        h1 = fwi.Handle(**kw, batch=1)
        out["tuning_single"] = autotune.apply(h1, cache=cache)
        h1.use_graph = True
        h1.gradient(c_eval[0], S[0], W[0], obs[0])
        side.synchronize()
        lat = []
        t0 = time.perf_counter()
        for i in range(B):
            t1 = time.perf_counter()
            m1, g1 = h1.gradient(c_eval[i], S[i], W[i], obs[i])
            side.synchronize()
            lat.append(time.perf_counter() - t1)
            if i == 0:
                g1_0 = g1[0].clone()
        t_s = time.perf_counter() - t0
        # problem 0 alone in the batched handle's tuning is the batched result
        # bit for bit; in its own tuning (other tile widths and radix plans,
        # other rounding) it agrees to FP32 rounding
        rel_own = float((g1_0 - g_b[0]).double().norm() / g_b[0].double().norm())
        h1.tuning = out["tuning_batched"]
        _, g1b = h1.gradient(c_eval[0], S[0], W[0], obs[0])
        side.synchronize()
        same = bool(torch.equal(g1b[0], g_b[0]))
        hb.close()
        h1.close()
    work = 3.0 * base.n_cells * base.nt * B
    out.update({
        "form": "batched", "batch": B, "grid": list(base.shape[::-1]), "nt": base.nt,
        "batched_Mcell_steps_per_s": work / t_b / 1e6, "batched_wall_s": t_b,
        "single_Mcell_steps_per_s": work / t_s / 1e6, "single_wall_s": t_s,
        "single_p50_ms": float(np.percentile(np.array(lat) * 1e3, 50)),
        "single_p99_ms": float(np.percentile(np.array(lat) * 1e3, 99)),
        "batched_equals_single": same, "single_own_tuning_rel_l2": rel_own, "hipgraph": True,
    })
    return out


def serve(args) -> dict:
    from synth import make_config
    names = ["serve96", "serve160", "serve224"]
    probs = {n: make_config(n) for n in names}
    levels = [Level(n, fwi.problem_kwargs(p)) for n, p in probs.items()]
    rng = np.random.default_rng(4)
    reqs = []
    for i in range(args.requests):
        lv = names[int(rng.integers(0, 3))]
        kind = "gradient" if rng.random() < 0.5 else "forward"
        p = probs[lv]
        c = p.c_eval + rng.uniform(-5, 5, size=p.shape) * p.gamma
        w = torch.from_numpy(fwi.rademacher(p.enc_seed + i, p.n_src))
        reqs.append((kind, lv, torch.from_numpy(c), torch.from_numpy(p.src_signals()), w))
    # observed data per level (synthetic: forward at c_true, computed up front)
    obs = {}
    for n, p in probs.items():
        h = fwi.Handle.from_problem(p)
        obs[n] = h.forward(torch.from_numpy(p.c_true), torch.from_numpy(p.src_signals()),
                           torch.from_numpy(fwi.rademacher(p.enc_seed, p.n_src)))[0].cpu()
        h.close()
    # tile widths of each level from the autotuner (applied to the solo handles
    # and to every handle the server creates)
    cache = os.path.join(tempfile.mkdtemp(), "tuning.json")
    # single-stream capacity: every request alone, one after another
    solo_lat = []
    hs = {n: fwi.Handle.from_problem(p) for n, p in probs.items()}
    for lv in levels:
        lv.tuning = autotune.apply(hs[lv.name], cache=cache)
    for n in names:   # warm-up
        hs[n].forward(torch.from_numpy(probs[n].c_eval), torch.from_numpy(probs[n].src_signals()),
                      torch.from_numpy(fwi.rademacher(1, probs[n].n_src)))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for kind, lv, c, s, w in reqs:
        t1 = time.perf_counter()
        if kind == "forward":
            hs[lv].forward(c, s, w)
        else:
            hs[lv].gradient(c, s, w, obs[lv])
        torch.cuda.synchronize()
        solo_lat.append(time.perf_counter() - t1)
        if len(solo_lat) % 25 == 0:
            print(json.dumps({"solo_done": len(solo_lat)}), file=sys.stderr, flush=True)
    t_solo = time.perf_counter() - t0
    for h in hs.values():
        h.close()
    work = sum(probs[lv].n_cells * probs[lv].nt * (3 if k == "gradient" else 1) for k, lv, *_ in reqs)
    out = {
        "form": "serve", "tuning": {lv.name: lv.tuning for lv in levels}, "requests": len(reqs),
        "levels": names, "solo_Mcell_steps_per_s": work / t_solo / 1e6,
        "solo_p50_ms": float(np.percentile(np.array(solo_lat) * 1e3, 50)),
        "solo_p99_ms": float(np.percentile(np.array(solo_lat) * 1e3, 99)),
        "inflight": args.inflight, "batch_per_call": args.serve_batch, "served": [],
    }
    budget = int(args.budget_gb * 2 ** 30)
    for lv in levels:
        lv.batch = args.serve_batch
    for load in args.loads:
        # Poisson arrivals at `load` times the single-stream capacity
        rate = load * len(reqs) / t_solo
        gaps = np.random.default_rng(40).exponential(1.0 / rate, size=len(reqs))
        srv = Server(levels, budget_bytes=budget, max_inflight=args.inflight)
        for n in names:      # warm-up: the resident handles of every level
            p = probs[n]
            srv.submit("forward", n, torch.from_numpy(p.c_eval), torch.from_numpy(p.src_signals()),
                       torch.from_numpy(fwi.rademacher(1, p.n_src))).result()
        srv.reset_stats()
        futs = []
        t_start = time.perf_counter()
        for k, ((kind, lv, c, s, w), gap) in enumerate(zip(reqs, gaps)):
            time.sleep(gap)
            futs.append(srv.submit(kind, lv, c, s, w, obs[lv] if kind == "gradient" else None))
            if (k + 1) % 50 == 0:
                print(json.dumps({"load": load, "submitted": k + 1}), file=sys.stderr, flush=True)
        for k, f in enumerate(futs):
            f.result()
            if (k + 1) % 25 == 0:
                print(json.dumps({"load": load, "served_done": k + 1}), file=sys.stderr, flush=True)
        st = srv.stats()
        srv.close()
        out["served"].append({
            "offered_load": load, "arrival_rate_per_s": rate,
            "Mcell_steps_per_s": st["Mcell-steps/s"], "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"],
            "calls": st["calls"], "mean_batch": st["mean_batch"], "handles": st["handles"],
            "device_bytes": st["device_bytes"], "wall_s": time.perf_counter() - t_start,
        })
    return out


def lbfgs(args) -> dict:
    """Two-loop recursion and pair push of the SLBFGS outer loop at the full
    workload's unknown count (|Gamma| = 4 954 176 voxels, FP32, m = 64 pairs)."""
    from .slbfgs import LbfgsHistory, VecOps
    dev = torch.device("cuda", 0)
    n, m = args.n, args.m
    ops = VecOps(dev, torch.float32)
    hist = LbfgsHistory(n, m, ops)
    gen = torch.Generator(device=dev)
    gen.manual_seed(5)
    s = torch.randn(n, device=dev, generator=gen)
    y = s + 0.1 * torch.randn(n, device=dev, generator=gen)
    g = torch.randn(n, device=dev, generator=gen)
    r = torch.empty_like(g)
    for _ in range(m):
        hist.push(s, y)
    torch.cuda.synchronize()
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        hist.apply(g, r, 1.0)
    torch.cuda.synchronize()
    t_apply = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        hist.push(s, y)
    torch.cuda.synchronize()
    t_push = (time.perf_counter() - t0) / reps
    hist.close()
    # per pair and loop: a dot (2 vectors read) and an axpy (2 read, 1 written)
    bytes_apply = 2.0 * m * 5 * n * 4 + 2 * n * 4
    return {"form": "lbfgs", "n": n, "m": m, "dtype": "f32", "apply_ms": t_apply * 1e3,
            "apply_GBps_algorithmic": bytes_apply / t_apply / 1e9, "push_ms": t_push * 1e3,
            "note": "two applies and one push per SLBFGS iteration, against two TR gradients"}


def multigrid(args) -> dict:
    """Grid transfers between the 224x224x112 (1 mm) and 448x448x224 (0.5 mm)
    levels: Fourier interpolation with Blackman smoothing of a speed field,
    and windowed-sinc resampling of 1024-receiver data from 2200 to 1100 steps."""
    from synth import make_config
    from .multigrid import coarse_cutoff, coarse_level, data_scale, interp_up, resample_time
    fine = make_config("full")
    kw = fwi.problem_kwargs(fine, nt=4)
    hf = fwi.Handle(**kw)
    from synth.configs import make_small
    coarse = make_small(shape=(112, 224, 224), dx=2 * fine.dx, nt=4, pml=10, layer=2, precision=4,
                        n_src=1, n_rec=2, r_transducer=6.0, r_gamma=4.0)
    hc = fwi.Handle.from_problem(coarse)
    dev = hf.device
    u = torch.full(hc.shape, 1500.0, device=dev)
    interp_up(hc, hf, u)
    torch.cuda.synchronize()
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        out = interp_up(hc, hf, u)
    torch.cuda.synchronize()
    t_interp = (time.perf_counter() - t0) / reps
    dt_c, nt_c = coarse_level(fine.dt, fine.nt, 2.0)
    f = torch.randn((fine.nt, fine.n_rec), device=dev)
    resample_time(f, fine.dt, dt_c, nt_c, coarse_cutoff(fine.c_min, 2 * fine.dx), scale=data_scale(2.0))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        g = resample_time(f, fine.dt, dt_c, nt_c, coarse_cutoff(fine.c_min, 2 * fine.dx), scale=data_scale(2.0))
    torch.cuda.synchronize()
    t_res = (time.perf_counter() - t0) / reps
    ok = bool(torch.isfinite(out).all()) and abs(float(out.mean()) - 1500.0) < 1e-2
    hc.close()
    hf.close()
    return {"form": "multigrid", "interp_ms": t_interp * 1e3, "interp": "224x224x112 -> 448x448x224 FP32",
            "resample_ms": t_res * 1e3, "resample": f"[{fine.nt}, {fine.n_rec}] -> [{nt_c}, {fine.n_rec}] FP32",
            "constant_preserved": ok}


def lossy(args) -> dict:
    from synth import make_config
    prob = make_config("full", nt=args.nt)
    h = fwi.Handle.from_problem(prob, precision=4)
    dev = h.device
    c_eval, c_true, S, w = (t.to(dev) for t in _gradient_inputs(prob, dev, torch.float32))
    grad = torch.empty((1, *h.shape), device=dev, dtype=torch.float32)
    work = 3.0 * prob.n_cells * prob.nt
    out = {"form": "lossy", "workload": "448x448x224, %d steps, 32 encoded emitters, 1024 receivers" % prob.nt,
           "alpha_db_MHz_cm": 0.75, "y": 1.5}
    for name, a_db in (("lossy", 0.75), ("lossless", 0.0)):
        h.set_absorption(fwi.db_to_neper(a_db, 1.5), 1.5)
        obs = h.forward(c_true, S, w)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h.forward(c_true, S, w)
        torch.cuda.synchronize()
        t_fwd = time.perf_counter() - t0
        h.gradient(c_eval, S, w, obs, out=grad)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            h.gradient(c_eval, S, w, obs, out=grad)
        torch.cuda.synchronize()
        t_grad = (time.perf_counter() - t0) / args.steps
        out[name] = {"gradient_s": t_grad, "Mcell_steps_per_s": work / t_grad / 1e6,
                     "forward_Mcell_steps_per_s": prob.n_cells * prob.nt / t_fwd / 1e6,
                     "grad_finite": bool(torch.isfinite(grad).all())}
        print(json.dumps({name: out[name]}), flush=True)
    h.close()
    out["lossy_over_lossless"] = out["lossy"]["gradient_s"] / out["lossless"]["gradient_s"]
    return out


def exact(args) -> dict:
    """The exact discrete gradient (FWI_EXACT: stored dp/dc0 history on Gamma,
    reverse sweep) against Alg. 1's TR gradient on the full workload, without
    and with absorption (0.75 dB MHz^-1.5 cm^-1)."""
    from synth import make_config
    nt = args.nt or 200
    prob = make_config("full", nt=nt)
    h = fwi.Handle.from_problem(prob, precision=4)
    dev = h.device
    c_eval, c_true, S, w = (t.to(dev) for t in _gradient_inputs(prob, dev, torch.float32))
    grad = torch.empty((1, *h.shape), device=dev, dtype=torch.float32)
    out = {"form": "exact", "workload": "448x448x224, %d steps, 32 encoded emitters, 1024 receivers" % nt,
           "history_GB": nt * int(prob.gamma.sum()) * 4 / 1e9}
    for name, a_db in (("lossless", 0.0), ("lossy", 0.75)):
        h.set_absorption(fwi.db_to_neper(a_db, 1.5), 1.5)
        obs = h.forward(c_true, S, w)
        res = {}
        for kind, ex in (("tr", False), ("exact", True)):
            h.gradient(c_eval, S, w, obs, out=grad, exact=ex)       # warm-up (allocates the history)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, g = h.gradient(c_eval, S, w, obs, exact=ex)
            torch.cuda.synchronize()
            res[kind + "_s"] = time.perf_counter() - t0
            res[kind] = g.clone()
        m = torch.from_numpy(prob.gamma.astype(bool)).to(dev)
        d = (res["tr"][0][m].double() - res["exact"][0][m].double()).norm() / res["exact"][0][m].double().norm()
        out[name] = {"tr_gradient_s": res["tr_s"], "exact_gradient_s": res["exact_s"],
                     "exact_over_tr": res["exact_s"] / res["tr_s"], "tr_vs_exact_rel_l2": float(d)}
        print(json.dumps({name: out[name]}), flush=True)
    h.close()
    return out


def latency(args) -> dict:
    from synth import make_config
    out = {"form": "latency"}
    for name, reps in (("c128", 5 * args.steps), ("full", args.steps)):
        prob = make_config(name, nt=args.nt if name == "full" else None)
        h = fwi.Handle.from_problem(prob, precision=4)
        dev = h.device
        c_eval, c_true, S, w = (t.to(dev) for t in _gradient_inputs(prob, dev, torch.float32))
        obs = h.forward(c_true, S, w)
        grad = torch.empty((1, *h.shape), device=dev, dtype=torch.float32)
        h.gradient(c_eval, S, w, obs, out=grad)
        torch.cuda.synchronize()
        lat = []
        for i in range(reps):
            t0 = time.perf_counter()
            h.gradient(c_eval, S, w, obs, out=grad)
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - t0)
            if name == "full":
                print(json.dumps({"solve": i, "s": lat[-1]}), flush=True)
        ms = np.array(lat) * 1e3
        out[name] = {"solves": reps, "p50_ms": float(np.percentile(ms, 50)), "p99_ms": float(np.percentile(ms, 99)),
                     "min_ms": float(ms.min()), "max_ms": float(ms.max()),
                     "Mcell_steps_per_s_p50": 3.0 * prob.n_cells * prob.nt / (np.percentile(ms, 50) / 1e3) / 1e6}
        h.close()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("form", choices=["batched", "serve", "lbfgs", "multigrid", "lossy", "latency", "exact"])
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--nt", type=int, default=None)
    ap.add_argument("--requests", type=int, default=200)
    ap.add_argument("--inflight", type=int, default=4)
    ap.add_argument("--budget-gb", type=float, default=64.0)
    ap.add_argument("--serve-batch", type=int, default=4, help="requests per batched call of a served level")
    ap.add_argument("--loads", type=float, nargs="+", default=[0.8, 2.0],
                    help="offered loads of the served trace, in units of the single-stream capacity")
    ap.add_argument("--n", type=int, default=4954176)
    ap.add_argument("--m", type=int, default=64)
    args = ap.parse_args()
    res = {"batched": batched, "serve": serve, "lbfgs": lbfgs, "multigrid": multigrid,
           "lossy": lossy, "latency": latency, "exact": exact}[args.form](args)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
