"""Benchmark: encoded TR gradient throughput on one MI355X.

One step = one encoded time-reversal gradient (forward + adjoint + TR
re-simulation, Alg. 1) of the full-size workload: 448x448x224 grid at
0.5 mm, 20-cell PML, 2200 FP32 time steps, 32 Rademacher-encoded emitters,
1024 receivers on a 2048-element golden-section bowl, breast-like phantom
with 60 inclusions.  Inputs are synthetic and resident in HBM before timing.

Prints one JSON line: throughput in Mcell-steps/s (3 simulations x cells x
steps per gradient), p50/p99 solve latency, the HBM roofline of the dominant
pass kernel (HIP events on the library's stream, sampled every few steps)
and the FP64 oracle timed on the host on a truncated horizon.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Mcell-steps/s of TR-gradient at 448x448x224 FP32; p50/p99 solve latency"
PEAK_HBM_GBS = 8000.0
def step_bytes_per_cell(shape, pml) -> float:
    """Algorithmic HBM bytes per cell and simulation step of the eight-pass
    step (4-byte field-sized reads and writes; the pass table of the
    kernels): 32 + 2 f + R passes, where f is the fraction of x-lines in a y
    or z PML slab (they keep three split densities and two derivative
    spectra; the others keep the undamped density sum, plus rho_x on the
    x-PML voxels, and one spectrum of d-_y v_y + d-_z v_z) and R the split
    density reads and writes per voxel."""
    nz, ny, nx = shape
    px, py, pz = pml

    def slab(i, n, p):
        return i < p or i > n - 1 - p
    f = sum(1 for z in range(nz) for y in range(ny) if slab(y, ny, py) or slab(z, nz, pz)) / (ny * nz)
    xp = sum(1 for n in range(nx // 2) if slab(2 * n, nx, px) or slab(2 * n + 1, nx, px))
    rho = 6.0 * f + (2.0 + 4.0 * xp / nx) * (1.0 - f)
    return 4.0 * (32.0 + 2.0 * f + rho)

KERNEL_SYMBOLS = {
    "y_fwd": "k_axis_y<float, {ny}, false, {ty}, {py}>",
    "y_inv": "k_axis_y<float, {ny}, true, {ty}, {py}>",
    "z_plus": "k_axis_z_plus<float, {nz}, {tzp}, {pzp}>",
    "z_minus": "k_axis_z_minus<float, {nz}, {tzm}, {pzm}>",
    "x_vel": "k_x_velocity<float, {m}, {px}>",
    "x_den_fwd": "k_x_density<float, {m}, 0, {px}>",
    "x_den_pair": "k_x_density<float, {m}, 1, {px}>",
    "y_vel_q": "k_axis_y_vel<float, {ny}, {ty}, {py}>",
}


def _plan_run(L: int, plan: int) -> int:
    """The radix plan a kernel of length L is instantiated with for the
    requested plan: 1 only where the power-of-two stages of the length are
    not a palindrome (otherwise both plans are the same kernel, plan 0)."""
    m = L
    for r in (7, 5, 3):
        while m % r == 0:
            m //= r
    pw = []
    while m > 1:
        if m == 16:
            pw += [4, 4]
            m = 1
        elif m % 8 == 0:
            pw.append(8)
            m //= 8
        elif m % 4 == 0:
            pw.append(4)
            m //= 4
        else:
            pw.append(2)
            m //= 2
    return plan if pw != pw[::-1] else 0


def kernel_symbol(name: str, nx: int, ny: int, nz: int, tuning: dict) -> str:
    """Demangled symbol of the kernel that runs pass `name` under `tuning`."""
    return KERNEL_SYMBOLS[name].format(
        nx=nx, ny=ny, nz=nz, m=nx // 2, ty=tuning["y_tile_bytes"], tzm=tuning["zm_tile_bytes"],
        tzp=tuning["zp_tile_bytes"], py=_plan_run(ny, tuning["y_plan"]), pzm=_plan_run(nz, tuning["zm_plan"]),
        pzp=_plan_run(nz, tuning["zp_plan"]), px=_plan_run(nx // 2, tuning["x_plan"]))


def measured_traffic(kernel: str, bytes_per_launch: float):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (profiles/*_pmc.txt): its measured/algorithmic ratio times this
    run's algorithmic bytes per launch.  None when no summary covers the
    kernel or when the library sources changed since the counters were taken
    (sha256 over csrc/)."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2102_00755_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    sha = h.hexdigest()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_pmc.txt"))):
        ratios, cur, file_sha = {}, None, None
        with open(path) as fh:
            for line in fh:
                if ": " not in line or line.startswith(" "):
                    continue
                k, v = line.rstrip("\n").split(": ", 1)
                if k == "kernel":
                    cur = v
                elif k == "traffic_over_algorithmic" and cur is not None:
                    ratios[cur] = float(v)
                elif k == "source_sha256":
                    file_sha = v
        if file_sha == sha and kernel in ratios:
            return round(ratios[kernel] * bytes_per_launch, 1)
    return None


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed TR gradients")
    ap.add_argument("--warmup", type=int, default=1, help="untimed TR gradients")
    ap.add_argument("--config", default="full", help="synth config name (default: the full-size workload)")
    ap.add_argument("--nt", type=int, default=None, help="override the number of time steps")
    ap.add_argument("--timing-every", type=int, default=16, help="sample pass launches every k steps")
    ap.add_argument("--cpu-nt", type=int, default=3, help="time steps of the oracle sample")
    ap.add_argument("--cpu-nt-single", type=int, default=2,
                    help="time steps of the single-thread oracle sample (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tile-bytes", type=int, nargs=3, metavar=("Y", "ZM", "ZP"), default=None,
                    help="axis-pass tile bytes (fwi_set_tuning) instead of the library defaults")
    ap.add_argument("--autotune", action="store_true", help="apply the autotuner's cached or measured choice")
    return ap.parse_args()


def executed_steps(nt: int) -> int:
    """Wave-simulation steps one TR gradient of nt steps executes (Alg. 1):
    nt forward, nt adjoint and nt - 1 TR steps (the TR pre-step and the
    nt - 2 paired steps; TR step k >= nt is never run)."""
    return 3 * nt - 1 if nt >= 2 else 2 * nt


def _time_oracle(prob, nt_cpu: int, workers: int):
    import numpy as np  # noqa: F401

    from oracle import kspace as ks
    from synth.configs import random_traces

    w = ks.rademacher(prob.enc_seed, prob.n_src)
    S = prob.src_signals()[:nt_cpu]
    obs = random_traces(nt_cpu, prob.n_rec, seed=99, scale=1e-3)
    saved = ks._WORKERS
    ks._WORKERS = workers            # the FFT thread count the oracle's calls read
    try:
        t0 = time.perf_counter()
        sch = ks.scheme_for(prob)
        t1 = time.perf_counter()
        ks.tr_gradient(sch, prob.c_eval, prob.src_ijk, S, w, prob.rec_ijk, obs, prob.gamma, prob.boundary,
                       nt_cpu)
        t2 = time.perf_counter()
    finally:
        ks._WORKERS = saved
    return t1 - t0, t2 - t1


def cpu_baseline(prob, nt_cpu: int, nt_single: int) -> dict:
    """FP64 oracle TR gradient of the same grid, geometry and medium on a
    truncated horizon, timed on this host: nt_cpu steps with the oracle's
    FFT thread count, and nt_single steps with one thread.  The rate credits
    only the simulation steps the truncated gradient executes."""
    from oracle import kspace as ks

    workers = int(ks._WORKERS)
    setup, t = _time_oracle(prob, nt_cpu, workers)
    steps = executed_steps(nt_cpu)
    out = {
        "value": prob.n_cells * steps / t / 1e6,
        "unit": "Mcell-steps/s",
        "cores": workers,
        "kind": "oracle",
        "sample": (f"FP64 oracle TR gradient on the same {prob.shape[2]}x{prob.shape[1]}x{prob.shape[0]} "
                   f"grid, geometry and medium, truncated to {nt_cpu} time steps = {steps} executed "
                   f"simulation steps ({nt_cpu} forward, {nt_cpu} adjoint, {max(nt_cpu - 1, 0)} TR), "
                   f"{t:.2f} s; rate = cells x executed steps / time; operator setup ({setup:.1f} s) "
                   f"excluded; scipy.fft workers={workers}; host {os.cpu_count()} logical CPUs"),
        "seconds": round(t, 3),
        "executed_steps": steps,
    }
    if nt_single > 0:
        _, t1 = _time_oracle(prob, nt_single, 1)
        s1 = executed_steps(nt_single)
        out["single_worker"] = {"value": round(prob.n_cells * s1 / t1 / 1e6, 3), "cores": 1,
                                "nt": nt_single, "executed_steps": s1, "seconds": round(t1, 3)}
    return out


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the multi-GPU path "
                          "(independent encoded gradients averaged across GPUs) is not built",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2102_00755_amd.fwi import Handle, rademacher
    from synth import make_config

    prob = make_config(args.config, nt=args.nt)
    nz, ny, nx = prob.shape
    h = Handle.from_problem(prob, batch=1, precision=4)
    if args.tile_bytes:
        h.tuning = dict(zip(("y_tile_bytes", "zm_tile_bytes", "zp_tile_bytes"), args.tile_bytes))
    if args.autotune:
        from paper_2102_00755_amd import autotune
        autotune.apply(h)
    dev = h.device
    w = torch.from_numpy(rademacher(prob.enc_seed, prob.n_src)).to(dev)
    S = torch.from_numpy(prob.src_signals()).to(dev, torch.float32)
    c_eval = torch.from_numpy(prob.c_eval).to(dev, torch.float32)
    c_true = torch.from_numpy(prob.c_true).to(dev, torch.float32)
    obs = h.forward(c_true, S, w)            # synthetic observed data (also the forward warm-up)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h.forward(c_true, S, w)                  # forward-only throughput (one simulation)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    grad = torch.empty((1, nz, ny, nx), device=dev, dtype=torch.float32)
    for _ in range(args.warmup):
        h.gradient(c_eval, S, w, obs, out=grad)
    torch.cuda.synchronize()

    h.timing_enable(args.timing_every)
    h.timing_read()
    lat = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        t0 = time.perf_counter()
        mis, _ = h.gradient(c_eval, S, w, obs, out=grad)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    h.timing_enable(0)
    passes = h.timing_read()
    misfit = float(mis[0])
    gfinite = bool(torch.isfinite(grad).all())

    cells = prob.n_cells
    work = 3.0 * cells * prob.nt * args.steps
    value = work / total / 1e6
    lat_ms = np.array(lat) * 1e3

    per_pass = {}
    for name, (n, ms, by) in passes.items():
        if n:
            per_pass[name] = {"launches_sampled": n, "avg_ms": ms / n, "GB/s": by / (ms * 1e-3) / 1e9,
                              "bytes_per_launch": by / n}
    dom = max(per_pass, key=lambda k: per_pass[k]["avg_ms"] * passes[k][0]) if per_pass else None
    tn = h.tuning
    roof = None
    if dom:
        d = per_pass[dom]
        roof = {
            "bound": "hbm",
            "achieved": round(d["GB/s"], 1),
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": round(d["GB/s"] / PEAK_HBM_GBS, 4),
            "traffic": measured_traffic(kernel_symbol(dom, nx, ny, nz, tn), d["bytes_per_launch"]),
            "kernel": kernel_symbol(dom, nx, ny, nz, tn),
            "avg_ms": round(d["avg_ms"], 4),
            "bytes_per_launch": d["bytes_per_launch"],
        }

    step_b = step_bytes_per_cell(prob.shape, prob.pml)
    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "Mcell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(total / args.steps * 1e3, 2),
        "p50_ms": round(float(np.percentile(lat_ms, 50)), 2),
        "p99_ms": round(float(np.percentile(lat_ms, 99)), 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"{args.config}: {nx}x{ny}x{nz} grid, dx {prob.dx * 1e3:g} mm, PML {prob.pml[0]}, "
                         f"{prob.nt} FP32 time steps, {prob.n_src} Rademacher-encoded emitters, "
                         f"{prob.n_rec} receivers, breast-like phantom; one encoded TR gradient "
                         f"(3 wave simulations) per step"),
            "grid": [nx, ny, nz], "nt": prob.nt, "n_src": prob.n_src, "n_rec": prob.n_rec,
            "gamma_voxels": int(prob.gamma.sum()), "boundary_voxels": int(prob.boundary.sum()),
        },
        "roofline": roof,
        "whole_gradient": {
            "bytes_per_cell_step": round(step_b, 2),
            "executed_steps": executed_steps(prob.nt),
            "achieved_GBps": round(step_b * cells * executed_steps(prob.nt) * args.steps
                                   / total / 1e9, 1),
            "frac": round(step_b * cells * executed_steps(prob.nt) * args.steps
                          / total / 1e9 / PEAK_HBM_GBS, 4),
        },
        "per_pass": {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                     for k, v in per_pass.items()},
        "misfit": misfit,
        "grad_finite": gfinite,
        "forward_Mcell_steps_per_s": round(cells * prob.nt / t_fwd / 1e6, 1),
        "gradients_per_hour": round(3600.0 * args.steps / total, 1),
        "tuning": h.tuning,
    }
    h.close()
    del obs, grad, c_eval, c_true, S
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_nt, args.cpu_nt_single)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
