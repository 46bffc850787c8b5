"""Autotuner of the launch tuning of a handle, with a persisted JSON cache.

The tunable launch parameters (``fwi_set_tuning``) are the row segments of
the axis-pass tiles (64 or 128 bytes) of the three axis-pass kinds — y
passes, the z pass of d- (Z1) and the z pass of d+ (Z2) — and the radix plans
of the transforms of the y passes, Z1, Z2 and the x passes (two orders of the
same radices each).  A short-horizon
twin of the handle (same grid, geometry, precision and batch, ``steps`` time
steps) runs a forward simulation per candidate, timing every pass launch
with the library's HIP-event timer:

* tiles: each kind runs as its own kernels, so per kind the width with the
  least time per launch wins;
* radix plans (y passes, Z1, Z2, x passes): with the chosen tiles, by
  coordinate descent on the total time per time step of all passes (a plan
  changes a pass's compute and memory timing, which the neighbouring passes
  feel): each kind's plan is switched to 1 if that lowers the total.

Results are bit-identical across tile widths; the two radix plans agree to
rounding.  The choice changes speed only.

The cache maps a key (device name, precision, grid, batch) to the chosen
tuning; it lives in ``$FWI_TUNING_CACHE`` or
``~/.cache/paper_2102_00755_amd/tuning.json``.

    from paper_2102_00755_amd import autotune
    autotune.apply(handle)            # cached choice, measured on a miss
"""

from __future__ import annotations

import json
import os
from typing import Callable, Dict, Optional

import torch

from . import fwi

TILE_BYTES = (64, 128)
# pass kinds of the per-pass timer that each tuning field governs
KIND_PASSES = {
    "y_tile_bytes": ("y_fwd", "y_inv", "y_vel_q"),
    "zm_tile_bytes": ("z_minus",),
    "zp_tile_bytes": ("z_plus",),
}


def cache_path() -> str:
    return os.environ.get("FWI_TUNING_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "paper_2102_00755_amd", "tuning.json")


def cache_key(device_name: str, precision: int, shape, batch: int) -> str:
    nz, ny, nx = (int(v) for v in shape)
    return f"{device_name}|fp{8 * int(precision)}|{nz}x{ny}x{nx}|B{int(batch)}"


def load_cache(path: Optional[str] = None) -> Dict[str, dict]:
    path = path or cache_path()
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def save_cache(cache: Dict[str, dict], path: Optional[str] = None) -> None:
    path = path or cache_path()
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def choose(per_width: Dict[int, Dict[str, float]]) -> dict:
    """Per tuning field, the tile width with the least summed ms per launch of
    its pass kinds.  per_width: {tile bytes: {pass name: ms per launch}}."""
    out = {}
    for field, passes in KIND_PASSES.items():
        best = None
        for tb, t in sorted(per_width.items()):
            cost = sum(t[p] for p in passes if p in t)
            if best is None or cost < best[1]:
                best = (tb, cost)
        out[field] = int(best[0])
    return out


def measure(handle: "fwi.Handle", steps: int = 24, repeats: int = 2) -> Dict[int, Dict[str, float]]:
    """ms per launch of every pass kind for each tile width, on a twin of
    `handle` with `steps` time steps (a forward simulation of zero sources in
    a homogeneous medium: the launch pattern and traffic of every step)."""
    kw = dict(handle.kwargs)
    kw["nt"] = int(steps)
    twin = fwi.Handle(**kw, batch=handle.batch, device=handle.device.index or 0)
    try:
        dev, dt = twin.device, twin.dtype
        c0 = 0.5 * (float(kw["c_min"]) + float(kw["c_max"]))
        c = torch.full((twin.batch,) + twin.shape, c0, device=dev, dtype=dt)
        src = torch.zeros((twin.batch, twin.nt, twin.n_src), device=dev, dtype=dt)
        w = torch.ones((twin.batch, twin.n_src), device=dev, dtype=torch.int8)
        out: Dict[int, Dict[str, float]] = {}
        for tb in TILE_BYTES:
            twin.tuning = {"y_tile_bytes": tb, "zm_tile_bytes": tb, "zp_tile_bytes": tb}
            twin.forward(c, src, w)                       # warm-up
            torch.cuda.synchronize(dev)
            best: Dict[str, float] = {}
            for _ in range(repeats):
                twin.timing_enable(1)
                twin.timing_read()
                twin.forward(c, src, w)
                torch.cuda.synchronize(dev)
                twin.timing_enable(0)
                for name, (n, ms, _) in twin.timing_read().items():
                    if n:
                        best[name] = min(best.get(name, float("inf")), ms / n)
            out[tb] = best
        return out
    finally:
        twin.close()


PLAN_FIELDS = ("y_plan", "zm_plan", "zp_plan", "x_plan")


def step_ms(handle: "fwi.Handle", tunings, steps: int = 24, repeats: int = 2) -> list:
    """Total ms per time step (all passes) of a forward simulation under each
    tuning of `tunings`, on the same kind of twin as ``measure``."""
    kw = dict(handle.kwargs)
    kw["nt"] = int(steps)
    twin = fwi.Handle(**kw, batch=handle.batch, device=handle.device.index or 0)
    try:
        dev, dt = twin.device, twin.dtype
        c0 = 0.5 * (float(kw["c_min"]) + float(kw["c_max"]))
        c = torch.full((twin.batch,) + twin.shape, c0, device=dev, dtype=dt)
        src = torch.zeros((twin.batch, twin.nt, twin.n_src), device=dev, dtype=dt)
        w = torch.ones((twin.batch, twin.n_src), device=dev, dtype=torch.int8)
        out = []
        for tuning in tunings:
            twin.tuning = tuning
            twin.forward(c, src, w)                       # warm-up
            torch.cuda.synchronize(dev)
            best = float("inf")
            for _ in range(repeats):
                twin.timing_enable(1)
                twin.timing_read()
                twin.forward(c, src, w)
                torch.cuda.synchronize(dev)
                twin.timing_enable(0)
                tim = twin.timing_read()
                best = min(best, sum(ms for (_, ms, _) in tim.values()) / twin.nt)
            out.append(best)
        return out
    finally:
        twin.close()


def choose_plans(handle: "fwi.Handle", tiles: dict, steps: int = 24, step_fn: Optional[Callable] = None):
    """Radix plans by coordinate descent on the total step time: starting from
    plan 0 everywhere, each pass kind's plan is switched to 1 if that lowers
    the time.  Returns (plans, [(tuning, ms per step), ...])."""
    fn = step_fn or step_ms
    cur = dict(tiles, **{f: 0 for f in PLAN_FIELDS})
    best = fn(handle, [cur], steps)[0]
    log = [(dict(cur), best)]
    for f in PLAN_FIELDS:
        trial = dict(cur, **{f: 1})
        t = fn(handle, [trial], steps)[0]
        log.append((dict(trial), t))
        if t < best:
            cur, best = trial, t
    return {f: int(cur[f]) for f in PLAN_FIELDS}, log


def tune(handle: "fwi.Handle", steps: int = 24, cache: Optional[str] = None,
         measure_fn: Optional[Callable] = None, step_fn: Optional[Callable] = None) -> dict:
    """Measure, choose, store in the cache and apply; returns the tuning."""
    per_width = (measure_fn or measure)(handle, steps)
    choice = choose(per_width)
    plans, log = choose_plans(handle, choice, steps, step_fn)
    choice.update(plans)
    key = cache_key(torch.cuda.get_device_name(handle.device), handle.precision, handle.shape, handle.batch)
    data = load_cache(cache)
    data[key] = dict(choice, measured_ms_per_launch={str(k): v for k, v in per_width.items()},
                     measured_ms_per_step_by_plans=[[t, ms] for t, ms in log], steps=int(steps))
    save_cache(data, cache)
    handle.tuning = choice
    return choice


def apply(handle: "fwi.Handle", cache: Optional[str] = None, steps: int = 24) -> dict:
    """Apply the cached tuning of the handle's key, measuring it on a miss."""
    key = cache_key(torch.cuda.get_device_name(handle.device), handle.precision, handle.shape, handle.batch)
    entry = load_cache(cache).get(key)
    if entry is not None and all(f in entry for f in PLAN_FIELDS):
        choice = {f: int(entry[f]) for f in tuple(KIND_PASSES) + PLAN_FIELDS}
        handle.tuning = choice
        return choice
    return tune(handle, steps=steps, cache=cache)
