"""Serving loop: concurrent forward / gradient solves over several grid levels.

Requests (a forward simulation or an encoded TR gradient on one of the
configured grid levels, e.g. the levels of a coarse-to-fine multigrid scheme,
Sec. 3.3) arrive at any time.  A dispatcher admits a waiting request as soon
as a solver slot is free and its device footprint fits the HBM budget: a
resident handle of that level is reused when one is idle, otherwise a new one
is created if ``fwi_workspace_bytes`` still fits.  Admitted requests run on
their own HIP streams from worker threads, so their kernels overlap on the
device with those of requests already running; handles (fields, spectra,
tape) stay on the device between requests.  Results are identical to a solve
run alone: every kernel is deterministic and a handle is used by one request
at a time.

Per-request latency runs from arrival to result; ``stats()`` reports
p50 / p99 latency and the aggregate throughput in Mcell-steps/s (a forward
solve counts one simulation, a gradient three).
"""

from __future__ import annotations

import collections
import concurrent.futures as cf
import dataclasses
import threading
import time
from typing import Dict, List, Optional

import numpy as np
import torch

from . import fwi


@dataclasses.dataclass
class Level:
    """One grid level: handle arguments (``fwi.problem_kwargs``) and precision;
    ``tuning`` (optional, e.g. from ``autotune.apply``) is set on every handle
    the server creates for the level."""

    name: str
    kwargs: dict
    tuning: Optional[dict] = None

    @property
    def n_cells(self) -> int:
        nz, ny, nx = self.kwargs["shape"]
        return nz * ny * nx

    @property
    def nt(self) -> int:
        return int(self.kwargs["nt"])


@dataclasses.dataclass
class _Request:
    rid: int
    kind: str                      # "forward" or "gradient"
    level: str
    c: torch.Tensor
    src: torch.Tensor
    w: torch.Tensor
    obs: Optional[torch.Tensor]
    t_arrival: float
    future: cf.Future
    t_start: float = 0.0
    t_done: float = 0.0


class Server:
    def __init__(self, levels: List[Level], budget_bytes: int, max_inflight: int = 4, device: int = 0):
        self.levels: Dict[str, Level] = {lv.name: lv for lv in levels}
        self.budget = int(budget_bytes)
        self.max_inflight = int(max_inflight)
        self.device = torch.device("cuda", device)
        self.footprint = {lv.name: fwi.workspace_bytes(**dict(lv.kwargs), batch=1) for lv in levels}
        for name, fp in self.footprint.items():
            if fp <= 0 or fp > self.budget:
                raise ValueError(f"level {name}: footprint {fp} does not fit the budget {self.budget}")
        self._idle: Dict[str, List[fwi.Handle]] = collections.defaultdict(list)
        self._all_handles: List[fwi.Handle] = []
        self._used = 0
        self._inflight = 0
        self._pending: collections.deque = collections.deque()
        self._done: List[_Request] = []
        self._lock = threading.Condition()
        self._pool = cf.ThreadPoolExecutor(max_workers=self.max_inflight)
        self._streams = [torch.cuda.Stream(device=self.device) for _ in range(self.max_inflight)]
        self._free_streams = list(range(self.max_inflight))
        self._rid = 0
        self._stop = False
        self._t0 = None
        self._dispatcher = threading.Thread(target=self._dispatch, daemon=True)
        self._dispatcher.start()

    # ------------------------------------------------------------------ API
    def submit(self, kind: str, level: str, c, src, w, obs=None) -> cf.Future:
        if kind not in ("forward", "gradient"):
            raise ValueError(kind)
        if level not in self.levels:
            raise KeyError(level)
        if kind == "gradient" and obs is None:
            raise ValueError("a gradient request needs observed data")
        fut: cf.Future = cf.Future()
        with self._lock:
            if self._t0 is None:
                self._t0 = time.perf_counter()
            req = _Request(self._rid, kind, level, c, src, w, obs, time.perf_counter(), fut)
            self._rid += 1
            self._pending.append(req)
            self._lock.notify_all()
        return fut

    def drain(self) -> None:
        with self._lock:
            while self._pending or self._inflight:
                self._lock.wait(0.05)

    def close(self) -> None:
        self.drain()
        with self._lock:
            self._stop = True
            self._lock.notify_all()
        self._dispatcher.join()
        self._pool.shutdown(wait=True)
        for h in self._all_handles:
            h.close()
        self._all_handles.clear()

    def stats(self) -> dict:
        with self._lock:
            done = list(self._done)
        if not done:
            return {}
        lat = np.array([r.t_done - r.t_arrival for r in done]) * 1e3
        work = 0.0
        for r in done:
            lv = self.levels[r.level]
            work += lv.n_cells * lv.nt * (3 if r.kind == "gradient" else 1)
        t_first = min(r.t_arrival for r in done)
        t_last = max(r.t_done for r in done)
        return {
            "requests": len(done),
            "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()),
            "Mcell-steps/s": work / (t_last - t_first) / 1e6,
            "wall_s": t_last - t_first,
            "device_bytes": self._used,
            "handles": len(self._all_handles),
        }

    # ------------------------------------------------------------ internals
    def _acquire(self, level: str) -> Optional[fwi.Handle]:
        """An idle resident handle of `level`, or a new one if it fits."""
        if self._idle[level]:
            return self._idle[level].pop()
        fp = self.footprint[level]
        if self._used + fp > self.budget:
            # free idle handles of other levels to make room
            for other, hs in self._idle.items():
                while hs and self._used + fp > self.budget:
                    h = hs.pop()
                    self._all_handles.remove(h)
                    h.close()
                    self._used -= self.footprint[other]
            if self._used + fp > self.budget:
                return None
        h = fwi.Handle(**self.levels[level].kwargs, batch=1, device=self.device.index or 0)
        if self.levels[level].tuning:
            h.tuning = self.levels[level].tuning
        self._used += fp
        self._all_handles.append(h)
        return h

    def _dispatch(self) -> None:
        with self._lock:
            while not self._stop:
                admitted = False
                if self._inflight < self.max_inflight:
                    for req in list(self._pending):
                        h = self._acquire(req.level)
                        if h is None:
                            continue
                        self._pending.remove(req)
                        self._inflight += 1
                        sidx = self._free_streams.pop()
                        req.t_start = time.perf_counter()
                        self._pool.submit(self._run, req, h, sidx)
                        admitted = True
                        break
                if not admitted:
                    self._lock.wait(0.01)

    def _run(self, req: _Request, h: fwi.Handle, sidx: int) -> None:
        stream = self._streams[sidx]
        try:
            with torch.cuda.stream(stream):
                c = req.c.to(h.device, h.dtype, non_blocking=False)
                src = req.src.to(h.device, h.dtype)
                w = req.w.to(h.device)
                if req.kind == "forward":
                    out = h.forward(c, src, w)
                else:
                    obs = req.obs.to(h.device, h.dtype)
                    out = h.gradient(c, src, w, obs)
                stream.synchronize()
            req.t_done = time.perf_counter()
            req.future.set_result(out)
        except Exception as e:  # noqa: BLE001 - reported through the future
            req.t_done = time.perf_counter()
            req.future.set_exception(e)
        finally:
            with self._lock:
                self._idle[req.level].append(h)
                self._free_streams.append(sidx)
                self._inflight -= 1
                if not req.future.exception():
                    self._done.append(req)
                self._lock.notify_all()
