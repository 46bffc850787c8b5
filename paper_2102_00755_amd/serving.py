"""Serving loop: continuous batching of forward / gradient solves over grid levels.

Requests (a forward simulation or an encoded TR gradient on one of the
configured grid levels, e.g. the levels of a coarse-to-fine multigrid scheme,
Sec. 3.3) arrive at any time.  Each level keeps resident handles of batch
capacity ``Level.batch`` on the device (fields, spectra, tape stay allocated
between requests).  Whenever a solver slot is free, the dispatcher takes the
oldest waiting request together with the later waiting requests of the same
level and kind, up to the capacity, and runs them as ONE batched call: every
pass launch of that call covers all of them.  Requests that arrive while
others are on the GPU are admitted as soon as a slot and device memory free
up (a new handle is created when its ``fwi_workspace_bytes`` footprint fits
the HBM budget, evicting idle handles of other levels if needed); admitted
calls run on their own HIP streams from worker threads, so their kernels
overlap on the device with the calls already running.

Results are identical to a solve run alone: every kernel is deterministic, a
batched call computes each problem exactly as a batch-1 call does, and a
handle serves one call at a time.

Per-request latency runs from arrival to result; ``stats()`` reports
p50 / p99 latency, the aggregate throughput in Mcell-steps/s (a forward solve
counts one simulation, a gradient three) and the mean number of requests per
batched call.
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
    """One grid level: handle arguments (``fwi.problem_kwargs``), the number of
    requests one batched call may hold (the handles' batch capacity), and an
    optional launch tuning (e.g. from ``autotune.apply``) set on every handle
    of the level.  Served calls launch their passes eagerly: a step-graph
    capture (FWI_GRAPH) on one worker's stream is invalidated when another
    worker makes a synchronous copy or creates a handle meanwhile."""

    name: str
    kwargs: dict
    tuning: Optional[dict] = None
    batch: int = 4

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
    ready: Optional[torch.cuda.Event]   # inputs written on the submitter's stream
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
        for lv in levels:
            if lv.batch < 1:
                raise ValueError(f"level {lv.name}: batch must be >= 1")
        self.footprint = {lv.name: fwi.workspace_bytes(**dict(lv.kwargs), batch=lv.batch) for lv in levels}
        for name, fp in self.footprint.items():
            if fp <= 0 or fp > self.budget:
                raise ValueError(f"level {name}: footprint {fp} does not fit the budget {self.budget}")
        self._idle: Dict[str, List[fwi.Handle]] = collections.defaultdict(list)
        self._all_handles: List[fwi.Handle] = []
        self._used = 0                  # bytes of resident and reserved handles
        self._inflight = 0
        self._pending: collections.deque = collections.deque()
        self._done: List[_Request] = []
        self._calls = 0
        self._lock = threading.Condition()
        self._pool = cf.ThreadPoolExecutor(max_workers=self.max_inflight)
        self._streams = [torch.cuda.Stream(device=self.device) for _ in range(self.max_inflight)]
        self._free_streams = list(range(self.max_inflight))
        self._rid = 0
        self._stop = False
        self._paused = False
        self._dispatcher = threading.Thread(target=self._dispatch, daemon=True)
        self._dispatcher.start()

    # ------------------------------------------------------------------ API
    def submit(self, kind: str, level: str, c, src, w, obs=None) -> cf.Future:
        """Queue one solve; the future's result is what ``Handle.forward``
        (traces [1, nt, n_rec]) or ``Handle.gradient`` ((misfit [1],
        gradient [1, nz, ny, nx])) returns for this problem alone.  Inputs may
        be host or device tensors; device inputs are read only after the work
        queued so far on the caller's current stream."""
        if kind not in ("forward", "gradient"):
            raise ValueError(kind)
        if level not in self.levels:
            raise KeyError(level)
        if kind == "gradient" and obs is None:
            raise ValueError("a gradient request needs observed data")
        ready = None
        if any(isinstance(t, torch.Tensor) and t.is_cuda for t in (c, src, w, obs)):
            ready = torch.cuda.Event()
            ready.record(torch.cuda.current_stream(self.device))
        fut: cf.Future = cf.Future()
        with self._lock:
            req = _Request(self._rid, kind, level, c, src, w, obs, ready, time.perf_counter(), fut)
            self._rid += 1
            self._pending.append(req)
            self._lock.notify_all()
        return fut

    def pause(self) -> None:
        """Stop admitting requests (calls already admitted keep running)."""
        with self._lock:
            self._paused = True

    def resume(self) -> None:
        with self._lock:
            self._paused = False
            self._lock.notify_all()

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

    def reset_stats(self) -> None:
        """Forget the completed requests (e.g. after a warm-up)."""
        with self._lock:
            self._done.clear()
            self._calls = 0

    def stats(self) -> dict:
        with self._lock:
            done = list(self._done)
            calls = self._calls
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
            "calls": calls,
            "mean_batch": len(done) / max(calls, 1),
            "device_bytes": self._used,
            "handles": len(self._all_handles),
        }

    # ------------------------------------------------------------ internals
    def _reserve(self, level: str):
        """Under the lock: an idle resident handle of `level`, else a
        reservation of its footprint (the handle is created by the worker,
        outside the lock), evicting idle handles of other levels if needed.
        Returns (handle or None, reserved, handles to close) or None when the
        level does not fit now."""
        if self._idle[level]:
            return self._idle[level].pop(), False, []
        fp = self.footprint[level]
        evict = []
        if self._used + fp > self.budget:
            freeable = sum(self.footprint[o] * len(hs) for o, hs in self._idle.items() if o != level)
            if self._used - freeable + fp > self.budget:
                return None
            for other, hs in self._idle.items():
                while hs and self._used + fp > self.budget:
                    h = hs.pop()
                    self._all_handles.remove(h)
                    self._used -= self.footprint[other]
                    evict.append(h)
        self._used += fp
        return None, True, evict

    def _dispatch(self) -> None:
        with self._lock:
            while not self._stop:
                admitted = False
                if not self._paused and self._inflight < self.max_inflight and self._pending:
                    seen = set()
                    for head in list(self._pending):
                        key = (head.level, head.kind)
                        if key in seen:
                            continue
                        seen.add(key)
                        got = self._reserve(head.level)
                        if got is None:
                            continue
                        cap = self.levels[head.level].batch
                        group = [r for r in self._pending if (r.level, r.kind) == key][:cap]
                        for r in group:
                            self._pending.remove(r)
                        self._inflight += 1
                        self._calls += 1
                        sidx = self._free_streams.pop()
                        now = time.perf_counter()
                        for r in group:
                            r.t_start = now
                        self._pool.submit(self._run, group, got, sidx)
                        admitted = True
                        break
                if not admitted:
                    self._lock.wait(0.01)

    def _run(self, group: List[_Request], got, sidx: int) -> None:
        h, reserved, evict = got
        lv = self.levels[group[0].level]
        stream = self._streams[sidx]
        error = None
        outs = None
        try:
            for e in evict:
                e.close()
            if h is None:
                h = fwi.Handle(**lv.kwargs, batch=lv.batch, device=self.device.index or 0)
                if lv.tuning:
                    h.tuning = lv.tuning
                with self._lock:
                    self._all_handles.append(h)
            h.use_graph = False
            with torch.cuda.stream(stream):
                for r in group:
                    if r.ready is not None:
                        stream.wait_event(r.ready)
                c = torch.stack([torch.as_tensor(r.c).to(h.device, h.dtype) for r in group])
                src = torch.stack([torch.as_tensor(r.src).to(h.device, h.dtype) for r in group])
                w = torch.stack([torch.as_tensor(r.w).to(h.device, torch.int8) for r in group])
                if group[0].kind == "forward":
                    tr = h.forward(c, src, w)
                    outs = [tr[b:b + 1].clone() for b in range(len(group))]
                else:
                    obs = torch.stack([torch.as_tensor(r.obs).to(h.device, h.dtype) for r in group])
                    mis, grad = h.gradient(c, src, w, obs)
                    outs = [(mis[b:b + 1].clone(), grad[b:b + 1].clone()) for b in range(len(group))]
                stream.synchronize()
        except Exception as e:  # noqa: BLE001 - reported through the futures
            error = e
        t_done = time.perf_counter()
        with self._lock:
            if h is not None:
                self._idle[lv.name].append(h)
            elif reserved:
                self._used -= self.footprint[lv.name]   # creation failed: release the reservation
            self._free_streams.append(sidx)
            self._inflight -= 1
            for r in group:
                r.t_done = t_done
                if error is None:
                    self._done.append(r)
            self._lock.notify_all()
        for b, r in enumerate(group):
            if error is None:
                r.future.set_result(outs[b])
            else:
                r.future.set_exception(error)
