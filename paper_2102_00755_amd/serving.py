"""Serving loop: continuous batching of forward / gradient solves over grid levels.

Requests (a forward simulation or an encoded TR gradient on one of the
configured grid levels, e.g. the levels of a coarse-to-fine multigrid scheme,
Sec. 3.3) arrive at any time.  Each level keeps resident handles of batch
capacity ``Level.batch`` on the device (fields, spectra, tape stay allocated
between requests).  Whenever one of ``max_inflight`` call slots is free, the
dispatcher takes the oldest waiting request together with the later waiting
requests of the same level and kind, up to the capacity, and enqueues them as
ONE batched call: every pass launch of that call covers all of them, and its
time step is replayed as a hipGraph.  Requests that arrive while others are
on the GPU are admitted as soon as a slot and device memory free up (a new
handle is created when its ``fwi_workspace_bytes`` footprint fits the HBM
budget, evicting idle handles of other levels if needed).

One dispatcher thread makes every GPU call of the server: the library's
calls are asynchronous, so the dispatcher enqueues each batched call on its
own HIP stream, records an event behind it and goes on admitting; calls on
different streams overlap on the device, and a request's future is resolved
when its call's event has completed.  (Keeping all GPU work of the server in
one thread also keeps the step-graph captures free of other threads'
synchronous copies, which invalidate a capture.)

Results are identical to a solve run alone: every kernel is deterministic, a
batched call computes each problem exactly as a batch-1 call does, graph
replay equals eager launches, and a handle serves one call at a time.

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
    requests one batched call may hold (the handles' batch capacity), whether
    calls replay their time step as a hipGraph, and an optional launch tuning
    (e.g. from ``autotune.apply``) set on every handle of the level."""

    name: str
    kwargs: dict
    tuning: Optional[dict] = None
    batch: int = 4
    graph: bool = True

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


@dataclasses.dataclass
class _Call:
    """One enqueued batched call: its requests, handle, stream and completion event."""

    group: List[_Request]
    level: str
    handle: Optional[fwi.Handle]
    reserved: bool
    evict: List[fwi.Handle]
    sidx: int
    event: Optional[torch.cuda.Event] = None
    outs: Optional[list] = None
    error: Optional[BaseException] = None


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
        self._inflight: List[_Call] = []
        self._pending: collections.deque = collections.deque()
        self._done: List[_Request] = []
        self._calls = 0
        self._lock = threading.Condition()
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

    def _admit(self) -> List[_Call]:
        """Under the lock: the calls to enqueue now (groups of waiting
        requests with a handle or a reservation each, and a stream)."""
        calls: List[_Call] = []
        if self._paused:
            return calls
        while len(self._inflight) + len(calls) < self.max_inflight and self._pending:
            admitted = None
            seen = set()
            for head in self._pending:
                key = (head.level, head.kind)
                if key in seen:
                    continue
                seen.add(key)
                got = self._reserve(head.level)
                if got is not None:
                    cap = self.levels[head.level].batch
                    group = [r for r in self._pending if (r.level, r.kind) == key][:cap]
                    admitted = _Call(group, head.level, got[0], got[1], got[2], self._free_streams.pop())
                    break
            if admitted is None:
                break
            now = time.perf_counter()
            for r in admitted.group:
                self._pending.remove(r)
                r.t_start = now
            self._calls += 1
            calls.append(admitted)
        self._inflight.extend(calls)
        return calls

    def _dispatch(self) -> None:
        while True:
            with self._lock:
                if self._stop and not self._pending and not self._inflight:
                    return
                calls = self._admit()
            for call in calls:
                self._enqueue(call)
            finished = [c for c in list(self._inflight) if c.error is not None or c.event.query()]
            for call in finished:
                self._finish(call)
            if not calls and not finished:
                with self._lock:
                    self._lock.wait(0.0005 if self._inflight else 0.01)

    def _enqueue(self, call: _Call) -> None:
        """Create the handle if reserved, copy the inputs and enqueue the
        batched call on the call's stream (asynchronous), then its event."""
        lv = self.levels[call.level]
        group = call.group
        stream = self._streams[call.sidx]
        try:
            for e in call.evict:
                e.close()
            if call.handle is None:
                call.handle = fwi.Handle(**lv.kwargs, batch=lv.batch, device=self.device.index or 0)
                if lv.tuning:
                    call.handle.tuning = lv.tuning
                with self._lock:
                    self._all_handles.append(call.handle)
            h = call.handle
            h.use_graph = lv.graph
            with torch.cuda.stream(stream):
                for r in group:
                    if r.ready is not None:
                        stream.wait_event(r.ready)
                c = torch.stack([torch.as_tensor(r.c).to(h.device, h.dtype) for r in group])
                src = torch.stack([torch.as_tensor(r.src).to(h.device, h.dtype) for r in group])
                w = torch.stack([torch.as_tensor(r.w).to(h.device, torch.int8) for r in group])
                if group[0].kind == "forward":
                    tr = h.forward(c, src, w)
                    call.outs = [tr[b:b + 1].clone() for b in range(len(group))]
                else:
                    obs = torch.stack([torch.as_tensor(r.obs).to(h.device, h.dtype) for r in group])
                    mis, grad = h.gradient(c, src, w, obs)
                    call.outs = [(mis[b:b + 1].clone(), grad[b:b + 1].clone()) for b in range(len(group))]
                call.event = torch.cuda.Event()
                call.event.record(stream)
        except Exception as e:  # noqa: BLE001 - reported through the futures
            call.error = e

    def _finish(self, call: _Call) -> None:
        t_done = time.perf_counter()
        with self._lock:
            self._inflight.remove(call)
            if call.handle is not None:
                self._idle[call.level].append(call.handle)
            elif call.reserved:
                self._used -= self.footprint[call.level]   # creation failed: release the reservation
            self._free_streams.append(call.sidx)
            for r in call.group:
                r.t_done = t_done
                if call.error is None:
                    self._done.append(r)
            self._lock.notify_all()
        for b, r in enumerate(call.group):
            if call.error is None:
                r.future.set_result(call.outs[b])
            else:
                r.future.set_exception(call.error)
