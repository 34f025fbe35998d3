"""Continuous-batching render server over ``voge_render_batch``.

Scenes stay resident in device memory.  Render requests (forward) and
gradient requests (forward + backward with an upstream image gradient) of any
image size arrive at any time.  The server

  * admits requests in arrival order while the transient device memory they
    need (image, upstream gradient, kernel gradients and their share of a
    batch workspace) fits under an HBM budget and a launch slot is free --
    requests that arrive while batches run join the next batch, so work from
    different arrivals overlaps on the device;
  * groups the admitted requests of one kind (render or gradient) into a
    batch and runs it with one ``voge_render_batch`` call on the slot's own
    stream (two slots: two batches in flight);
  * completes a batch's requests when its HIP event fires, releases their
    memory from the budget, and records arrival-to-completion latency;
  * fails a request that passes its deadline (queued: it is never launched;
    in flight: it completes at once as failed, its results are dropped, and
    its memory returns to the budget when its batch ends), and cancels a
    request on demand the same way -- the server keeps running.

The scheduling logic is host code and does not touch the GPU: an executor
does (``GpuExecutor``); tests drive the same scheduler with a simulated
executor on the CPU.
"""

from __future__ import annotations

import collections
import dataclasses
import time
from typing import Any, Callable, Deque, Dict, List, Optional, Sequence

import numpy as np

from . import _native as nat


@dataclasses.dataclass
class Request:
    """One render (backward=False) or gradient request (backward=True)."""

    scene: int
    camera: Any                        # scenes.Camera
    backward: bool = False
    K: int = 20
    eta: float = 0.01
    grad_image: Any = None             # (H, W, C) upstream gradient, host or device, for backward
    arrival: float = 0.0               # server clock, seconds
    with_camera: bool = False          # also return dL/dcamera
    deadline: Optional[float] = None   # server clock, seconds: fail the request if not done by then
    rid: int = -1
    # filled in by the server and executor
    nbytes: int = 0
    admitted: Optional[float] = None
    done: Optional[float] = None
    error: Optional[str] = None
    status: int = 0
    image: Any = None
    grad_means: Any = None
    grad_covs: Any = None
    grad_attrs: Any = None
    grad_camera: Any = None

    @property
    def rays(self) -> int:
        return int(self.camera.height) * int(self.camera.width)

    @property
    def latency(self) -> Optional[float]:
        return None if self.done is None else self.done - self.arrival


class Executor:
    """What the server needs from a device (see GpuExecutor)."""

    n_slots: int = 2

    def scene_shape(self, scene: int):            # (N, C) or None if unknown
        raise NotImplementedError

    def item_bytes(self, req: Request) -> int:    # transient device bytes of one request
        raise NotImplementedError

    def launch(self, slot: int, reqs: List[Request]):   # -> handle
        raise NotImplementedError

    def ready(self, handle) -> bool:
        raise NotImplementedError

    def collect(self, handle) -> None:            # fill outputs; raise on failure
        raise NotImplementedError

    def now(self) -> float:
        return time.perf_counter()


@dataclasses.dataclass
class _Batch:
    slot: int
    reqs: List[Request]
    nbytes: int
    handle: Any


class Server:
    """The scheduler.  Not thread-safe: one thread calls submit/pump."""

    def __init__(self, executor: Executor, budget_bytes: int, max_batch_items: int = 64,
                 max_batch_rays: int = 1 << 24, on_done: Optional[Callable[[Request], None]] = None):
        if max_batch_items < 1 or max_batch_items > nat.VOGE_MAX_BATCH:
            raise ValueError(f"max_batch_items must be in [1, {nat.VOGE_MAX_BATCH}]")
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_items = int(max_batch_items)
        self.max_rays = int(max_batch_rays)
        self.on_done = on_done
        self.queue: Deque[Request] = collections.deque()
        self.inflight: Dict[int, _Batch] = {}          # slot -> batch
        self.inflight_bytes = 0
        self.peak_bytes = 0
        self.completed: List[Request] = []
        self.batches = 0
        self._next_rid = 0

    # ---------------------------------------------------------------- intake
    def submit(self, req: Request) -> bool:
        """Queue a request; False (with req.error set) if it can never run."""
        req.rid = self._next_rid
        self._next_rid += 1
        shape = self.ex.scene_shape(req.scene)
        err = None
        if shape is None:
            err = f"unknown scene {req.scene}"
        elif req.backward and req.grad_image is None:
            err = "a gradient request needs grad_image"
        elif not 1 <= req.K <= 64 or not 0.0 < req.eta < 1.0:
            err = "K must be in [1, 64] and eta in (0, 1)"
        if err is None:
            try:
                req.nbytes = int(self.ex.item_bytes(req))
            except Exception as e:          # shapes the library rejects
                err = str(e)
        if err is None and req.nbytes > self.budget:
            err = f"request needs {req.nbytes} bytes, more than the budget of {self.budget}"
        if err is not None:
            self._finish(req, err)
            return False
        self.queue.append(req)
        return True

    @staticmethod
    def _drop_outputs(r: Request) -> None:
        r.image = r.grad_means = r.grad_covs = r.grad_attrs = r.grad_camera = None

    def _finish(self, r: Request, error: Optional[str]) -> None:
        r.done = self.ex.now()
        if error is not None:
            r.error = error
            self._drop_outputs(r)        # a failed or cancelled request hands back no results
        self.completed.append(r)
        if self.on_done:
            self.on_done(r)

    def cancel(self, req: Request) -> bool:
        """Cancel a request that is not done yet: a queued request leaves the
        queue, an in-flight one completes now as cancelled (the device work
        of its batch runs on; its memory is released when the batch ends).
        Returns False if the request was already done or is unknown."""
        if req.done is not None:
            return False
        for i, r in enumerate(self.queue):
            if r is req:
                del self.queue[i]
                self._finish(req, "cancelled")
                return True
        for b in self.inflight.values():
            if any(r is req for r in b.reqs):
                self._finish(req, "cancelled")
                return True
        return False

    def _expire(self) -> int:
        """Fail every request past its deadline, queued or in flight."""
        now = self.ex.now()
        n = 0
        late = [r for r in self.queue if r.deadline is not None and now >= r.deadline]
        if late:
            gone = {id(r) for r in late}
            self.queue = collections.deque(r for r in self.queue if id(r) not in gone)
            for r in late:
                self._finish(r, "deadline exceeded")
                n += 1
        for b in self.inflight.values():
            for r in b.reqs:
                if r.done is None and r.deadline is not None and now >= r.deadline:
                    self._finish(r, "deadline exceeded")
                    n += 1
        return n

    # -------------------------------------------------------------- progress
    def idle(self) -> bool:
        return not self.queue and not self.inflight

    def pump(self) -> int:
        """Complete finished batches, fail requests past their deadlines, then
        admit and launch while possible.  Returns the number of requests
        completed (successfully or not)."""
        n = self._complete()
        n += self._expire()
        self._admit()
        return n

    def drain(self, poll: float = 0.0) -> None:
        while not self.idle():
            if self.pump() == 0 and poll > 0:
                time.sleep(poll)

    def _complete(self) -> int:
        n = 0
        for slot in sorted(self.inflight):
            b = self.inflight[slot]
            if not self.ex.ready(b.handle):
                continue
            err = None
            try:
                self.ex.collect(b.handle)
            except Exception as e:
                err = f"batch failed: {e}"
            for r in b.reqs:
                if r.done is not None:          # cancelled or past its deadline already
                    self._drop_outputs(r)
                    continue
                self._finish(r, err)
                n += 1
            self.inflight_bytes -= b.nbytes
            del self.inflight[slot]
        return n

    def _pick(self, backward: bool) -> List[Request]:
        """Requests of one kind, in arrival order, while they fit; stops at
        the first that does not (no request overtakes an earlier one of its
        kind)."""
        out, nbytes, rays = [], 0, 0
        for r in self.queue:
            if r.backward != backward:
                continue
            if len(out) == self.max_items or (out and rays + r.rays > self.max_rays):
                break
            if self.inflight_bytes + nbytes + r.nbytes > self.budget:
                break
            out.append(r)
            nbytes += r.nbytes
            rays += r.rays
        return out

    def _admit(self) -> None:
        while self.queue:
            free = [s for s in range(self.ex.n_slots) if s not in self.inflight]
            if not free:
                return
            # the kind of the oldest waiting request goes first; the other kind
            # may go if the oldest cannot fit yet
            kinds = []
            for r in self.queue:
                if r.backward not in kinds:
                    kinds.append(r.backward)
                if len(kinds) == 2:
                    break
            batch = []
            for kind in kinds:
                batch = self._pick(kind)
                if batch:
                    break
            if not batch:
                return
            chosen = {id(r) for r in batch}
            self.queue = collections.deque(r for r in self.queue if id(r) not in chosen)
            nbytes = sum(r.nbytes for r in batch)
            t = self.ex.now()
            for r in batch:
                r.admitted = t
            slot = free[0]
            try:
                handle = self.ex.launch(slot, batch)
            except Exception as e:
                for r in batch:
                    self._finish(r, f"launch failed: {e}")
                continue
            self.inflight[slot] = _Batch(slot, batch, nbytes, handle)
            self.inflight_bytes += nbytes
            self.peak_bytes = max(self.peak_bytes, self.inflight_bytes)
            self.batches += 1


def latency_stats(reqs: Sequence[Request]) -> dict:
    lat = np.array([r.latency for r in reqs if r.error is None and r.latency is not None])
    if lat.size == 0:
        return {"n": 0}
    return {"n": int(lat.size), "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 4),
            "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 4),
            "mean_ms": round(float(lat.mean()) * 1e3, 4)}


def serve_trace(server: Server, reqs: Sequence[Request], poll: float = 0.0) -> float:
    """Feed requests at their arrival times (seconds from the call) and run
    the server until all are done.  Returns the elapsed time."""
    order = sorted(reqs, key=lambda r: r.arrival)
    t0 = server.ex.now()
    for r in order:
        r.arrival += t0
    i = 0
    while i < len(order) or not server.idle():
        now = server.ex.now()
        while i < len(order) and order[i].arrival <= now:
            server.submit(order[i])
            i += 1
        if server.pump() == 0 and poll > 0:
            time.sleep(poll)
    return server.ex.now() - t0


# ----------------------------------------------------------------- device
class GpuExecutor(Executor):
    """Runs batches with voge_render_batch, one stream per slot."""

    def __init__(self, scenes, device, n_slots: int = 2):
        import torch

        from . import render as R

        self.torch, self.R = torch, R
        self.device = device
        self.scenes = []
        for m, c, a in scenes:
            R._check_inputs(m, c, a)
            self.scenes.append((m, c, a))
        self.n_slots = n_slots
        self.streams = [torch.cuda.Stream(device) for _ in range(n_slots)]
        self.ctx = R.context(device)

    def scene_shape(self, scene: int):
        if not 0 <= scene < len(self.scenes):
            return None
        m, _, a = self.scenes[scene]
        return int(m.shape[0]), int(a.shape[1])

    def _item(self, req: Request) -> nat.VogeItem:
        m, c, a = self.scenes[req.scene]
        it = nat.VogeItem()
        it.means, it.covs, it.attrs = m.data_ptr(), c.data_ptr(), a.data_ptr()
        it.N, it.C = int(m.shape[0]), int(a.shape[1])
        it.camera = self.R.camera_struct(req.camera)
        it.params = self.R.params_struct(req.K, req.eta)
        return it

    def item_bytes(self, req: Request) -> int:
        N, C = self.scene_shape(req.scene)
        H, W = int(req.camera.height), int(req.camera.width)
        b = 4 * H * W * C                                         # image
        if req.backward:
            b += 4 * H * W * C + 4 * N * (9 + C) + 4 * 15           # upstream gradient, kernel and camera grads
        return b + nat.voge_batch_workspace_size([self._item(req)], req.backward)

    def launch(self, slot: int, reqs: List[Request]):
        """Runs the batch on the slot's stream.  The slot stream first waits
        for the caller's stream, so inputs the caller has just produced there
        (upstream gradients, scene updates) are complete before the batch
        reads them; every output is marked as used on the caller's stream, so
        the caching allocator does not hand its memory to a later launch while
        work the caller queues on it is still pending."""
        torch = self.torch
        s = self.streams[slot]
        caller = torch.cuda.current_stream(self.device)
        s.wait_stream(caller)
        arr = (nat.VogeItem * len(reqs))()
        keep = []
        f32 = dict(dtype=torch.float32, device=self.device)
        with torch.cuda.stream(s):
            for i, r in enumerate(reqs):
                it = self._item(r)
                H, W, C = int(r.camera.height), int(r.camera.width), it.C
                r.image = torch.empty((H, W, C), **f32)
                it.image = r.image.data_ptr()
                if r.backward:
                    g = r.grad_image
                    g = torch.as_tensor(g).to(self.device, torch.float32).reshape(H, W, C).contiguous()
                    keep.append(g)
                    it.grad_image = g.data_ptr()
                    r.grad_means = torch.empty((it.N, 3), **f32)
                    r.grad_covs = torch.empty((it.N, 6), **f32)
                    r.grad_attrs = torch.empty((it.N, C), **f32)
                    it.grad_means, it.grad_covs, it.grad_attrs = (r.grad_means.data_ptr(), r.grad_covs.data_ptr(),
                                                                  r.grad_attrs.data_ptr())
                    if r.with_camera:
                        r.grad_camera = torch.empty(15, **f32)
                        it.grad_camera = r.grad_camera.data_ptr()
                arr[i] = it
            backward = reqs[0].backward
            ws_bytes = nat.voge_batch_workspace_size(arr, backward)
            ws = torch.empty(ws_bytes, dtype=torch.uint8, device=self.device)
            flags = nat.VOGE_FORWARD | (nat.VOGE_BACKWARD if backward else 0)
            nat.voge_render_batch(self.ctx, arr, flags, ws.data_ptr(), ws_bytes, s.cuda_stream)
            ev = torch.cuda.Event()
            ev.record(s)
        for r in reqs:
            for t in (r.image, r.grad_means, r.grad_covs, r.grad_attrs, r.grad_camera):
                if t is not None:
                    t.record_stream(caller)
        return {"event": ev, "ws": ws, "keep": keep, "reqs": reqs, "stream": s, "n": len(reqs), "caller": caller}

    def ready(self, handle) -> bool:
        return handle["event"].query()

    def collect(self, handle) -> None:
        st = nat.voge_batch_status(handle["ws"].data_ptr(), handle["n"], handle["stream"].cuda_stream)
        for r, v in zip(handle["reqs"], st):
            r.status = int(v)
        # the caller's later work on the outputs is ordered after the batch
        handle["caller"].wait_event(handle["event"])
