"""Serving loop: continuous batching of CM loss + gradient requests.

Windows arrive one by one (as in on-device online learning, where every
freshly accumulated window is a training sample).  A scheduler thread keeps up
to `n_streams` batches in flight: whenever a stream is free it admits the
queued windows in arrival order while their HBM footprint fits the budget,
packs them into one batched forward + backward (cm_loss_forward_batched /
cm_loss_backward_batched) on that stream, and retires finished batches by
polling their completion events.  Requests that arrive while others run are
admitted as soon as a stream and memory free up, so batches overlap on the
device.  Each request's Future resolves to its loss (on the host) and its
gradients (on the device).

Footprint of a window (bytes): its share of the batch state (splat images
32 R H W, header, tiled workspace: the single-window state size), the events
(13 N), inverse depth and its gradient (8 F H W for F flow sets) and the small
per-window vectors; the admitted batches' footprints never sum above the
budget.  A
window larger than the whole budget is refused with CM_ERR_BUDGET.
"""

from __future__ import annotations

import collections
import threading
import time
from concurrent.futures import Future
from typing import List, Optional

import numpy as np
import torch

from . import binding
from .binding import CMError, WindowDesc

CM_ERR_BUDGET = -5


class Request:
    __slots__ = ("window", "desc", "n", "footprint", "future", "t_arrival")

    def __init__(self, window, desc, footprint):
        self.window = window
        self.desc = desc
        self.n = int(window.n)
        self.footprint = footprint
        self.future = Future()
        self.t_arrival = time.perf_counter()


def window_footprint(desc: WindowDesc, n_events: int) -> int:
    hw = desc.width * desc.height
    return binding.state_bytes(desc, n_events) + 13 * n_events + 8 * hw * desc.F + 48 * desc.F + 16


class _Staging:
    """A stream slot's pinned host buffer, reused from batch to batch and grown
    when a batch needs more (allocating pinned memory per batch costs
    milliseconds, which showed up in the tail latency).  A slot's buffer is
    refilled only after its previous batch has retired, so its copies are
    complete."""

    def __init__(self):
        self.buf = None
        self.loss = None
        self.dev = None

    def device_buffer(self, nbytes, device):
        """The slot's device workspace (inputs and state of its batch: the
        caller gets only the gradients, which are allocated per batch)."""
        if self.dev is None or self.dev.numel() < nbytes:
            cap = max(nbytes, 2 * (self.dev.numel() if self.dev is not None else 0))
            self.dev = torch.empty(cap, dtype=torch.uint8, device=device)
        return self.dev

    def arrays(self, spec):
        """spec: [(name, numpy dtype, count)] -> {name: numpy view} in one
        pinned buffer (16-byte aligned pieces) and {name: torch view}."""
        offs, total = [], 0
        for _, dt, cnt in spec:
            offs.append(total)
            total += (np.dtype(dt).itemsize * cnt + 15) // 16 * 16
        if self.buf is None or self.buf.numel() < total:
            cap = max(total, 2 * (self.buf.numel() if self.buf is not None else 0))
            self.buf = torch.empty(cap, dtype=torch.uint8, pin_memory=True)
        raw = self.buf.numpy()
        np_views, t_views = {}, {}
        for (name, dt, cnt), o in zip(spec, offs):
            nb = np.dtype(dt).itemsize * cnt
            np_views[name] = raw[o:o + nb].view(dt)
            t_views[name] = self.buf[o:o + nb].view(torch.int8 if dt == np.int8 else torch.float32)
        return np_views, t_views

    def loss_buffer(self, n):
        if self.loss is None or self.loss.numel() < n:
            self.loss = torch.empty(max(n, 64), dtype=torch.float32, pin_memory=True)
        return self.loss[:n]


class _InFlight:
    def __init__(self, reqs, batch, stream, event, keep, loss_host, footprint):
        self.reqs = reqs
        self.batch = batch
        self.stream = stream
        self.event = event
        self.keep = keep
        self.loss_host = loss_host
        self.footprint = footprint


class Server:
    """Continuous-batching server for CM loss + gradient requests on one GPU."""

    def __init__(self, budget_bytes: int, max_batch: int = 64, n_streams: int = 2,
                 device: int = 0, mode: int = binding.CM_MODE_ATOMIC, poll_s: float = 50e-6):
        self.budget = int(budget_bytes)
        self.max_batch = max_batch
        self.device = device
        self.mode = mode
        self.poll_s = poll_s
        self._queue = collections.deque()
        self._lock = threading.Lock()
        self._wake = threading.Event()
        self._streams = [torch.cuda.Stream(device=device) for _ in range(n_streams)]
        self._staging = [_Staging() for _ in range(n_streams)]
        self._busy = [None] * n_streams
        self._used = 0
        self._running = True
        self.latencies: List[float] = []
        self.events_done = 0
        self.windows_done = 0
        self.batches = 0
        self.max_used = 0
        self.t_first = None
        self.t_last = None
        self._thread = threading.Thread(target=self._loop, name="cm-server", daemon=True)
        self._thread.start()

    # -- client side ------------------------------------------------------
    def submit(self, window) -> Future:
        desc = WindowDesc.from_window(window, mode=self.mode)
        fp = window_footprint(desc, window.n)
        req = Request(window, desc, fp)
        if fp > self.budget:
            req.future.set_exception(CMError(CM_ERR_BUDGET, "window footprint exceeds the budget"))
            return req.future
        with self._lock:
            self._queue.append(req)
        self._wake.set()
        return req.future

    def close(self):
        self._running = False
        self._wake.set()
        self._thread.join()

    def drain(self, timeout: float = 60.0):
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < timeout:
            with self._lock:
                idle = not self._queue and all(b is None for b in self._busy)
            if idle:
                return
            time.sleep(1e-3)
        raise TimeoutError("server did not drain")

    def stats(self) -> dict:
        lat = np.array(self.latencies) * 1e3
        span = (self.t_last - self.t_first) if self.t_first is not None else 0.0
        return {
            "windows": self.windows_done,
            "events": self.events_done,
            "batches": self.batches,
            "p50_ms": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_ms": float(np.percentile(lat, 99)) if lat.size else None,
            "mean_ms": float(lat.mean()) if lat.size else None,
            "events_per_s": self.events_done / span if span > 0 else None,
            "max_used_bytes": self.max_used,
            "budget_bytes": self.budget,
        }

    # -- scheduler ----------------------------------------------------------
    def _loop(self):
        torch.cuda.set_device(self.device)
        try:
            while self._running:
                progressed = self._retire()
                progressed |= self._admit()
                if not progressed:
                    self._wake.wait(self.poll_s)
                    self._wake.clear()
        except Exception as exc:       # fail every pending request loudly
            with self._lock:
                pending = list(self._queue)
                self._queue.clear()
            for r in pending:
                if not r.future.done():
                    r.future.set_exception(exc)
            raise

    def _retire(self) -> bool:
        done_any = False
        for i, fl in enumerate(self._busy):
            if fl is None or not fl.event.query():
                continue
            t = time.perf_counter()
            loss = fl.loss_host.numpy()
            g_rho, g_ego = fl.keep["g_rho"], fl.keep["g_ego"]
            offs, sets = fl.batch.pixel_offsets, fl.batch.set_offsets
            for w, r in enumerate(fl.reqs):
                lead = (r.desc.F,) if r.desc.F > 1 else ()
                res = {"loss": float(loss[w]),
                       "grad_inv_depth": g_rho[offs[w]:offs[w + 1]].view(
                           *lead, r.desc.height, r.desc.width),
                       "grad_ego": g_ego[6 * sets[w]:6 * sets[w + 1]].view(*lead, 6),
                       "latency_s": t - r.t_arrival}
                self.latencies.append(t - r.t_arrival)
                self.events_done += r.n
                self.windows_done += 1
                r.future.set_result(res)
            self.t_last = t
            with self._lock:
                self._used -= fl.footprint
            fl.batch.close()
            self._busy[i] = None
            done_any = True
        return done_any

    def _admit(self) -> bool:
        try:
            slot = self._busy.index(None)
        except ValueError:
            return False
        with self._lock:
            reqs = []
            fp = 0
            while self._queue and len(reqs) < self.max_batch:
                r = self._queue[0]
                if self._used + fp + r.footprint > self.budget:
                    break
                reqs.append(self._queue.popleft())
                fp += r.footprint
            self._used += fp
            self.max_used = max(self.max_used, self._used)
        if not reqs:
            return False
        if self.t_first is None:
            self.t_first = min(r.t_arrival for r in reqs)
        try:
            self._busy[slot] = self._launch(reqs, self._streams[slot], self._staging[slot], fp)
        except Exception as exc:       # these requests fail; the server keeps serving
            with self._lock:
                self._used -= fp
            for r in reqs:
                r.future.set_exception(exc)
            return True
        self.batches += 1
        return True

    def _launch(self, reqs, stream, staging, fp) -> _InFlight:
        wins = [r.window for r in reqs]
        batch = binding.Batch([r.desc for r in reqs], [r.n for r in reqs], device=self.device)
        dev = torch.device("cuda", self.device)
        n = batch.event_offsets[-1]
        spec = [("x", np.float32, n), ("y", np.float32, n), ("t", np.float32, n),
                ("p", np.int8, n), ("rho", np.float32, batch.pixel_offsets[-1]),
                ("ego", np.float32, 6 * batch.set_offsets[-1])]
        host, tv = staging.arrays(spec)
        for name, field in (("x", "x"), ("y", "y"), ("t", "t"), ("p", "p"), ("rho", "rho"),
                            ("ego", "theta")):
            dt = host[name].dtype
            np.concatenate([np.asarray(getattr(w, field), dtype=dt).ravel() for w in wins],
                           out=host[name])
        with torch.cuda.stream(stream):
            # one device workspace per slot: inputs, state, loss, grad_loss
            sizes = [v.numel() * v.element_size() for v in tv.values()] + \
                [batch.state_bytes, 4 * batch.n, 4 * batch.n]
            offs, total = [], 0
            for nb in sizes:
                offs.append(total)
                total += (nb + 255) // 256 * 256
            dbuf = staging.device_buffer(total, dev)
            d = {}
            for (k, v), o, nb in zip(tv.items(), offs, sizes):
                d[k] = dbuf[o:o + nb].view(v.dtype)
                d[k].copy_(v, non_blocking=True)
            state = dbuf[offs[6]:offs[6] + batch.state_bytes]
            loss = dbuf[offs[7]:offs[7] + 4 * batch.n].view(torch.float32)
            gl = dbuf[offs[8]:offs[8] + 4 * batch.n].view(torch.float32)
            gl.fill_(1.0)
            batch.forward(d["x"], d["y"], d["t"], d["p"], d["rho"], d["ego"], state=state,
                          loss=loss)
            g_rho, g_ego = batch.backward(d["x"], d["y"], d["t"], d["p"], d["rho"], d["ego"],
                                          state, gl)
            loss_host = staging.loss_buffer(batch.n)
            loss_host.copy_(loss, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(stream)
        keep = dict(d=d, state=state, loss=loss, gl=gl, g_rho=g_rho, g_ego=g_ego)
        return _InFlight(reqs, batch, stream, ev, keep, loss_host, fp)
