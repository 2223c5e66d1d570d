"""Serving loop: continuous batching of CM loss + gradient requests.

Windows arrive one by one (as in on-device online learning, where every
freshly accumulated window is a training sample).  A scheduler thread keeps up
to `n_streams` batches in flight: whenever a stream is free it admits the
queued windows in arrival order while their device memory fits the budget,
packs them into one batched forward + backward (cm_loss_forward_batched /
cm_loss_backward_batched) on that stream, and retires finished batches by
polling their completion events.  Requests that arrive while others run are
admitted as soon as a stream and memory free up, so batches overlap on the
device.  Each request's Future resolves to its loss (on the host) and its
gradients (on the device).

Memory.  The budget bounds the device memory allocated through torch's
allocator on the server's device since the server started (torch's
memory_allocated above its value at start): the stream slots' workspaces
(inputs, batch state, loss), the gradient buffers of batches in flight and the
gradients of delivered results the client still holds.  A batch is admitted
only if that figure plus what the batch will allocate stays within the budget
(a slot workspace too small for the batch is freed first and reallocated at
the batch's exact size).  If the head of the queue cannot fit while nothing is
in flight (held results and workspaces fill the budget), it fails with
CM_ERR_BUDGET instead of waiting forever; a window larger than the whole
budget is refused on submission.

Streams.  Delivered gradients are complete when the Future resolves.  They
were written on a server stream; the server records their use on the stream
that was current in the submitting thread, so the caching allocator does not
hand their memory to a later batch while work the client queued on that
stream may still read them.  A client that reads them on another stream must
call record_stream for it.

Shutdown and failures.  close() lets the scheduler finish every submitted
request (queued and in flight) before it stops.  If the scheduler itself fails,
every request it has not resolved (queued or in flight) fails with the same
exception, and later submissions raise.
"""

from __future__ import annotations

import collections
import threading
import time
from concurrent.futures import Future, ThreadPoolExecutor
from typing import List

import numpy as np
import torch

from . import binding
from .binding import CMError, WindowDesc

CM_ERR_BUDGET = -5


def _align(n: int) -> int:
    return (n + 255) // 256 * 256


def window_footprint(desc: WindowDesc, n_events: int) -> int:
    """Device bytes a batch of this window alone allocates: its workspace
    (events 13 N, inverse depth 4 F H W, ego, the single-window state, loss
    and grad_loss, each 256-byte aligned) and its gradients (4 F H W + 24 F).
    A batch of several windows needs about the sum of theirs."""
    hw = desc.width * desc.height
    F = desc.F
    ws = (3 * _align(4 * n_events) + _align(n_events) + _align(4 * F * hw) + _align(24 * F)
          + _align(binding.state_bytes(desc, n_events)) + 2 * 256)
    return ws + _align(4 * F * hw) + _align(24 * F)


class Request:
    __slots__ = ("window", "desc", "n", "footprint", "future", "t_arrival", "stream")

    def __init__(self, window, desc, footprint, stream):
        self.window = window
        self.desc = desc
        self.n = int(window.n)
        self.footprint = footprint
        self.future = Future()
        self.t_arrival = time.perf_counter()
        self.stream = stream        # the client's current stream at submission


class _Staging:
    """A stream slot's pinned host buffer (reused from batch to batch, grown
    when a batch needs more: allocating pinned memory per batch costs
    milliseconds) and its device workspace (inputs, state, loss, grad_loss of
    its batch; sized exactly, reallocated when a batch needs more).  A slot is
    refilled only after its previous batch has retired."""

    def __init__(self):
        self.buf = None
        self.loss = None
        self.dev = None

    def device_bytes(self) -> int:
        return 0 if self.dev is None else self.dev.numel()

    def release_device(self):
        self.dev = None

    def device_buffer(self, nbytes, device):
        if self.dev is None or self.dev.numel() < nbytes:
            self.dev = None                     # freed before the larger one is allocated
            self.dev = torch.empty(nbytes, dtype=torch.uint8, device=device)
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
    def __init__(self, reqs, batch, stream, event, keep, loss_host):
        self.reqs = reqs
        self.batch = batch
        self.stream = stream
        self.event = event
        self.keep = keep
        self.loss_host = loss_host


def _workspace_sizes(batch, tv) -> List[int]:
    return [v.numel() * v.element_size() for v in tv.values()] + \
        [batch.state_bytes, 4 * batch.n, 4 * batch.n]


def _batch_need(batch) -> tuple:
    """(workspace bytes, gradient bytes) a batch allocates on the device."""
    n = batch.event_offsets[-1]
    ins = [4 * n, 4 * n, 4 * n, n, 4 * batch.pixel_offsets[-1], 24 * batch.set_offsets[-1]]
    ws = sum(_align(b) for b in ins + [batch.state_bytes, 4 * batch.n, 4 * batch.n])
    grads = _align(4 * batch.pixel_offsets[-1]) + _align(24 * batch.set_offsets[-1])
    return ws, grads


class Server:
    """Continuous-batching server for CM loss + gradient requests on one GPU."""

    def __init__(self, budget_bytes: int, max_batch: int = 64, n_streams: int = 2,
                 device: int = 0, mode: int = binding.CM_MODE_ATOMIC, poll_s: float = 50e-6,
                 copy_threads: int = 6, parallel_copy_bytes: int = 8 << 20):
        self.budget = int(budget_bytes)
        # host threads for the staging copies of large batches
        self.parallel_copy_bytes = parallel_copy_bytes
        self._copier = ThreadPoolExecutor(max_workers=max(1, copy_threads),
                                          thread_name_prefix="cm-copy")
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
        self._closing = False
        self._failed = None
        self.latencies: List[float] = []
        self.events_done = 0
        self.windows_done = 0
        self.batches = 0
        self.max_used = 0
        self.t_first = None
        self.t_last = None
        torch.cuda.synchronize(device)
        self._base = torch.cuda.memory_stats_as_nested_dict(device)["allocated_bytes"]["all"][
            "current"]
        torch.cuda.reset_peak_memory_stats(device)
        self._thread = threading.Thread(target=self._loop, name="cm-server", daemon=True)
        self._thread.start()

    # -- client side ------------------------------------------------------
    def used_bytes(self) -> int:
        """Device memory allocated on the server's device since the server
        started (what the budget bounds).  Read from the allocator's nested
        statistics: torch.cuda.memory_allocated() flattens the whole
        statistics dictionary on every call, which cost the scheduler a
        quarter of its time."""
        st = torch.cuda.memory_stats_as_nested_dict(self.device)
        return st["allocated_bytes"]["all"]["current"] - self._base

    def submit(self, window) -> Future:
        if self._failed is not None:
            raise RuntimeError("the server's scheduler failed") from self._failed
        if self._closing:
            raise RuntimeError("the server is closed")
        desc = WindowDesc.from_window(window, mode=self.mode)
        fp = window_footprint(desc, window.n)
        req = Request(window, desc, fp, torch.cuda.current_stream(self.device))
        if fp > self.budget:
            req.future.set_exception(CMError(CM_ERR_BUDGET, "window footprint exceeds the budget"))
            return req.future
        with self._lock:
            self._queue.append(req)
        self._wake.set()
        return req.future

    def close(self, timeout: float = 120.0):
        """Finish every submitted request, then stop the scheduler."""
        self._closing = True
        self._wake.set()
        self._thread.join(timeout)
        if self._thread.is_alive():
            raise TimeoutError("server did not finish its requests")
        self._copier.shutdown(wait=True)

    def drain(self, timeout: float = 60.0):
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < timeout:
            if self._failed is not None:
                raise RuntimeError("the server's scheduler failed") from self._failed
            with self._lock:
                idle = not self._queue and all(b is None for b in self._busy)
            if idle:
                return
            time.sleep(1e-3)
        raise TimeoutError("server did not drain")

    def reset_stats(self):
        """Clears the latency and throughput counters (call while idle, e.g.
        after drain(), to leave a warm-up out of the figures)."""
        with self._lock:
            self.latencies.clear()
            self.events_done = self.windows_done = self.batches = 0
            self.t_first = self.t_last = None

    def stats(self) -> dict:
        lat = np.array(self.latencies) * 1e3
        span = (self.t_last - self.t_first) if self.t_first is not None else 0.0
        return {
            "windows": self.windows_done,
            "events": self.events_done,
            "batches": self.batches,
            "windows_per_batch": self.windows_done / self.batches if self.batches else None,
            "p50_ms": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_ms": float(np.percentile(lat, 99)) if lat.size else None,
            "mean_ms": float(lat.mean()) if lat.size else None,
            "events_per_s": self.events_done / span if span > 0 else None,
            "max_used_bytes": self.max_used,
            "peak_allocated_bytes": torch.cuda.max_memory_allocated(self.device) - self._base,
            "budget_bytes": self.budget,
        }

    # -- scheduler ----------------------------------------------------------
    def _loop(self):
        torch.cuda.set_device(self.device)
        try:
            while True:
                progressed = self._retire()
                progressed |= self._admit()
                if self._closing:
                    with self._lock:
                        idle = not self._queue and all(b is None for b in self._busy)
                    if idle:
                        return
                if not progressed:
                    self._wake.wait(self.poll_s)
                    self._wake.clear()
        except BaseException as exc:       # fail every unresolved request loudly
            self._failed = exc
            with self._lock:
                pending = list(self._queue)
                self._queue.clear()
            for fl in self._busy:
                if fl is not None:
                    pending.extend(fl.reqs)
            for r in pending:
                if not r.future.done():
                    r.future.set_exception(exc)
            # every client sees the failure (its future, submit(), drain());
            # only an interpreter exit propagates further
            if not isinstance(exc, Exception):
                raise

    def _note_usage(self):
        self.max_used = max(self.max_used, self.used_bytes())

    def _retire(self) -> bool:
        done_any = False
        for i, fl in enumerate(self._busy):
            if fl is None or not fl.event.query():
                continue
            t = time.perf_counter()
            loss = fl.loss_host.numpy()
            g_rho, g_ego = fl.keep["g_rho"], fl.keep["g_ego"]
            # the client's streams may read the gradients from now on
            for s in {r.stream for r in fl.reqs}:
                g_rho.record_stream(s)
                g_ego.record_stream(s)
            offs, sets = fl.batch.pixel_offsets, fl.batch.set_offsets
            self._busy[i] = None
            fl.batch.close()
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
            done_any = True
        return done_any

    def _reclaimable(self, slot) -> int:
        """Bytes of idle slot workspaces (slots with no batch in flight,
        `slot` included) that can be freed."""
        return sum(st.device_bytes() for j, st in enumerate(self._staging)
                   if j == slot or self._busy[j] is None)

    def _fits(self, slot, ws, grads) -> bool:
        """Whether a batch needing `ws` workspace and `grads` gradient bytes
        fits on `slot`.  Frees idle workspaces when that makes the difference:
        first the other free slots', then the slot's own (a workspace larger
        than this batch needs, kept from an earlier batch; it is then
        reallocated at the exact size)."""
        own = self._staging[slot]
        extra = max(0, ws - own.device_bytes())
        if self.used_bytes() + extra + grads <= self.budget:
            return True
        for j, st in enumerate(self._staging):
            if j != slot and self._busy[j] is None and st.device_bytes():
                st.release_device()
        if self.used_bytes() + extra + grads <= self.budget:
            return True
        own.release_device()
        return self.used_bytes() + ws + grads <= self.budget

    def _plan(self, slot):
        """Requests of the next batch for `slot` (removed from the queue) and
        their plan, or (None, None).  Greedy in arrival order by footprint
        estimate, then checked against the plan's exact sizes."""
        with self._lock:
            avail = self.budget - self.used_bytes() + self._reclaimable(slot)
            reqs, fp = [], 0
            for r in self._queue:
                if len(reqs) >= self.max_batch or fp + r.footprint > avail:
                    break
                reqs.append(r)
                fp += r.footprint
        while reqs:
            batch = binding.Batch([r.desc for r in reqs], [r.n for r in reqs],
                                  device=self.device)
            if self._fits(slot, *_batch_need(batch)):
                with self._lock:
                    for _ in reqs:
                        self._queue.popleft()
                return reqs, batch
            batch.close()
            reqs.pop()
        if all(b is None for b in self._busy):
            # Nothing in flight will free memory: the budget is held by
            # results the client keeps.  Fail the head instead of waiting.
            with self._lock:
                head = self._queue.popleft() if self._queue else None
            if head is not None:
                head.future.set_exception(CMError(
                    CM_ERR_BUDGET, "device memory budget exhausted (results held by the client)"))
        return None, None

    def _admit(self) -> bool:
        try:
            slot = self._busy.index(None)
        except ValueError:
            return False
        if not self._queue:
            return False
        reqs, batch = self._plan(slot)
        if not reqs:
            return False
        if self.t_first is None:
            self.t_first = min(r.t_arrival for r in reqs)
        try:
            self._busy[slot] = self._launch(reqs, batch, self._streams[slot],
                                            self._staging[slot])
        except Exception as exc:       # these requests fail; the server keeps serving
            batch.close()
            for r in reqs:
                r.future.set_exception(exc)
            return True
        self._note_usage()
        self.batches += 1
        return True

    def _launch(self, reqs, batch, stream, staging) -> _InFlight:
        wins = [r.window for r in reqs]
        dev = torch.device("cuda", self.device)
        n = batch.event_offsets[-1]
        spec = [("x", np.float32, n), ("y", np.float32, n), ("t", np.float32, n),
                ("p", np.int8, n), ("rho", np.float32, batch.pixel_offsets[-1]),
                ("ego", np.float32, 6 * batch.set_offsets[-1])]
        host, tv = staging.arrays(spec)
        # every window's fields into the pinned buffer (strided event arrays go
        # in as they are, cast to the buffer's dtype); large batches split the
        # copies over a few host threads (numpy releases the GIL in them)
        # (a job: one field of a run of consecutive windows, one concatenation)
        jobs = []
        split = 4 if len(wins) >= 8 else 1
        for name, field in (("x", "x"), ("y", "y"), ("t", "t"), ("p", "p"), ("rho", "rho"),
                            ("ego", "theta")):
            parts = [np.asarray(getattr(w, field)) for w in wins]
            parts = [a if a.ndim == 1 else a.reshape(-1) for a in parts]
            k = split if name in ("rho", "x", "y", "t") else 1
            bounds = [len(parts) * i // k for i in range(k + 1)]
            o = 0
            for i in range(k):
                chunk = parts[bounds[i]:bounds[i + 1]]
                sz = sum(a.size for a in chunk)
                if sz:
                    jobs.append((host[name][o:o + sz], chunk))
                o += sz
        total = sum(sum(a.nbytes for a in c) for _, c in jobs)

        def run(job):
            dst, chunk = job
            np.concatenate(chunk, out=dst, casting="same_kind")
        if total >= self.parallel_copy_bytes and len(jobs) > 1:
            list(self._copier.map(run, jobs))
        else:
            for job in jobs:
                run(job)
        with torch.cuda.stream(stream):
            # one device workspace per slot: inputs, state, loss, grad_loss
            sizes = _workspace_sizes(batch, tv)
            offs, total = [], 0
            for nb in sizes:
                offs.append(total)
                total += _align(nb)
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
        return _InFlight(reqs, batch, stream, ev, keep, loss_host)
