"""Autotuner for batched launches.

A batch's launch shape in the atomic mode has three tunables (cm_tuning):
the number of event blocks the count / scatter / sweep kernels aim for
(which sets events per lane), the forward tile kernel's thread count, and
the tile size of the owner-computes splat and backward (32 x 32, 64 x 32,
32 x 16 or 16 x 16).  `tune` times candidates on a real batch -- forward +
backward, replayed from a hipGraph, between HIP events on the current stream
-- and returns the fastest: by default event blocks x tile threads at 32 x 32
tiles first, then the other tile sizes at the best pair.  Results are cached
per shape class (mode, flow model, references, flow sets, sensor size, total
events and window count, the last three rounded to powers of two) in a JSON
file, so that a serving loop or a training run tunes once per class:

    from paper_2412_06359_amd import autotune
    tuning = autotune.tune(descs, counts, inputs, cache_path="tune.json")
    batch = Batch(descs, counts, tuning=tuning)

The deterministic mode's launch shape defines its operation order, so it is
not tuned (`tune` returns the defaults).  The cache path defaults to the
environment variable CM_AUTOTUNE_CACHE (no file when unset).
"""

import json
import math
import os
from typing import Optional, Sequence

import torch

from . import binding as cm

DEFAULT = dict(event_blocks=4096, tile_threads=512, tile_w=32, tile_h=32)
# first stage: launch geometry at 32 x 32 tiles; second stage: tile sizes
CANDIDATES = [dict(event_blocks=e, tile_threads=t, tile_w=32, tile_h=32)
              for e in (1024, 2048, 4096, 8192, 16384) for t in (256, 512)]
TILE_SIZES = [(32, 32), (64, 32), (32, 16), (16, 16)]


def _tuning(d: dict) -> dict:
    """A cached or given tuning with every field (older caches lack the tile size)."""
    return dict(event_blocks=int(d["event_blocks"]), tile_threads=int(d["tile_threads"]),
                tile_w=int(d.get("tile_w", 32)), tile_h=int(d.get("tile_h", 32)))


def _pow2(v: float) -> int:
    return 1 << max(0, int(math.ceil(math.log2(max(1.0, float(v))))))


def shape_class(descs: Sequence[cm.WindowDesc], n_events: Sequence[int]) -> str:
    """Cache key of a batch."""
    d0 = descs[0]
    R = max(d.R for d in descs)
    F = max(d.F for d in descs)
    px = max(int(d.width) * int(d.height) for d in descs)
    return (f"mode{int(d0.mode)}-flow{int(d0.flow_model)}-R{R}-F{F}-px{_pow2(px)}"
            f"-ev{_pow2(sum(int(n) for n in n_events))}-nw{_pow2(len(descs))}")


def load_cache(path: Optional[str]) -> dict:
    if not path or not os.path.exists(path):
        return {}
    with open(path) as fh:
        data = json.load(fh)
    return data if isinstance(data, dict) else {}


def save_cache(path: str, data: dict):
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
        fh.write("\n")
    os.replace(tmp, path)


def time_step(batch: "cm.Batch", inputs: dict, steps: int = 5, warmup: int = 2) -> float:
    """ms per forward + backward of `batch` on `inputs` (dict x, y, t, p, rho,
    ego device tensors), HIP events on the current stream."""
    dev = inputs["rho"].device
    state = batch.new_state()
    loss = torch.empty(batch.n, device=dev)
    g_rho = torch.empty_like(inputs["rho"])
    g_ego = torch.empty_like(inputs["ego"])
    gl = torch.ones(batch.n, device=dev)
    a = (inputs["x"], inputs["y"], inputs["t"], inputs["p"], inputs["rho"], inputs["ego"])

    def step():
        batch.forward(*a, state=state, loss=loss)
        batch.backward(*a, state, gl, grad_rho=g_rho, grad_ego=g_ego)

    for _ in range(warmup):
        step()
    stream = torch.cuda.current_stream(dev)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        step()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / steps


def tune(descs: Sequence[cm.WindowDesc], n_events: Sequence[int], inputs: Optional[dict] = None,
         candidates=None, steps: int = 5, warmup: int = 2, cache_path: Optional[str] = None,
         device: int = 0, log: Optional[list] = None) -> dict:
    """The fastest candidate tuning for this batch's shape class (cached).

    inputs: the batch's packed device tensors (x, y, t, p, rho, ego); without
    them only the cache is consulted (defaults on a miss).  log, if given,
    receives (tuning, ms) for every candidate timed."""
    if int(descs[0].mode) == cm.CM_MODE_DETERMINISTIC:
        return dict(DEFAULT)
    path = cache_path if cache_path is not None else os.environ.get("CM_AUTOTUNE_CACHE")
    key = shape_class(descs, n_events)
    cache = load_cache(path)
    if key in cache:
        return _tuning(cache[key])
    if inputs is None:
        return dict(DEFAULT)
    best, best_ms = None, float("inf")

    def run(cands):
        nonlocal best, best_ms
        for cand in cands:
            b = cm.Batch(descs, n_events, device=device, graph=True, tuning=cand)
            try:
                ms = time_step(b, inputs, steps, warmup)
            finally:
                b.close()
            if log is not None:
                log.append((dict(cand), ms))
            if ms < best_ms:
                best, best_ms = _tuning(cand), ms
    if candidates is not None:
        run(candidates)
    else:
        run(CANDIDATES)
        run([dict(best, tile_w=w, tile_h=h) for w, h in TILE_SIZES
             if (w, h) != (best["tile_w"], best["tile_h"])])
    if path:
        cache = load_cache(path)
        cache[key] = dict(best, ms=best_ms)
        save_cache(path, cache)
    return best


def _time_window(desc, win, path: int, device: int, steps: int, warmup: int) -> float:
    """ms per forward + backward of one window through the single-window calls
    on the given path, HIP events on the current stream."""
    dev = torch.device("cuda", device)
    f32 = lambda a: torch.as_tensor(a, dtype=torch.float32).reshape(-1).contiguous().to(dev)
    x, y, t = f32(win.x), f32(win.y), f32(win.t)
    p = torch.as_tensor(win.p, dtype=torch.int8).to(dev)
    rho, ego = f32(win.rho), f32(win.theta)
    prev = cm.get_path(device)
    cm.set_path(device, path)
    try:
        st = torch.empty(cm.state_bytes(desc, win.n), dtype=torch.uint8, device=dev)
        loss = torch.empty(1, device=dev)
        g_rho, g_ego = torch.empty_like(rho), torch.empty_like(ego)
        g = torch.ones(1, device=dev)

        def step():
            cm.forward(desc, x, y, t, p, rho, ego, state=st, loss=loss)
            cm.backward(desc, x, y, t, p, rho, ego, st, g, grad_rho=g_rho, grad_ego=g_ego)
        for _ in range(warmup):
            step()
        stream = torch.cuda.current_stream(dev)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            step()
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / steps
    finally:
        cm.set_path(device, prev)


def tune_crossover(windows, device: int = 0, steps: int = 5, warmup: int = 2,
                   log: Optional[list] = None, apply: bool = True) -> int:
    """The single-window direct / tiled crossover (cm_tuning.tiled_min_records):
    times each window (ascending event-reference records) on both paths and
    returns the record count from which the tiled path is faster -- the
    geometric mean of the largest window the direct path wins and the smallest
    the tiled path wins from there on (the first or last window's count when
    one path wins everywhere).  apply: set it on the device's handle."""
    rows = []
    for win in sorted(windows, key=lambda w: w.n * len(w.refs)):
        desc = cm.WindowDesc.from_window(win)
        recs = int(win.n) * len(win.refs)
        md = _time_window(desc, win, cm.CM_PATH_DIRECT, device, steps, warmup)
        mt = _time_window(desc, win, cm.CM_PATH_TILED, device, steps, warmup)
        rows.append((recs, md, mt))
        if log is not None:
            log.append(dict(records=recs, direct_ms=md, tiled_ms=mt))
    # the smallest index from which the tiled path wins every larger window
    k = len(rows)
    while k > 0 and rows[k - 1][2] < rows[k - 1][1]:
        k -= 1
    if k == len(rows):
        cross = rows[-1][0] + 1                 # the direct path wins everywhere measured
    elif k == 0:
        cross = rows[0][0]
    else:
        cross = int(round(math.sqrt(rows[k - 1][0] * rows[k][0])))
    cross = max(1, cross)
    if apply:
        cur = cm.get_tuning(device)
        cur["tiled_min_records"] = cross
        cm.set_tuning(device, **cur)
    return cross
