#!/usr/bin/env python3
"""Throughput of the contrast-maximization loss forward + backward on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c3|c2|c1|c5]

One step is one pass of the whole path (forward: warp, splat, reduce, loss;
backward: recomputed warp, adjoint, d inverse depth, d ego-motion) over the
workload, through the C ABI with buffers allocated once; inputs are resident in
HBM before the timed region.  The default workload is the batched one (64
windows of uneven size): `value` is the batched path (one launch sequence for
all windows, replayed as a hipGraph) and `plain_events_per_s` the same windows
one call each on the same GPU.  Prints one JSON line.  Inputs are seeded
synthetic windows (edge maps under rigid camera motion, see eventgen).
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "events/sec for CM loss fwd+bwd (batched vs plain); p50/p99 per-window latency"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "c1": "c1: 64x64 f=50, 2k uniform events, refs {1}, fwd+bwd",
    "c2": "c2: 640x480 f=300, 100k edge-map events (50 segments), refs {0,0.5,1}, fwd+bwd",
    "c3": "c3: 64 windows 346x260 f=200, log-uniform 5k..200k edge-map events, refs {0,1}, "
          "fwd+bwd",
    "c5": "c5: 1280x720 f=600, 2M edge-map events (400 segments), 8 refs in [0,1], fwd+bwd",
    "c6": "c6: 64 windows 346x260 f=200, 10 slices of log-uniform 1k..10k edge-map events, "
          "refs at the 11 slice edges, one depth + ego-motion per slice (10 flow sets), fwd+bwd",
}


# L_geo forward + backward per (pixel, pair): rho_a and the rho_{f+1} image
# read twice (8 + 8 bytes), d rho_a and d rho_{f+1} read-modify-written
# (8 + 8 bytes); pose partials and pair sums are negligible.
GEO_BYTES_PER_PIXEL_PAIR = 32


def kernel_source_sha() -> str:
    from paper_2412_06359_amd.build import source_sha
    return source_sha()


# Bytes of splat state per pixel and reference that the measurement plan
# counts as algorithmic: C and S of both polarities at FP32 (2 x 2 x 4 B).
# The library keeps the images in FP64 (32 B per pixel and reference, for the
# precision of the adjoint seeds); the FP64 figure is reported beside it,
# labelled, and is not the roofline fraction.
STATE_BYTES_PLAN = 16.0
STATE_BYTES_FP64 = 32.0


def algorithmic_bytes(phase: str, n: int, HW: int, R: int, tiled: bool, F: int = 1,
                      active=None, state_bytes: float = STATE_BYTES_PLAN) -> float:
    """Bytes a phase must move at minimum for one window.

    events: 13 B each (x, y, t FP32 + p int8); rho: 4 B per pixel and flow set;
    d rho 4 B per pixel and flow set; splat state: `state_bytes` per pixel and
    reference.  The direct path writes every pixel of the images; the tiled
    path stores only the pixels some tap reached, the sum over references of
    N_r (`active`, from cm_batch_active_pixels): the others are neither
    written nor read.  The backward gathers the state at those pixels only.
    The tiled path's records, bin tables and histograms are not counted:
    they are the implementation's traffic, not the method's."""
    ev = 13.0 * n
    rho = 4.0 * HW * F
    img = state_bytes * R * HW
    act = img if active is None else state_bytes * active
    if tiled:
        table = {"zero": 0.0, "count": ev + rho, "scan": 0.0, "scatter": ev + rho,
                 "splat": act, "reduce": 0.0, "finalize": 0.0,
                 "grad_count": ev + rho, "grad_scan": 0.0, "adjoint": ev + rho + act,
                 "grad_tile": 8.0 * HW * F, "grad_finalize": 0.0}
    else:
        table = {"zero": img, "splat": ev + rho + img, "reduce": img, "finalize": 0.0,
                 "grad_zero": 4.0 * HW * F, "adjoint": ev + rho + act + 4.0 * HW * F,
                 "grad_finalize": 0.0}
    return table.get(phase, 0.0)


def roofline_of(phases: dict, steps: int, wins, active, tiled: bool, workload: str):
    """The dominant phase (by total time) against the HBM roofline: its
    algorithmic bytes per launch (the measurement plan's byte model) over its
    average launch time (HIP events on the launch stream)."""
    per_launch = {k: (ms / max(c, 1), c) for k, (ms, c) in phases.items() if c > 0}
    dom = max(per_launch, key=lambda k: per_launch[k][0] * per_launch[k][1])
    dom_ms = per_launch[dom][0]
    launches_per_step = per_launch[dom][1] / steps

    def alg(sb):
        return sum(algorithmic_bytes(dom, w.n, w.width * w.height, len(w.refs), tiled,
                                     w.rho.shape[0] if w.rho.ndim == 3 else 1, a, sb)
                   for w, a in zip(wins, active)) / launches_per_step
    a16, a32 = alg(STATE_BYTES_PLAN), alg(STATE_BYTES_FP64)
    achieved = a16 / (dom_ms * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(workload, dom),
            "algorithmic_bytes_per_launch": a16, "avg_launch_ms": dom_ms,
            "byte_model": "events 13 B, rho 4 B/px, splat state 16 B per active pixel and "
                          "reference (C, S, both polarities, FP32 as the plan counts it)",
            "fp64_state": {"algorithmic_bytes_per_launch": a32,
                           "achieved": a32 / (dom_ms * 1e-3) / 1e9,
                           "frac": a32 / (dom_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                           "note": "the same kernel with the state at the 32 B per pixel and "
                                   "reference the library stores (FP64 images); not the "
                                   "roofline fraction"}}, per_launch


def launches_per_splat(per_launch: dict, steps: int) -> float:
    return per_launch["splat"][1] / steps


def splat_atomic_roofline(n_valid: int, R: int, splat_ms: float, launches_per_step: float) -> dict:
    """The tiled splat against the atomic roofline: 8 LDS FP64 adds per valid
    event and reference (4 taps x {C, S}; taps off the sensor or of zero
    weight add nothing, so this is an upper bound of the issued count) per
    launch, over the LDS FP64 atomic-add rate of random addresses in a
    workgroup's array, measured in this run by the probe kernel."""
    from paper_2412_06359_amd import probe
    peak = probe.lds_atomic_rate(32768 // 8, 8) / 1e9
    atomics = 8.0 * R * n_valid / launches_per_step
    achieved = atomics / (splat_ms * 1e-3) / 1e9
    return {"bound": "lds_atomic", "kernel": "splat", "atomics_per_launch": atomics,
            "achieved": achieved, "peak": peak, "unit": "G atomics/s", "frac": achieved / peak,
            "peak_source": "LDS FP64 atomic adds, random addresses, measured in this run"}


def active_pixels(cm, wins, dev, tuning=None):
    """Per window, the sum over references of N_r (pixels some tap reached),
    from one batched forward of the windows (at the timed run's tuning, so a
    profiled run holds no other launch shape), read back before any backward."""
    import torch
    d = to_device(wins, dev)
    b = cm.Batch([cm.WindowDesc.from_window(w) for w in wins], [w.n for w in wins],
                 tuning=tuning)
    try:
        _, st = b.forward(d["x"], d["y"], d["t"], d["p"], d["rho"], d["ego"])
        return [float(sum(nr)) for nr in b.active_pixels(st)]
    finally:
        b.close()
        torch.cuda.synchronize()


def measured_traffic(workload: str, phase: str):
    """HBM bytes per launch of a phase's kernel from the committed rocprofv3
    counter summary (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy), if it
    was taken on the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_sha") != kernel_source_sha():
        return None
    ph = rec.get("phases", {}).get(phase)
    return ph["bytes_per_launch"] if ph else None


def host_cpu() -> dict:
    """The host's logical CPU count and CPU model (from /proc/cpuinfo)."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model}


# Host cores a one-GPU job is given on the MI355X hosts this is measured on
# (their CPU share per GPU); os.cpu_count() there reports the whole machine.
HOST_CORES_PER_GPU = 16


def cpu_baseline(wins, seconds: float, threads: int) -> dict:
    """The FP64 oracle (forward + backward) over a bounded sample of the
    workload's windows, one window per thread (ctypes releases the GIL)."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor

    def one(w):
        oracle.forward(w)
        oracle.backward(w)
        return w.n

    done_events = 0
    done_windows = 0
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as pool:
        i = 0
        while time.perf_counter() - t0 < seconds:
            chunk = [wins[(i + j) % len(wins)] for j in range(threads)]
            i += threads
            done_events += sum(pool.map(one, chunk))
            done_windows += len(chunk)
    el = time.perf_counter() - t0
    out = {"value": done_events / el, "unit": "events/s", "cores": threads, "kind": "oracle",
           "sample": f"{done_windows} windows of the workload ({done_events} events), FP64 "
                     f"oracle forward+backward, {threads} threads (one window each), {el:.1f} s"}
    out.update(host_cpu())
    out["cores_note"] = (f"{threads} threads: the host cores one GPU's job gets on this machine "
                         f"(os.cpu_count() reports the whole host)")
    return out


def to_device(wins, dev):
    import numpy as np
    import torch
    f = lambda arrs: torch.from_numpy(np.ascontiguousarray(np.concatenate(
        [np.asarray(a, np.float32).ravel() for a in arrs]))).to(dev)
    return dict(x=f([w.x for w in wins]), y=f([w.y for w in wins]), t=f([w.t for w in wins]),
                p=torch.from_numpy(np.concatenate([np.asarray(w.p, np.int8) for w in wins])).to(dev),
                rho=f([w.rho for w in wins]), ego=f([w.theta for w in wins]))


def timed(fn, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def plain_step_fn(cm, wins, dev):
    """One window per call through the C ABI (the library picks its kernel path
    per window), buffers allocated once."""
    import torch
    items = []
    for w in wins:
        d = to_device([w], dev)
        desc = cm.WindowDesc.from_window(w)
        st = torch.empty(cm.state_bytes(desc, w.n), dtype=torch.uint8, device=dev)
        items.append((desc, d, st, torch.empty(1, device=dev), torch.empty_like(d["rho"]),
                      torch.empty(6, device=dev)))
    g = torch.ones(1, device=dev)

    def step():
        for desc, d, st, loss, g_rho, g_ego in items:
            cm.forward(desc, d["x"], d["y"], d["t"], d["p"], d["rho"], d["ego"], state=st,
                       loss=loss)
            cm.backward(desc, d["x"], d["y"], d["t"], d["p"], d["rho"], d["ego"], st, g,
                        grad_rho=g_rho, grad_ego=g_ego)
    return step


def _serve_run(cm, pool, rate: float, seconds: float, budget_gib: float, seed=None):
    """One Poisson stream of c4 windows into a fresh server; the client consumes
    each result as it arrives.  Returns the server's stats and the offered rate."""
    import collections
    import eventgen
    from paper_2412_06359_amd.serve import Server
    trace = (eventgen.poisson_stream(rate_hz=rate, duration_s=seconds) if seed is None else
             eventgen.poisson_stream(rate_hz=rate, duration_s=seconds, seed=seed))
    reqs = [eventgen.thin(pool[s][i % 2], n, offset=i) for i, (_, s, n) in enumerate(trace)]
    srv = Server(budget_bytes=int(budget_gib * (1 << 30)), max_batch=64, n_streams=2)
    try:
        # warm-up: one request per sensor (allocator, code objects)
        for s in pool:
            srv.submit(eventgen.thin(pool[s][0], 10000)).result(timeout=60)
        srv.drain()
        srv.reset_stats()
        pending = collections.deque()
        t0 = time.perf_counter()
        for (ta, _, _), w in zip(trace, reqs):
            dt = t0 + ta - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
            pending.append(srv.submit(w))
            while pending and pending[0].done():
                pending.popleft().result()
        while pending:
            pending.popleft().result(timeout=300)
        srv.drain()
        st = srv.stats()
    finally:
        srv.close()
    st["offered_events_per_s"] = sum(w.n for w in reqs) / seconds
    st["offered_windows_per_s"] = len(reqs) / seconds
    return st


def serve_stream(cm, seconds: float, rate: float, budget_gib: float) -> dict:
    """Workload c4: Poisson arrivals of windows (sensors 50/50 346x260 / 640x480,
    event counts log-uniform in [1k, 500k], refs {0,1}) into the continuous-
    batching server; each request is a forward + backward.  Windows are thinned
    from a pool of 2 base windows per sensor (500k events each).  Latency is
    arrival -> loss on the host and gradients ready on the device, and includes
    the host-to-device copy of the window."""
    import eventgen
    pool = eventgen.stream_pool(2, 500_000)
    st = _serve_run(cm, pool, rate, seconds, budget_gib)
    return {"workload": f"c4: Poisson {rate:.0f} windows/s for {seconds:.0f} s, 346x260/640x480 "
                        f"50/50, log-uniform 1k..500k events, refs {{0,1}}, fwd+bwd",
            "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"], "mean_ms": st["mean_ms"],
            "events_per_s": st["events_per_s"], "offered_events_per_s": st["offered_events_per_s"],
            "windows": st["windows"], "batches": st["batches"],
            "windows_per_batch": st["windows_per_batch"],
            "budget_GiB": budget_gib, "max_admitted_GiB": st["max_used_bytes"] / (1 << 30),
            "latency_includes": "H2D copy of the window, batching wait, fwd+bwd, loss D2H"}


def serve_saturation(cm, budget_gib: float, seconds: float = 3.0, start_rate: float = 500.0,
                     max_levels: int = 7) -> dict:
    """The c4 stream at rising Poisson rates (doubling from start_rate), a
    fresh server per level, until the server no longer keeps up: served
    events/s below 95 % of the offered rate.  Reports every level (p50/p99
    included: latency grows with the queue as the rate nears saturation) and
    the highest rate sustained."""
    import eventgen
    pool = eventgen.stream_pool(2, 500_000)
    levels = []
    rate = start_rate
    sustained = None
    for lvl in range(max_levels):
        st = _serve_run(cm, pool, rate, seconds, budget_gib, seed=100 + lvl)
        ok = (st["events_per_s"] is not None and
              st["events_per_s"] >= 0.95 * st["offered_events_per_s"])
        levels.append({"rate_windows_per_s": rate, "offered_events_per_s": st["offered_events_per_s"],
                       "events_per_s": st["events_per_s"], "p50_ms": st["p50_ms"],
                       "p99_ms": st["p99_ms"], "windows": st["windows"],
                       "windows_per_batch": st["windows_per_batch"], "kept_up": ok})
        print(f"# serving level {rate:.0f} windows/s: {st['events_per_s'] / 1e6:.1f} Mev/s "
              f"served of {st['offered_events_per_s'] / 1e6:.1f} offered, p99 {st['p99_ms']:.2f} ms, "
              f"{st['windows_per_batch']:.2f} windows/batch", file=sys.stderr, flush=True)
        if not ok:
            break
        sustained = levels[-1]
        rate *= 2.0
    return {"workload": "c4 windows (346x260/640x480 50/50, log-uniform 1k..500k events, refs "
                        "{0,1}, fwd+bwd), Poisson arrivals, rate doubled per level, "
                        f"{seconds:.0f} s per level",
            "criterion": "served >= 95% of offered events/s",
            "max_sustained": sustained, "levels": levels}


def single_window_line(cm, win, mode: int, steps: int, warmup: int, dev, stream,
                       workload: str, forward_only: bool = False) -> dict:
    """One window per call through the C ABI (the library picks its path),
    buffers allocated once: ms per fwd+bwd (or forward only), events/s, and the
    dominant phase against the HBM roofline."""
    import torch
    d = to_device([win], dev)
    desc = cm.WindowDesc.from_window(win, mode=mode)
    st = torch.empty(cm.state_bytes(desc, win.n), dtype=torch.uint8, device=dev)
    loss = torch.empty(1, device=dev)
    g_rho, g_ego = torch.empty_like(d["rho"]), torch.empty(d["ego"].numel(), device=dev)
    g = torch.ones(1, device=dev)

    def step():
        cm.forward(desc, d["x"], d["y"], d["t"], d["p"], d["rho"], d["ego"], state=st, loss=loss)
        if not forward_only:
            cm.backward(desc, d["x"], d["y"], d["t"], d["p"], d["rho"], d["ego"], st, g,
                        grad_rho=g_rho, grad_ego=g_ego)
    ms = timed(step, steps, warmup, stream)
    cm.profile_enable(0, True)
    cm.profile_read(0)
    for _ in range(steps):
        step()
    phases = cm.profile_read(0)
    cm.profile_enable(0, False)
    tiled = phases["count"][1] > 0
    act = active_pixels(cm, [win], dev) if tiled else [None]
    roof, per_launch = roofline_of(phases, steps, [win], act, tiled, workload)
    return {"workload": WORKLOADS.get(workload, workload) if not forward_only else
            WORKLOADS[workload].replace("fwd+bwd", "forward only"),
            "mode": "deterministic" if mode == 1 else "atomic",
            "path": "tiled" if tiled else "direct", "n_events": win.n,
            "ms_per_step": ms, "events_per_s": win.n / (ms * 1e-3), "roofline": roof,
            "phases_ms_per_launch": {k: v[0] for k, v in per_launch.items()}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the c6 (flow sets), c2, c5 and c1 lines")
    ap.add_argument("--serve-seconds", type=float, default=20.0,
                    help="length of the served Poisson stream (0: skip)")
    ap.add_argument("--serve-rate", type=float, default=500.0)
    ap.add_argument("--serve-budget-gib", type=float, default=32.0)
    ap.add_argument("--saturation-seconds", type=float, default=3.0,
                    help="seconds per level of the rising-rate serving run (0: skip)")
    ap.add_argument("--tuning", default=None,
                    help="EVENT_BLOCKS,TILE_THREADS[,TILE_W,TILE_H] for the batched workload "
                         "instead of the autotuner's choice (profiled runs pass the timed run's "
                         "tuning)")
    ap.add_argument("--path", default="auto", choices=["auto", "direct", "tiled"],
                    help="kernel path of the library handle (plain calls)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); windows are "
              f"independent and shard across GPUs with no exchange, see the design notes",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import eventgen
    import paper_2412_06359_amd as cm

    cm.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    cm.set_path(0, {"auto": cm.CM_PATH_AUTO, "direct": cm.CM_PATH_DIRECT,
                    "tiled": cm.CM_PATH_TILED}[args.path])
    batched = args.workload in ("c3", "c6")
    wins = eventgen.make_batch(args.workload, 64) if batched else \
        [eventgen.make_window(args.workload)]
    n_events = sum(w.n for w in wins)
    out_extra = {}

    plain = plain_step_fn(cm, wins, dev)
    ms_plain = timed(plain, args.steps, args.warmup, stream)
    if batched:
        from paper_2412_06359_amd import autotune
        d = to_device(wins, dev)
        descs = [cm.WindowDesc.from_window(w) for w in wins]
        if args.tuning:
            vals = [int(v) for v in args.tuning.split(",")]
            if len(vals) not in (2, 4):
                ap.error("--tuning takes EVENT_BLOCKS,TILE_THREADS[,TILE_W,TILE_H]")
            tuning = dict(event_blocks=vals[0], tile_threads=vals[1])
            if len(vals) == 4:
                tuning.update(tile_w=vals[2], tile_h=vals[3])
            out_extra["tuning"] = {"chosen": tuning, "source": "--tuning"}
        else:
            tune_log = []
            tuning = autotune.tune(descs, [w.n for w in wins], d, steps=3, warmup=1,
                                   log=tune_log)
            out_extra["tuning"] = {"chosen": tuning, "candidates": [dict(c, ms=ms)
                                                                    for c, ms in tune_log]}
        batch = cm.Batch(descs, [w.n for w in wins], graph=True, tuning=tuning)
        state = batch.new_state()
        loss = torch.empty(batch.n, device=dev)
        g_rho = torch.empty_like(d["rho"])
        g_ego = torch.empty_like(d["ego"])
        gl = torch.ones(batch.n, device=dev)

        def step():
            batch.forward(d["x"], d["y"], d["t"], d["p"], d["rho"], d["ego"], state=state,
                          loss=loss)
            batch.backward(d["x"], d["y"], d["t"], d["p"], d["rho"], d["ego"], state, gl,
                           grad_rho=g_rho, grad_ego=g_ego)
        ms_per_step = timed(step, args.steps, args.warmup, stream)
        n_valid = sum(v for _, v in batch.diagnostics(state))
        # per-kernel timing of the same launch sequence without the graph
        batch.set_graph(False)
        cm.profile_enable(0, True)
        cm.profile_read(0)
        for _ in range(args.steps):
            step()
        phases = cm.profile_read(0)
        cm.profile_enable(0, False)
        path_used = "tiled"
        # the single-window direct / tiled crossover on windows spanning the
        # workload's sizes (measured, not applied to the handle)
        by_size = sorted(wins, key=lambda w: w.n)
        sample = [by_size[i * (len(by_size) - 1) // 7] for i in range(8)]
        cross_log = []
        cross = autotune.tune_crossover(sample, steps=3, warmup=1, log=cross_log, apply=False)
        out_extra["crossover"] = {"tiled_min_records": cross, "handle_default": 1 << 17,
                                  "windows": cross_log}
        out_extra["plain_events_per_s"] = n_events / (ms_plain * 1e-3)
        out_extra["plain_ms_per_step"] = ms_plain
        out_extra["batched_over_plain"] = ms_plain / ms_per_step
    else:
        ms_per_step = ms_plain
        cm.profile_enable(0, True)
        cm.profile_read(0)
        for _ in range(args.steps):
            plain()
        phases = cm.profile_read(0)
        cm.profile_enable(0, False)
        path_used = "tiled" if phases["count"][1] > 0 else "direct"
        n_valid = None

    act = active_pixels(cm, wins, dev, tuning if batched else None)
    roof, per_launch = roofline_of(phases, args.steps, wins,
                                   act if path_used == "tiled" else [None] * len(wins),
                                   path_used == "tiled", args.workload)
    roof["active_pixel_fraction"] = sum(act) / sum(len(w.refs) * w.width * w.height for w in wins)

    if not args.no_extras and args.workload == "c3":
        # the paper's training setting: 10 slices per window, one flow per slice
        w6 = eventgen.make_batch("c6", 64)
        d6 = to_device(w6, dev)
        descs6 = [cm.WindowDesc.from_window(w) for w in w6]
        if args.tuning:
            tuning6 = tuning
        else:
            from paper_2412_06359_amd import autotune
            tuning6 = autotune.tune(descs6, [w.n for w in w6], d6, steps=2, warmup=1)
        b6 = cm.Batch(descs6, [w.n for w in w6], graph=True, tuning=tuning6)
        st6 = b6.new_state()
        l6 = torch.empty(b6.n, device=dev)
        gr6, ge6 = torch.empty_like(d6["rho"]), torch.empty_like(d6["ego"])
        gl6 = torch.ones(b6.n, device=dev)

        def step6():
            b6.forward(d6["x"], d6["y"], d6["t"], d6["p"], d6["rho"], d6["ego"], state=st6,
                       loss=l6)
            b6.backward(d6["x"], d6["y"], d6["t"], d6["p"], d6["rho"], d6["ego"], st6, gl6,
                        grad_rho=gr6, grad_ego=ge6)
        ms6 = timed(step6, args.steps, args.warmup, stream)
        n6 = sum(w.n for w in w6)
        out_extra["c6_batched"] = {"workload": WORKLOADS["c6"], "n_events": n6,
                                   "ms_per_step": ms6, "events_per_s": n6 / (ms6 * 1e-3),
                                   "tuning": tuning6}
        # the full training loss of Eq. 4: L_CM + 0.05 L_geo over consecutive slices
        gst6 = torch.empty(b6.geo_state_bytes(), dtype=torch.uint8, device=dev)

        def step6_full():
            step6()
            b6.geo_forward(d6["rho"], d6["ego"], cm.LAMBDA_GEO, l6, state=gst6)
            b6.geo_backward(d6["rho"], d6["ego"], gst6, gl6, gr6, ge6, cm.LAMBDA_GEO)

        def step6_geo():
            b6.geo_forward(d6["rho"], d6["ego"], cm.LAMBDA_GEO, l6, state=gst6)
            b6.geo_backward(d6["rho"], d6["ego"], gst6, gl6, gr6, ge6, cm.LAMBDA_GEO)
        ms6f = timed(step6_full, args.steps, args.warmup, stream)
        ms6g = timed(step6_geo, args.steps, args.warmup, stream)
        pairs = sum((w.rho.shape[0] - 1) * w.width * w.height for w in w6)
        geo_bytes = GEO_BYTES_PER_PIXEL_PAIR * pairs
        out_extra["c6_full_loss"] = {
            "workload": WORKLOADS["c6"] + " + lambda L_geo (Eq. 4, lambda 0.05) over the 9 "
                        "consecutive slice pairs",
            "ms_per_step": ms6f, "events_per_s": n6 / (ms6f * 1e-3),
            "geo_ms_per_step": ms6g, "pixel_pairs": pairs,
            "geo_algorithmic_bytes": geo_bytes,
            "geo_achieved_gbs": geo_bytes / (ms6g * 1e-3) / 1e9}
        b6.close()
        del d6, st6, gst6
        torch.cuda.empty_cache()

    if not args.no_extras and args.workload != "c2":
        w2 = eventgen.make_window("c2")
        dd = to_device([w2], dev)
        desc2 = cm.WindowDesc.from_window(w2)
        rho2 = dd["rho"].clone().requires_grad_(True)
        ego2 = dd["ego"].clone().requires_grad_(True)

        def step2():
            L = cm.cm_loss(dd["x"], dd["y"], dd["t"], dd["p"], rho2, ego2, desc2)
            L.backward()
        ms2 = timed(step2, args.steps, args.warmup, stream)
        out_extra["c2_single_window_autograd"] = {
            "workload": WORKLOADS["c2"], "ms_per_step": ms2,
            "events_per_s": w2.n / (ms2 * 1e-3)}

    if not args.no_extras and args.workload not in ("c5", "c1"):
        cm.set_path(0, cm.CM_PATH_AUTO)
        # the large window, atomic and deterministic (sort-by-pixel) modes
        w5 = eventgen.make_window("c5")
        out_extra["c5_atomic"] = single_window_line(cm, w5, cm.CM_MODE_ATOMIC, args.steps,
                                                    args.warmup, dev, stream, "c5")
        out_extra["c5_deterministic"] = single_window_line(cm, w5, cm.CM_MODE_DETERMINISTIC,
                                                           args.steps, args.warmup, dev, stream,
                                                           "c5")
        del w5
        torch.cuda.empty_cache()
        w1 = eventgen.make_window("c1")
        out_extra["c1_forward"] = single_window_line(cm, w1, cm.CM_MODE_ATOMIC, args.steps,
                                                     args.warmup, dev, stream, "c1",
                                                     forward_only=True)
        out_extra["c1_fwd_bwd"] = single_window_line(cm, w1, cm.CM_MODE_ATOMIC, args.steps,
                                                     args.warmup, dev, stream, "c1")
        cm.set_path(0, {"auto": cm.CM_PATH_AUTO, "direct": cm.CM_PATH_DIRECT,
                        "tiled": cm.CM_PATH_TILED}[args.path])

    R = len(wins[0].refs)
    out = {
        "metric": METRIC,
        "value": n_events / (ms_per_step * 1e-3),
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload],
                   "path": ("batched: 64 windows per launch sequence, hipGraph replay, tiled "
                            "kernels" if batched else f"plain (one window per call), "
                                                      f"{path_used} kernels"),
                   "windows": len(wins), "n_events": n_events, "refs": R,
                   "valid_fraction": (n_valid / n_events) if n_valid is not None else None,
                   "mode": "atomic",
                   "inputs": "FP32 events/rho/ego, FP64 warp and splat images"},
        "roofline": roof,
        "phases_ms_per_launch": {k: v[0] for k, v in per_launch.items()},
    }
    if batched and "splat" in per_launch and n_valid:
        out["atomic_roofline"] = splat_atomic_roofline(n_valid, R, per_launch["splat"][0],
                                                       launches_per_splat(per_launch, args.steps))
    out.update(out_extra)
    if args.serve_seconds > 0:
        cm.set_path(0, cm.CM_PATH_AUTO)
        out["serving"] = serve_stream(cm, args.serve_seconds, args.serve_rate,
                                      args.serve_budget_gib)
    if args.saturation_seconds > 0:
        cm.set_path(0, cm.CM_PATH_AUTO)
        out["serving_saturation"] = serve_saturation(cm, args.serve_budget_gib,
                                                     args.saturation_seconds,
                                                     start_rate=args.serve_rate)
    if not args.no_cpu_baseline:
        threads = min(os.cpu_count() or 1, HOST_CORES_PER_GPU) if batched else 1
        out["cpu_baseline"] = cpu_baseline(wins, args.cpu_seconds, threads)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
