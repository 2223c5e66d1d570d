"""Roofline denominators measured on the running GPU (libcmprobe.so).

HBM stream-copy bandwidth and the throughput of global and LDS floating-point
atomic adds; the CM loss kernels are reported against these and against the
published HBM peak.
"""

from __future__ import annotations

import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
PROBE_PATH = os.path.join(_PKG, "libcmprobe.so")
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(PROBE_PATH):
            raise RuntimeError(f"{PROBE_PATH} is missing: build with "
                               "`python -m paper_2412_06359_amd.build`")
        lib = ctypes.CDLL(PROBE_PATH)
        P, sz, i = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int
        lib.cmprobe_copy.argtypes = [P, P, sz, i, P]
        lib.cmprobe_global_atomic.argtypes = [P, sz, i, i, i, i, i, P]
        lib.cmprobe_lds_atomic.argtypes = [P, sz, i, i, i, i, P]
        lib.cmprobe_random_access.argtypes = [P, sz, i, i, i, i, P, P]
        for f in (lib.cmprobe_copy, lib.cmprobe_global_atomic, lib.cmprobe_lds_atomic,
                  lib.cmprobe_random_access):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _timed(launch, reps):
    s = torch.cuda.current_stream()
    launch(1)                                   # warm-up
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(s)
    launch(reps)
    b.record(s)
    torch.cuda.synchronize()
    return a.elapsed_time(b) * 1e-3 / reps      # seconds per launch


def copy_bandwidth(nbytes: int = 1 << 30, reps: int = 10) -> float:
    """GB/s of a read+write stream copy (bytes moved = 2 * nbytes)."""
    lib = _load()
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    st = torch.cuda.current_stream().cuda_stream

    def launch(r):
        rc = lib.cmprobe_copy(src.data_ptr(), dst.data_ptr(), nbytes, r, st)
        assert rc == 0, rc
    t = _timed(launch, reps)
    return 2 * nbytes / t / 1e9


def global_atomic_rate(n_elems: int, elem_bytes: int, pattern: int = 0, blocks: int = 8192,
                       ops: int = 64, reps: int = 5) -> float:
    """Atomic adds per second into an array of n_elems (pattern 0 random, 1 contiguous)."""
    lib = _load()
    dt = torch.float64 if elem_bytes == 8 else torch.float32
    arr = torch.zeros(n_elems, dtype=dt, device="cuda")
    st = torch.cuda.current_stream().cuda_stream

    def launch(r):
        rc = lib.cmprobe_global_atomic(arr.data_ptr(), n_elems, elem_bytes, blocks, ops, pattern,
                                       r, st)
        assert rc == 0, rc
    t = _timed(launch, reps)
    return blocks * 256 * ops / t


def lds_atomic_rate(lds_elems: int, elem_bytes: int, blocks: int = 8192, ops: int = 256,
                    reps: int = 5) -> float:
    """LDS atomic adds per second (random addresses in a per-workgroup array)."""
    lib = _load()
    dt = torch.float64 if elem_bytes == 8 else torch.float32
    out = torch.zeros(blocks, dtype=dt, device="cuda")
    st = torch.cuda.current_stream().cuda_stream

    def launch(r):
        rc = lib.cmprobe_lds_atomic(out.data_ptr(), lds_elems, elem_bytes, blocks, ops, r, st)
        assert rc == 0, rc
    t = _timed(launch, reps)
    return blocks * 256 * ops / t


def random_access_rate(n_elems: int, store: bool, blocks: int = 8192, ops: int = 64,
                       reps: int = 5) -> float:
    """Random 16-byte stores or loads per second into an array of n_elems."""
    lib = _load()
    arr = torch.zeros(n_elems * 2, dtype=torch.float64, device="cuda")
    sink = torch.zeros(1, dtype=torch.float64, device="cuda")
    st = torch.cuda.current_stream().cuda_stream

    def launch(r):
        rc = lib.cmprobe_random_access(arr.data_ptr(), n_elems, int(store), blocks, ops, r,
                                       sink.data_ptr(), st)
        assert rc == 0, rc
    t = _timed(launch, reps)
    return blocks * 256 * ops / t


def measure_all() -> dict:
    res = {"copy_GBps": copy_bandwidth()}
    for label, n in (("l2", 1 << 16), ("large", (256 << 20) // 16)):
        res[f"random_store16_{label}_per_s"] = random_access_rate(n, True)
        res[f"random_load16_{label}_per_s"] = random_access_rate(n, False)
    for eb in (4, 8):
        for label, n in (("l2", 1 << 18), ("large", (256 << 20) // eb)):
            for pat, pname in ((0, "random"), (1, "contig")):
                res[f"global_f{eb * 8}_{label}_{pname}_per_s"] = global_atomic_rate(n, eb, pat)
        res[f"lds_f{eb * 8}_per_s"] = lds_atomic_rate((32768 // eb), eb)
    return res


if __name__ == "__main__":
    import json
    print(json.dumps(measure_all(), indent=1))
