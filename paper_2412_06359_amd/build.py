"""Compile the HIP library (libcmloss.so) for gfx950, in place.

    python -m paper_2412_06359_amd.build
"""

from __future__ import annotations

import os
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libcmloss.so")
PROBE_LIB = os.path.join(PKG, "libcmprobe.so")

SOURCES = ["cm_api.hip", "cm_kernels.hip", "cm_batch.hip", "cm_geo.hip"]
PROBE_SOURCES = ["cm_probe.hip"]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
    # every FP operation is the one written (explicit fma where intended)
    "-ffp-contract=off",
    # no packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]



def source_sha() -> str:
    """Short hash of the kernel sources (csrc/); counter summaries record it so
    that figures taken on older kernels are not reported against newer ones."""
    import hashlib
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(name.encode() + f.read())
    return h.hexdigest()[:16]

def _hipcc(sources, out, verbose):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = out + ".tmp"
    cmd = [hipcc] + HIPCC_FLAGS + ["-I", os.path.join(ROOT, "include")] + \
        [os.path.join(CSRC, s) for s in sources] + ["-o", tmp]
    t0 = time.time()
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed building {os.path.basename(out)}")
    os.replace(tmp, out)
    if verbose:
        print(f"built {out} in {time.time() - t0:.1f}s")


def build(verbose: bool = False) -> str:
    """Compile libcmloss.so (the loss) and libcmprobe.so (roofline microbenchmarks)."""
    _hipcc(SOURCES, LIB, verbose)
    _hipcc(PROBE_SOURCES, PROBE_LIB, verbose)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
