"""rocprofv3 output -> short text summaries (kernel times, HBM traffic).

    python -m paper_2412_06359_amd.profsum copy --mib 512
        one plain copy kernel of a known size (run it under `rocprofv3 --pmc`
        to calibrate FETCH_SIZE / WRITE_SIZE against bytes that are known);
    python -m paper_2412_06359_amd.profsum trace DIR --title T --cmd C
        markdown table of a `--kernel-trace` run (kernel_trace.csv), grouped by
        kernel and grid size;
    python -m paper_2412_06359_amd.profsum traffic --kernel NAME:PHASE [...]
        --workload W --fetch DIR --write DIR --copy-fetch DIR --copy-write DIR
        --copy-mib M --cmd C [--cmd C ...] --out FILE.json
        HBM bytes per dispatch of the largest-grid launches of each kernel,
        each counter scaled by what it reads for the copy kernel; writes the
        JSON record and a markdown table beside it (FILE.md);
    python -m paper_2412_06359_amd.profsum counters DIR [DIR ...] --kernel NAME:PHASE
        [...] --title T --cmd C [--cmd C ...] --out FILE.md
        mean per dispatch of every counter the runs collected, for the
        largest-grid launches of each kernel, with the wave-state ratios
        (waiting / wave cycles, busy / wave cycles) where the counters exist.

The profiled runs pass the timed run's launch tuning explicitly, so the
largest-grid launch of a kernel is the batched launch that was timed.

The traffic summary records the hash of the kernel sources it was taken on;
the benchmark reports it only while the sources are unchanged.
"""

from __future__ import annotations

import argparse
import collections
import csv
import glob
import json
import os
import statistics
import sys

from .build import source_sha


def _csv(d: str, suffix: str):
    files = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not files:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    rows = []
    for f in files:
        with open(f, newline="") as fh:
            rows.extend(csv.DictReader(fh))
    return rows


def _short(name: str) -> str:
    name = name.split("(")[0]
    return name.replace("void ", "").strip()


def _grid(row) -> int:
    for k in ("Grid_Size", "Grid_Size_X"):
        if k in row and row[k] not in ("", None):
            g = int(float(row[k]))
            if k == "Grid_Size_X":
                g *= int(float(row.get("Grid_Size_Y", 1))) * int(float(row.get("Grid_Size_Z", 1)))
            return g
    return 0


def trace_table(d: str, title: str, cmd: str, top: int = 24) -> str:
    rows = _csv(d, "kernel_trace.csv")
    groups = collections.defaultdict(list)
    for r in rows:
        dur = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3   # us
        groups[(_short(r["Kernel_Name"]), _grid(r))].append(dur)
    total = sum(sum(v) for v in groups.values())
    out = [f"# {title}", "", "Command (from the repository root, one MI355X):", "", "```",
           cmd, "```", "",
           "| kernel | grid | calls | total us | avg us | median us | % |",
           "|---|---|---|---|---|---|---|"]
    for (name, grid), v in sorted(groups.items(), key=lambda kv: -sum(kv[1]))[:top]:
        out.append(f"| `{name}` | {grid} | {len(v)} | {sum(v):.1f} | {sum(v) / len(v):.3f} | "
                   f"{statistics.median(v):.3f} | {100 * sum(v) / total:.1f} |")
    return "\n".join(out) + "\n"


def _counter(d: str, counter: str, match: str):
    """Per-dispatch values of `counter` for kernels whose name contains `match`,
    keyed by grid size."""
    rows = _csv(d, "counter_collection.csv")
    by_grid = collections.defaultdict(list)
    for r in rows:
        if r["Counter_Name"] != counter or match not in r["Kernel_Name"]:
            continue
        by_grid[_grid(r)].append(float(r["Counter_Value"]))
    if not by_grid:
        raise ValueError(f"no {counter} rows for a kernel matching {match!r} in {d}")
    return by_grid


def traffic(args) -> dict:
    copy_bytes = args.copy_mib * (1 << 20)
    cf = _counter(args.copy_fetch, "FETCH_SIZE", "copy_kernel")
    cw = _counter(args.copy_write, "WRITE_SIZE", "copy_kernel")
    cf_kib = max(max(v) for v in cf.values())
    cw_kib = max(max(v) for v in cw.values())
    f_scale = copy_bytes / (cf_kib * 1024.0)
    w_scale = copy_bytes / (cw_kib * 1024.0)
    kernels = {}
    for spec in args.kernel:
        name, phase = spec.split(":")
        kf = _counter(args.fetch, "FETCH_SIZE", name)
        kw = _counter(args.write, "WRITE_SIZE", name)
        grid = max(kf)
        fk = statistics.mean(kf[grid])
        wk = statistics.mean(kw[grid])
        kernels[phase] = {"kernel": name, "grid": grid,
                          "dispatches": [len(kf[grid]), len(kw[grid])],
                          "fetch_kib_raw": fk, "write_kib_raw": wk,
                          "fetch_bytes_per_launch": fk * 1024.0 * f_scale,
                          "write_bytes_per_launch": wk * 1024.0 * w_scale,
                          "bytes_per_launch": fk * 1024.0 * f_scale + wk * 1024.0 * w_scale}
    return {"workload": args.workload, "source_sha": source_sha(), "commands": args.cmd,
            "copy_bytes": copy_bytes, "copy_fetch_kib": cf_kib, "copy_write_kib": cw_kib,
            "fetch_scale": f_scale, "write_scale": w_scale, "phases": kernels}


def counter_table(dirs, kernels, title: str, cmds) -> str:
    """Mean per dispatch of each counter in the runs under `dirs`, for the
    largest-grid launches of each kernel (NAME:PHASE, NAME a substring of
    the kernel name)."""
    rows = []
    for d in dirs:
        rows.extend(_csv(d, "counter_collection.csv"))
    names = sorted({r["Counter_Name"] for r in rows})
    out = [f"# {title}", "", "Commands (from the repository root, one MI355X):", "", "```"]
    out += list(cmds)
    out += ["```", "", "Mean value per dispatch (summed over the GPU's counter instances) of the "
            "largest-grid launches of each kernel.", ""]
    derived = []
    if "SQ_WAVE_CYCLES" in names:
        if "SQ_WAIT_ANY" in names:
            derived.append(("wait/wave", "SQ_WAIT_ANY"))
        if "SQ_BUSY_CYCLES" in names:
            derived.append(("busy/wave", "SQ_BUSY_CYCLES"))
        if "SQ_WAIT_INST_LDS" in names:
            derived.append(("lds-wait/wave", "SQ_WAIT_INST_LDS"))
    out.append("| phase | kernel | grid | dispatches | " + " | ".join(names) +
               "".join(f" | {n}" for n, _ in derived) + " |")
    out.append("|---" * (4 + len(names) + len(derived)) + "|")
    for spec in kernels:
        name, phase = spec.split(":")
        vals = {}
        grid = None
        nd = 0
        for c in names:
            try:
                by = _counter_rows(rows, c, name)
            except ValueError:
                continue
            g = max(by)
            grid = g if grid is None else grid
            vals[c] = statistics.mean(by[g])
            nd = max(nd, len(by[g]))
        cells = [f"{vals[c]:.4g}" if c in vals else "" for c in names]
        for _, c in derived:
            cells.append(f"{vals[c] / vals['SQ_WAVE_CYCLES']:.3f}"
                         if c in vals and vals.get("SQ_WAVE_CYCLES") else "")
        out.append(f"| {phase} | `{name}` | {grid} | {nd} | " + " | ".join(cells) + " |")
    return "\n".join(out) + "\n"


def _counter_rows(rows, counter: str, match: str):
    by_grid = collections.defaultdict(list)
    for r in rows:
        if r["Counter_Name"] != counter or match not in r["Kernel_Name"]:
            continue
        by_grid[_grid(r)].append(float(r["Counter_Value"]))
    if not by_grid:
        raise ValueError(f"no {counter} rows for a kernel matching {match!r}")
    return by_grid


def traffic_md(rec: dict) -> str:
    out = [f"# HBM traffic per launch, workload {rec['workload']}", "",
           "Commands (from the repository root, one MI355X):", "", "```"]
    out += rec["commands"]
    out += ["```", "",
            f"Calibration: a plain copy of {rec['copy_bytes']} B reads "
            f"FETCH_SIZE {rec['copy_fetch_kib']:.0f} KiB and WRITE_SIZE "
            f"{rec['copy_write_kib']:.0f} KiB; the counters are scaled by "
            f"{rec['fetch_scale']:.4f} and {rec['write_scale']:.4f}.  Kernel sources "
            f"{rec['source_sha']}.", "",
            "| phase | kernel | grid | fetch MB | write MB | total MB |",
            "|---|---|---|---|---|---|"]
    for ph, k in rec["phases"].items():
        out.append(f"| {ph} | `{k['kernel']}` | {k['grid']} | "
                   f"{k['fetch_bytes_per_launch'] / 1e6:.1f} | "
                   f"{k['write_bytes_per_launch'] / 1e6:.1f} | {k['bytes_per_launch'] / 1e6:.1f} |")
    return "\n".join(out) + "\n"


def copy_once(mib: int):
    import torch
    from . import probe
    lib = probe._load()
    n = mib * (1 << 20)
    src = torch.ones(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    rc = lib.cmprobe_copy(src.data_ptr(), dst.data_ptr(), n, 1,
                          torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    if rc != 0:
        raise RuntimeError(f"cmprobe_copy failed: {rc}")
    print(f"copied {n} bytes", flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_2412_06359_amd.profsum")
    sub = ap.add_subparsers(dest="cmd_name", required=True)
    c = sub.add_parser("copy")
    c.add_argument("--mib", type=int, default=512)
    t = sub.add_parser("trace")
    t.add_argument("dir")
    t.add_argument("--title", required=True)
    t.add_argument("--cmd", required=True)
    t.add_argument("--out")
    f = sub.add_parser("traffic")
    for k in ("workload", "fetch", "write", "copy_fetch", "copy_write", "out"):
        f.add_argument("--" + k.replace("_", "-"), dest=k, required=True)
    f.add_argument("--kernel", action="append", required=True, help="NAME:PHASE")
    f.add_argument("--copy-mib", type=int, default=512)
    f.add_argument("--cmd", action="append", default=[])
    k = sub.add_parser("counters")
    k.add_argument("dirs", nargs="+")
    k.add_argument("--kernel", action="append", required=True, help="NAME:PHASE")
    k.add_argument("--title", required=True)
    k.add_argument("--cmd", action="append", default=[])
    k.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    if a.cmd_name == "copy":
        copy_once(a.mib)
    elif a.cmd_name == "counters":
        with open(a.out, "w") as fh:
            fh.write(counter_table(a.dirs, a.kernel, a.title, a.cmd))
    elif a.cmd_name == "trace":
        s = trace_table(a.dir, a.title, a.cmd)
        if a.out:
            with open(a.out, "w") as fh:
                fh.write(s)
        else:
            sys.stdout.write(s)
    else:
        rec = traffic(a)
        with open(a.out, "w") as fh:
            json.dump(rec, fh, indent=1)
            fh.write("\n")
        with open(os.path.splitext(a.out)[0] + ".md", "w") as fh:
            fh.write(traffic_md(rec))


if __name__ == "__main__":
    main()
