"""Summaries of rocprofv3 output for the sweep kernels.

``stats``: turn a ``--kernel-trace --stats --output-format csv`` run into a short
markdown table.  ``traffic``: HBM bytes per launch of a kernel from two
``--pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE`` runs of a program that also made a
device copy of known size (``bench.py --calibrate-copy``): each counter is scaled
by what it reads for that copy, which moves exactly its size in each direction.

    python -m paper_1411_0127_amd.profiling stats  <stats.csv> <out.md> "<command>"
    python -m paper_1411_0127_amd.profiling traffic <fetch.csv> <write.csv> <workload> <copy_bytes> "<command>"
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import re
import statistics
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SWEEP_KERNEL = "k_fused"
COPY_KERNEL = "copyBuffer"


def _code_only(src: str) -> str:
    """The source without comments and blank lines: what the compiler sees."""
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    return "\n".join(line.rstrip() for line in src.splitlines() if line.strip())


def kernel_source_sha() -> str:
    """Hash of the sweep kernels' code; counters taken on other code are stale."""
    h = hashlib.sha256()
    for f in ("kernels_sweep_fused.hip", "sg_internal.h"):
        with open(os.path.join(ROOT, "paper_1411_0127_amd", "csrc", f)) as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def stats(csv_path: str, out_md: str, command: str) -> str:
    rows = list(csv.DictReader(open(csv_path)))
    lines = [
        f"# rocprofv3 kernel statistics",
        "",
        f"Command: `{command}`",
        "",
        "| kernel | calls | average (us) | min (us) | max (us) | share |",
        "|---|---|---|---|---|---|",
    ]
    for r in rows:
        name = (r.get("Name") or r.get("KernelName") or "").replace("(anonymous namespace)::", "")
        short = name.replace("void ", "")
        short = short[: short.index(">") + 1] if "<" in short.split("(")[0] else short.split("(")[0]
        calls = int(float(r.get("Calls", 0)))
        avg = float(r.get("AverageNs", 0)) / 1e3
        mn = float(r.get("MinNs", 0)) / 1e3
        mx = float(r.get("MaxNs", 0)) / 1e3
        pct = float(r.get("Percentage", 0))
        lines.append(f"| `{short}` | {calls} | {avg:.2f} | {mn:.2f} | {mx:.2f} | {pct:.1f}% |")
    lines.append("")
    with open(out_md, "w") as f:
        f.write("\n".join(lines))
    return out_md


def _per_dispatch(path: str, counter: str):
    vals = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        vals.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return vals


def traffic(fetch_csv: str, write_csv: str, workload: str, copy_bytes: int, command: str) -> str:
    f = _per_dispatch(fetch_csv, "FETCH_SIZE")
    w = _per_dispatch(write_csv, "WRITE_SIZE")

    def pick(d, key):
        ks = [k for k in d if key in k]
        if not ks:
            raise SystemExit(f"no {key} dispatches in the counter file")
        return [v for k in ks for v in d[k]]

    sweep_f = pick(f, SWEEP_KERNEL)
    sweep_w = pick(w, SWEEP_KERNEL)
    names = sorted({k for k in f if SWEEP_KERNEL in k})
    short = sorted({n.replace("(anonymous namespace)::", "").replace("void ", "").split("(")[0] for n in names})
    copy_f = max(pick(f, COPY_KERNEL))
    copy_w = max(pick(w, COPY_KERNEL))
    # counters are in KiB; the copy read and wrote copy_bytes each
    f_scale = copy_bytes / (copy_f * 1024.0)
    w_scale = copy_bytes / (copy_w * 1024.0)
    fb = statistics.median(sweep_f) * 1024.0 * f_scale
    wb = statistics.median(sweep_w) * 1024.0 * w_scale
    rec = {
        "kernel": ", ".join(short),
        "workload": workload,
        "kernel_source_sha": kernel_source_sha(),
        "fetch_kib_per_launch_raw": statistics.median(sweep_f),
        "write_kib_per_launch_raw": statistics.median(sweep_w),
        "copy_bytes": copy_bytes,
        "copy_fetch_kib": copy_f,
        "copy_write_kib": copy_w,
        "fetch_scale": f_scale,
        "write_scale": w_scale,
        "hbm_read_bytes_per_launch": fb,
        "hbm_write_bytes_per_launch": wb,
        "hbm_bytes_per_launch": fb + wb,
        "command_fetch": command.replace("<COUNTER>", "FETCH_SIZE"),
        "command_write": command.replace("<COUNTER>", "WRITE_SIZE"),
    }
    out = os.path.join(ROOT, "profiles", f"traffic_sweep_fused_{workload}.json")
    with open(out, "w") as fh:
        json.dump(rec, fh, indent=1)
    return out


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        print(stats(sys.argv[2], sys.argv[3], sys.argv[4]))
    elif sys.argv[1] == "traffic":
        print(traffic(sys.argv[2], sys.argv[3], sys.argv[4], int(sys.argv[5]), sys.argv[6]))
    else:
        raise SystemExit(__doc__)
