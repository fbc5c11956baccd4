"""Summaries of rocprofv3 output for the sweep kernels.

``stats``: turn a ``--kernel-trace --stats --output-format csv`` run into a short
markdown table.  ``trace``: the same from the per-dispatch kernel trace, for the
dispatches between the first two marker kernels (``k_probe_fill``; bench.py
queues one right before and one right after its timed region), so that the
table covers exactly the timed launches and no autotuner candidate.  ``traffic``: HBM bytes per launch of a kernel from two
``--pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE`` runs of a program that also made a
device copy of known size (``bench.py --calibrate-copy``): each counter is scaled
by what it reads for that copy, which moves exactly its size in each direction;
only the sweep dispatches between the two marker fills count, and only the copies
after the second one (the autotuner copies spins before the timed region).
``valu``: VALU wave instructions per launch of the timed sweep launches, from a
``--pmc SQ_INSTS_VALU GRBM_GUI_ACTIVE`` run, for the ALU roofline of sizes that
the VALU rather than HBM bounds.

    python -m paper_1411_0127_amd.profiling stats  <stats.csv> <out.md> "<command>"
    python -m paper_1411_0127_amd.profiling trace  <kernel_trace.csv> <out.md> "<command>"
    python -m paper_1411_0127_amd.profiling traffic <fetch.csv> <write.csv> <workload> <copy_bytes> "<command>" [tile]
    python -m paper_1411_0127_amd.profiling valu <counters.csv> <workload> "<command>" <tile>
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


MARKER_KERNEL = "k_probe_fill"


def _short(name: str) -> str:
    name = name.replace("(anonymous namespace)::", "").replace("void ", "")
    return name[: name.index(">") + 1] if "<" in name.split("(")[0] else name.split("(")[0]


def _table(rows):
    by = {}
    for name, ns in rows:
        by.setdefault(_short(name), []).append(ns)
    total = sum(sum(v) for v in by.values()) or 1.0
    lines = ["| kernel | calls | average (us) | min (us) | max (us) | total (ms) | share |",
             "|---|---|---|---|---|---|---|"]
    for k, v in sorted(by.items(), key=lambda kv: -sum(kv[1])):
        lines.append(f"| `{k}` | {len(v)} | {statistics.mean(v) / 1e3:.2f} | {min(v) / 1e3:.2f} | "
                     f"{max(v) / 1e3:.2f} | {sum(v) / 1e6:.3f} | {100.0 * sum(v) / total:.1f}% |")
    return lines


def trace(csv_path: str, out_md: str, command: str) -> str:
    rows = []
    for r in csv.DictReader(open(csv_path)):
        name = r.get("Kernel_Name") or r.get("Name") or ""
        t0, t1 = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
        rows.append((t0, t1, name))
    rows.sort()
    marks = [k for k, (_, _, n) in enumerate(rows) if MARKER_KERNEL in n]
    lines = ["# rocprofv3 kernel trace", "", f"Command: `{command}`", ""]
    if len(marks) >= 2:
        a, b = marks[0], marks[1]
        inside = [(n, t1 - t0) for t0, t1, n in rows[a + 1:b]]
        span = (rows[b][0] - rows[a][1]) / 1e6
        lines += [f"Timed region (dispatches between the two marker fills): {len(inside)} dispatches, "
                  f"{span:.3f} ms from the end of the first marker to the start of the second.", ""]
        lines += _table(inside)
        lines.append("")
    lines += ["All dispatches of the program:", ""]
    lines += _table([(n, t1 - t0) for t0, t1, n in rows])
    lines.append("")
    with open(out_md, "w") as f:
        f.write("\n".join(lines))
    return out_md


def _per_dispatch(path: str, counter: str, part: str = "all"):
    """Counter value per dispatch, by kernel name.  part = "timed": only the
    dispatches between the first two marker fills (the timed region); "after":
    only those after the second (where bench.py makes its calibration copies)."""
    rows = []
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        rows.append((int(r.get("Dispatch_Id") or 0), r["Kernel_Name"], float(r["Counter_Value"])))
    rows.sort(key=lambda t: t[0])
    if part != "all":
        marks = [k for k, (_, n, _) in enumerate(rows) if MARKER_KERNEL in n]
        if len(marks) < 2:
            raise SystemExit("the counter file has no two marker fills")
        rows = rows[marks[0] + 1:marks[1]] if part == "timed" else rows[marks[1] + 1:]
    vals = {}
    for _, name, v in rows:
        vals.setdefault(name, []).append(v)
    return vals


def traffic(fetch_csv: str, write_csv: str, workload: str, copy_bytes: int, command: str, out_dir: str = "",
            tile: str = "") -> str:
    """HBM bytes per sweep launch of `workload`; `tile` ("kind,tile_x,tile_y,z_chunk,band,planes", the
    `bench.py --tile` the counter runs were given) is recorded and names the file, so that a
    benchmark run applies the record only to launches of that shape."""
    # the sweep launches of the timed region only (no autotuner candidate), and the
    # calibration copies made after it (not the autotuner's copies of the spins)
    ft = _per_dispatch(fetch_csv, "FETCH_SIZE", "timed")
    wt = _per_dispatch(write_csv, "WRITE_SIZE", "timed")
    f = _per_dispatch(fetch_csv, "FETCH_SIZE", "after")
    w = _per_dispatch(write_csv, "WRITE_SIZE", "after")

    def pick(d, key):
        ks = [k for k in d if key in k]
        if not ks:
            raise SystemExit(f"no {key} dispatches in the counter file")
        return [v for k in ks for v in d[k]]

    sweep_f = pick(ft, SWEEP_KERNEL)
    sweep_w = pick(wt, SWEEP_KERNEL)
    names = sorted({k for k in ft if SWEEP_KERNEL in k})
    short = sorted({n.replace("(anonymous namespace)::", "").replace("void ", "").split("(")[0] for n in names})
    copy_f = statistics.median(pick(f, COPY_KERNEL))
    copy_w = statistics.median(pick(w, COPY_KERNEL))
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
    name = workload
    if tile:
        rec["tile"], tag = _tile_list(tile)
        name += "_" + tag
    out = os.path.join(out_dir or os.path.join(ROOT, "profiles"), f"traffic_sweep_fused_{name}.json")
    with open(out, "w") as fh:
        json.dump(rec, fh, indent=1)
    return out


def _tile_list(tile: str):
    parts = [t.strip() for t in tile.split(",")]
    return [parts[0]] + [int(v) for v in parts[1:]], "_".join(parts)


def valu(csv_path: str, workload: str, command: str, tile: str, out_dir: str = "") -> str:
    """VALU wave instructions (SQ_INSTS_VALU, summed over the device) and GPU-active
    cycles (GRBM_GUI_ACTIVE) per timed sweep launch of `bench.py --tile <tile>`."""
    insts = _per_dispatch(csv_path, "SQ_INSTS_VALU", "timed")
    active = _per_dispatch(csv_path, "GRBM_GUI_ACTIVE", "timed")

    def sweep(d):
        v = [x for k in d if SWEEP_KERNEL in k for x in d[k]]
        if not v:
            raise SystemExit("no sweep dispatches in the timed region of the counter file")
        return v

    names = sorted({k for k in insts if SWEEP_KERNEL in k})
    short = sorted({n.replace("(anonymous namespace)::", "").replace("void ", "").split("(")[0] for n in names})
    tl, tag = _tile_list(tile)
    rec = {
        "kernel": ", ".join(short),
        "workload": workload,
        "tile": tl,
        "kernel_source_sha": kernel_source_sha(),
        "valu_wave_insts_per_launch": statistics.median(sweep(insts)),
        "gui_active_cycles_per_launch": statistics.median(sweep(active)),
        "launches": len(sweep(insts)),
        "command": command,
    }
    out = os.path.join(out_dir or os.path.join(ROOT, "profiles"), f"valu_sweep_fused_{workload}_{tag}.json")
    with open(out, "w") as fh:
        json.dump(rec, fh, indent=1)
    return out


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        print(stats(sys.argv[2], sys.argv[3], sys.argv[4]))
    elif sys.argv[1] == "trace":
        print(trace(sys.argv[2], sys.argv[3], sys.argv[4]))
    elif sys.argv[1] == "traffic":
        print(traffic(sys.argv[2], sys.argv[3], sys.argv[4], int(sys.argv[5]), sys.argv[6],
                      tile=sys.argv[7] if len(sys.argv) > 7 else ""))
    elif sys.argv[1] == "valu":
        print(valu(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5]))
    else:
        raise SystemExit(__doc__)
