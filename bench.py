#!/usr/bin/env python3
"""Benchmark of the checkerboard Metropolis sweep on one MI355X.

A step is one job of the workload: ``sweeps_per_step`` sweeps of every replica
(couplings read once per sweep for both replicas), then the energy of each replica
and their overlap read back.  Lattices, couplings and streams are created on the
device before the timed region.  The JSON line reports ps per spin flip
(psFlip, lower is better) as ``value``; the roofline object covers the sweep kernel,
whose average duration per launch is measured with HIP events on the stream the
kernel runs on.  ``cpu_baseline`` times the CPU oracle on a bounded sample of the
same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ps per spin flip (psFlip) + HBM GB/s, single lattice and batched; job p50/p99"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    # L=256 cube, 64 samples per word, 2 replicas sharing the couplings, T=0.7
    "c1": dict(L=256, replicas=2, beta=1 / 0.7, sweeps=1000, prng="minstd",
               variant=("mt19937", "parisi_rapuano", "philox"),
               desc="L=256 periodic cube, 64 samples multispin-coded per uint64, 2 replicas sharing "
                    "J=+-1 (p=1/2), random start, T=0.7, 1000 sweeps per step, MINSTD per-site streams "
                    "(variants: MT19937 and Parisi-Rapuano per-column streams; one Philox number per sample)"),
    # L=1024 cube, 64 samples, one replica, T=1.1, 100 sweeps
    "c2": dict(L=1024, replicas=1, beta=1 / 1.1, sweeps=100, prng="minstd", variant=None,
               desc="L=1024 periodic cube, 64 samples multispin-coded per uint64, J=+-1 (p=1/2), "
                    "random start, T=1.1, 100 sweeps per step, MINSTD per-site streams"),
    # 256 lattices in one batch: L from {32,...,512}, T in [0.5, 1.5], 100-2000 sweeps
    "c3": dict(L=0, replicas=1, beta=0, sweeps=0, prng="minstd", variant=None,
               desc="batch of 256 lattices, L uniform over {32,64,128,256,512}, 64 samples each, T uniform "
                    "[0.5,1.5], sweeps uniform 100-2000 (times sweep_scale), all present at t=0, admitted by "
                    "HBM budget, one launch per round, MINSTD"),
    # Poisson job stream at 50 jobs/s: L from {64,...,512}, T in [0.6, 1.4], 10^U(2,4) sweeps
    "c4": dict(L=0, replicas=1, beta=0, sweeps=0, prng="minstd", variant=None,
               desc="served Poisson job stream (mean 50 jobs/s), L uniform over {64,128,256,512}, 64 samples, "
                    "T uniform [0.6,1.4], sweeps 10^U(2,4) (times sweep_scale), admitted by HBM budget, "
                    "continuous batching, MINSTD"),
    # L=16 cube, 1 sample, energy after every sweep
    "c0": dict(L=16, replicas=1, beta=1 / 0.7, sweeps=1000, prng="minstd", variant=None, samples=1,
               desc="L=16 periodic cube, 1 sample, T=0.7, 1000 sweeps per step, MINSTD"),
}


def algorithmic_bytes_per_site(prng: str, replicas: int, sweeps_per_launch: int = 1) -> int:
    """Bytes one fused sweep launch must move per lattice site.

    Couplings: 3 words read once for all replicas (24 B).  Per replica: the spin
    word read and written (16 B); with MT19937 or Parisi-Rapuano also the draw of
    every sweep of the launch, read from the buffer the fill kernel wrote (4 B
    each).  MINSTD draws are computed from the site and the sweep, nothing is read
    for them.  The fill kernel's own state traffic is not part of the sweep kernel.
    A two-sweep launch reads and writes every spin and coupling word once for both
    sweeps.
    """
    draws = 4 * sweeps_per_launch if prng in ("mt19937", "parisi_rapuano") else 0
    return 24 + replicas * (16 + draws)


def kernel_source_sha() -> str:
    from paper_1411_0127_amd.profiling import kernel_source_sha as sha

    return sha()


def load_traffic(workload: str):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were
    taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_sweep_fused_{workload}.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_sha") != kernel_source_sha():
        return None
    return rec.get("hbm_bytes_per_launch")


def run_gpu(args, wl):
    import torch

    from paper_1411_0127_amd import sg

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    L, R, beta, nsw = wl["L"], wl["replicas"], wl["beta"], args.sweeps or wl["sweeps"]
    S = wl.get("samples", 64)  # coded samples per word; flips are counted for these only
    V = L**3

    def measure(prng):
        base = sg.Lattice(L, S, prng, coupling_seed=1, spin_seed=2, replica=0, device=dev, stream=stream)
        lats = [base] + [sg.Lattice.replica_of(base, spin_seed=2, replica=r) for r in range(1, R)]
        shape = None
        if args.tile:
            parts = args.tile.split(",")
            kind = parts[0] if not parts[0].isdigit() else "fused"
            nums = tuple(int(v) for v in (parts[1:] if not parts[0].isdigit() else parts))
            buffered = prng in ("mt19937", "parisi_rapuano")
            for l in lats:
                l.set_kernel(kind, *nums[:4])
                if len(nums) > 4:
                    l.set_ring(5 if buffered else nums[4])  # buffered draws: five planes in flight
        elif args.kernel == "auto":
            # pick the fused kernel and tile on these lattices, before the timed region
            shape, _ = sg.autotune(lats[:2], reps=5)
            for l in lats[2:]:
                l.set_kernel(shape[0], *shape[1:])
        else:
            for l in lats:
                l.set_kernel(args.kernel)
        if shape is not None or args.tile:
            shape = lats[0].kernel()  # kind, tile_x, tile_y, z_chunk, band, planes in flight
        kind = shape[0] if shape else args.kernel
        per_launch = 2 if kind in ("fused2", "auto") and nsw % 2 == 0 else 1

        def step(ev=None):
            if ev is not None:
                ev[0].record(stream)
            if R == 1:
                lats[0].sweep(nsw, beta)
            else:
                sg.sweep_replicas(lats, nsw, beta)
            if ev is not None:
                ev[1].record(stream)
            out = [l.energy() for l in lats]
            if R >= 2:
                out.append(sg.overlap(lats[0], lats[1]))
            return out

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                  for _ in range(args.steps)]
        t0 = time.perf_counter()
        for k in range(args.steps):
            last = step(events[k])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        sweep_ms = [a.elapsed_time(b) for a, b in events]
        res = dict(
            wall_s=wall,
            ms_per_step=wall * 1e3 / args.steps,
            sweep_ms_per_step=sweep_ms,
            launch_ms=sum(sweep_ms) / (args.steps * nsw / per_launch),
            sweeps_per_launch=per_launch,
            kind=kind,
            energy_per_spin=[float(x) for x in last[0][1][:4]],
            tile=shape,
        )
        flips = R * S * V * nsw
        res["ps_per_flip"] = res["ms_per_step"] * 1e9 / flips
        res["sweep_ps_per_flip"] = (sum(sweep_ms) / args.steps) * 1e9 / flips
        for l in lats:
            l.close()
        del lats, base
        torch.cuda.empty_cache()
        return res

    main = measure(wl["prng"])
    if args.layout_ab:
        main["layout_ab"] = layout_ab(sg, torch, wl, stream, dev)
    variants = {}
    if not args.no_variant:
        for v in wl.get("variant") or ():
            variants[v] = measure(v)
    return main, variants


def layout_ab(sg, torch, wl, stream, dev, nsw=4):
    """ms per sweep of the two-pass kernel on the cube and on the colour-separated
    layout (conversion excluded: the difference of nsw sweeps and none), same lattice."""
    L, beta = wl["L"], wl["beta"]
    lat = sg.Lattice(L, 64, wl["prng"], coupling_seed=1, spin_seed=2, device=dev, stream=stream)
    work = torch.empty(sg.sliced_footprint(L), dtype=torch.uint8, device=dev)
    lat.set_kernel("twopass")

    def timed(fn):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        fn()  # warm-up
        torch.cuda.synchronize()
        a.record(stream)
        fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b)

    cube = timed(lambda: lat.sweep(nsw, beta)) / nsw
    full = timed(lambda: lat.sweep_sliced(nsw, beta, work))
    conv = timed(lambda: lat.sweep_sliced(0, beta, work))
    lat.set_kernel("auto")
    fused = timed(lambda: lat.sweep(nsw, beta)) / nsw
    lat.close()
    del work
    torch.cuda.empty_cache()
    return {"lattice": f"L={L}, 64 samples, one replica", "twopass_cube_ms_per_sweep": round(cube, 4),
            "twopass_sliced_ms_per_sweep": round((full - conv) / nsw, 4), "sliced_conversion_ms": round(conv, 4),
            "fused_default_ms_per_sweep": round(fused, 4)}


def _budget_bytes(torch, frac=0.8):
    return int(torch.cuda.get_device_properties(0).total_memory * frac)


def solo_sweep_ms(sg, torch, L, nsw=6):
    """ms per sweep of one lattice alone (autotuned fused kernel), on its own stream."""
    stream = torch.cuda.Stream(torch.device("cuda:0"))
    lat = sg.Lattice(L, 64, "minstd", coupling_seed=3, spin_seed=4, stream=stream)
    if L >= 64:
        sg.autotune([lat], reps=3)
    lat.sweep(2, 1.0)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    lat.sweep(nsw, 1.0)
    b.record(stream)
    torch.cuda.synchronize()
    lat.close()
    return a.elapsed_time(b) / nsw


def run_mix(args, wl):
    """Batched (c3) or served (c4) mix through the continuous-batching server."""
    import torch

    from paper_1411_0127_amd import sg
    from paper_1411_0127_amd.serve import GpuBackend, Server, trace_batch, trace_served

    scale = args.sweep_scale
    budget = _budget_bytes(torch)
    out = {}
    if args.workload == "c3":
        jobs = trace_batch(args.jobs or 256, seed=args.seed, sweep_scale=scale)
        be = GpuBackend(rounds_per_graph=8)
        be.pretune(j.L for j in jobs)  # one-time per side, outside the measured span
        rep = Server(be, budget, chunk_rounds=200, min_rounds=8).serve(jobs)
        s = rep.summary()
        sizes = sorted({j.L for j in jobs})
        t_solo = {L: solo_sweep_ms(sg, torch, L) for L in sizes}
        plain_s = sum(j.nsweeps * t_solo[j.L] for j in jobs) / 1e3
        out["ps_per_flip"] = s["ps_per_flip_makespan"]
        out["plain_ps_per_flip"] = plain_s * 1e12 / s["flips"]
        out["batched_over_plain"] = out["ps_per_flip"] / out["plain_ps_per_flip"]
        out["solo_ms_per_sweep"] = {str(L): round(v, 4) for L, v in t_solo.items()}
        out["summary"] = s
        out["bytes"] = sum(40 * j.L**3 * j.nsweeps for j in jobs)
        out["seconds"] = s["makespan_s"]
    else:
        jobs = trace_served(args.jobs or 64, rate=50.0, seed=args.seed, sweep_scale=scale)
        be = GpuBackend(rounds_per_graph=8)
        be.pretune(j.L for j in jobs)
        rep = Server(be, budget, chunk_rounds=100).serve(jobs)
        s = rep.summary()
        mean_job_s = s["busy_s"] / max(1, s["jobs"])
        rate = 0.7 / max(mean_job_s, 1e-6)
        jobs2 = trace_served(max(8, (args.jobs or 64) // 2), rate=rate, seed=args.seed + 1, sweep_scale=scale)
        rep2 = Server(be, budget, chunk_rounds=100).serve(jobs2)
        s2 = rep2.summary()
        out["ps_per_flip"] = s["ps_per_flip_busy"]
        out["summary"] = s
        out["sub_saturating"] = dict(rate_jobs_per_s=rate, **s2)
        out["bytes"] = sum(40 * j.L**3 * j.nsweeps for j in jobs)
        out["seconds"] = s["busy_s"]
    return out


def cpu_baseline(wl, budget_s: float):
    """The oracle as it stands, single-threaded, on one sample of one replica."""
    import numpy as np

    import oracle
    import seeded_inputs as si

    L, beta = wl["L"], wl["beta"]
    L = min(L, 256)
    J = si.coupling_words(L, 1) & np.uint64(1)
    S0 = si.spin_words(L, 2, 0) & np.uint64(1)
    lat = oracle.OracleLattice((L, L, L), 1, J, S0, oracle.MINSTD, si.minstd_seeds(L, 2, 0))
    t0 = time.perf_counter()
    lat.run(1, beta)
    one = time.perf_counter() - t0
    n = max(1, min(int(budget_s / max(one, 1e-9)), 2000))
    t0 = time.perf_counter()
    lat.run(n, beta)
    dt = time.perf_counter() - t0
    return dict(value=dt * 1e12 / (L**3 * n), unit="ps/flip", cores=1, kind="oracle",
                sample=f"L={L} cube, 1 of the 64 samples, 1 replica, {n} MINSTD sweeps at T={1 / beta:.2f}, "
                       f"one byte per spin, single thread ({dt:.1f} s)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c1", choices=sorted(WORKLOADS))
    ap.add_argument("--sweeps", type=int, default=0, help="sweeps per step (default: the workload's)")
    ap.add_argument("--kernel", default="auto", choices=["auto", "fused", "fused2", "twopass"])
    ap.add_argument("--tile", default="",
                    help="kernel and tile [fused|fused2,]tile_x,tile_y,z_chunk,band[,planes] (skips the autotuner)")
    ap.add_argument("--no-variant", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0, help="seconds of oracle work for cpu_baseline")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--sweep-scale", type=float, default=0.1,
                    help="c3/c4: multiply every job's sweep count (the full mixes take minutes)")
    ap.add_argument("--jobs", type=int, default=0, help="c3/c4: number of jobs (default 256 / 64)")
    ap.add_argument("--seed", type=int, default=1, help="c3/c4: trace seed")
    ap.add_argument("--layout-ab", action="store_true",
                    help="also time the two-pass kernel on the cube and on the colour-separated layout")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="also make 3 device copies of BYTES bytes, for counter calibration")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only; --gpus {args.gpus} is not supported "
              "(independent lattices and replicas would shard by job placement, one GPU each).",
              file=sys.stderr)
        sys.exit(2)

    wl = WORKLOADS[args.workload]
    if args.workload in ("c3", "c4"):
        res = run_mix(args, wl)
        gbs = res["bytes"] / res["seconds"] / 1e9
        line = {
            "metric": METRIC,
            "value": round(res["ps_per_flip"], 6),
            "unit": "ps/flip",
            "n_gpus": 1,
            "steps": 1,
            "warmup": 0,
            "ms_per_step": round(res["seconds"] * 1e3, 3),
            "higher_is_better": False,
            "scaling": "weak",
            "vs_baseline": None,
            "dtype": "u64",
            "data": "synthetic",
            "config": {"workload": wl["desc"], "sweep_scale": args.sweep_scale, "jobs": res["summary"]["jobs"],
                       "seed": args.seed, "parallelism": "single GPU"},
            "hbm_gbs_algorithmic": round(gbs, 1),
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": None,
                         "kernel": "sg::k_fused_batch (all resident lattices, one launch per round)",
                         "bytes_per_site": 40},
        }
        for k in ("plain_ps_per_flip", "batched_over_plain", "solo_ms_per_sweep", "sub_saturating"):
            if k in res:
                line[k] = res[k]
        line["summary"] = res["summary"]
        print(json.dumps(line), flush=True)
        return
    main_res, variants = run_gpu(args, wl)
    if args.calibrate_copy:
        import torch

        src = torch.empty(args.calibrate_copy, dtype=torch.uint8, device="cuda:0").fill_(1)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    L, R = wl["L"], wl["replicas"]
    V = L**3
    bps = algorithmic_bytes_per_site(wl["prng"], R, main_res["sweeps_per_launch"])
    achieved = bps * V / (main_res["launch_ms"] * 1e-3) / 1e9
    eq = achieved * main_res["sweeps_per_launch"]
    traffic = load_traffic(args.workload)
    line = {
        "metric": METRIC,
        "value": round(main_res["ps_per_flip"], 6),
        "unit": "ps/flip",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_res["ms_per_step"], 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {
            "workload": wl["desc"],
            "L": L,
            "samples_per_word": wl.get("samples", 64),
            "replicas": R,
            "sweeps_per_step": args.sweeps or wl["sweeps"],
            "prng": wl["prng"],
            "kernel": args.kernel,
            "tile": main_res["tile"],
            "parallelism": "single GPU",
        },
        "hbm_gbs_algorithmic": round(achieved, 1),
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "kernel": ("sg::k_fused2 (two sweeps per launch, replicas interleaved)"
                       if main_res["sweeps_per_launch"] == 2 else "sg::k_fused (one launch per sweep, all replicas)"),
            "bytes_per_site": bps,
            "sweeps_per_launch": main_res["sweeps_per_launch"],
            "launch_ms": round(main_res["launch_ms"], 5),
            # what a one-sweep kernel would have to sustain for the same time per sweep
            "one_sweep_equivalent": {
                "achieved": round(eq, 1),
                "frac": round(eq / HBM_PEAK_GBS, 4),
            },
        },
    }
    if "layout_ab" in main_res:
        line["layout_ab"] = main_res["layout_ab"]
    if variants:
        line["variants"] = {
            name: {
                "ps_per_flip": round(v["ps_per_flip"], 6),
                "ms_per_step": round(v["ms_per_step"], 4),
                "launch_ms": round(v["launch_ms"], 5),
                "sweeps_per_launch": v["sweeps_per_launch"],
                "kernel": v["kind"],
            }
            for name, v in variants.items()
        }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(wl, args.cpu_budget)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
