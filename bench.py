#!/usr/bin/env python3
"""Benchmark of the checkerboard Metropolis sweep on one MI355X.

Headline (``--workload c2``, the default): one L=1024 lattice of 64 coded
samples at T=1.1, MINSTD.  A step is ``sweeps_per_step`` (100) sweeps followed
by the energy of every sample read back.  The lattice, its couplings and its
streams are created on the device before the timed region; the sweep kernel is
autotuned there too.  ``value`` is ps per spin flip (psFlip, Sec. 4.1 of the
paper, counted over 64-bit words: time / (samples x replicas x L^3 x sweeps)).

The same run adds, outside the timed region:
  roofline       the dominant kernel's algorithmic bytes per launch over its
                 average launch time (HIP events on the stream it runs on);
  measured_peak  read-only, copy and fill bandwidth of probe kernels over 4 GiB
                 buffers (the paper's analog: a device copy's peak, Sec. 4.1);
  depth1         the one-sweep-per-launch kernel on the same lattice, whose
                 bandwidth is the fraction read at temporal depth 1;
  c1             L=256, two replicas (MINSTD, MT19937, Parisi-Rapuano, and one
                 Philox number per sample);
  c3             the batched mix of 256 lattices, against plain launches: every
                 job alone, its lattice created, swept and its energies read
                 back, from per-side timings of the same steps;
  c4             the served Poisson job stream: p50/p99 latency, psFlip, and the
                 same comparison;
  cpu_baseline   the CPU oracle on bit-planes 0 and 63 of the same L=1024
                 lattice, threaded over all host cores, plus the L=16 one-sample
                 configuration on one core and on all cores.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ps per spin flip (psFlip) + HBM GB/s, single lattice and batched; job p50/p99"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "c0": dict(L=16, replicas=1, beta=1 / 0.7, sweeps=1000, prng="minstd", samples=1, energy_every_sweep=True,
               desc="c0: L=16 periodic cube, 1 sample, J=+-1 (p=1/2) and spins from seed, T=0.7, 1000 sweeps "
                    "per step with the energy per spin read after every sweep, MINSTD per-site streams"),
    "c1": dict(L=256, replicas=2, beta=1 / 0.7, sweeps=1000, prng="minstd",
               desc="c1: L=256 periodic cube, 64 samples multispin-coded per uint64, 2 replicas sharing J=+-1 "
                    "(p=1/2), random start, T=0.7, 1000 sweeps per step, MINSTD per-site streams"),
    "c2": dict(L=1024, replicas=1, beta=1 / 1.1, sweeps=100, prng="minstd",
               desc="c2: L=1024 periodic cube, 64 samples multispin-coded per uint64 (8 GiB spins, 24 GiB "
                    "couplings), J=+-1 (p=1/2), random start, T=1.1, 100 sweeps per step, MINSTD per-site "
                    "streams"),
}
MIX_DESC = {
    "c3": "c3: batch of 256 lattices, L uniform over {32,64,128,256,512}, 64 samples each, T uniform [0.5,1.5], "
          "sweeps uniform 100-2000 (times sweep_scale), all present at t=0, admitted by HBM budget, MINSTD",
    "c4": "c4: served Poisson job stream (mean 50 jobs/s), L uniform over {64,128,256,512}, 64 samples, T uniform "
          "[0.6,1.4], sweeps 10^U(2,4) (times sweep_scale), admitted by HBM budget, continuous batching, MINSTD",
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


def batch_bytes(jobs) -> int:
    """Compulsory bytes of a batched mix: 40 B per site and round, a round being
    two sweeps on the two-sweep march (one for an odd last sweep)."""
    return sum(40 * j.L**3 * ((j.nsweeps + 1) // 2) for j in jobs)


def kernel_source_sha() -> str:
    from paper_1411_0127_amd.profiling import kernel_source_sha as sha

    return sha()


def _load_record(prefix: str, field: str, name: str, kind: str, tile=None):
    """`field` of the committed rocprofv3 counter record (profiles/<prefix>_<name>*.json)
    of workload `name`, if it was taken on sweep kernel `kind` ("fused2", "fused"), on
    the current kernel source and (when `tile` is given) on launches of that shape
    (kind, tile_x, tile_y, z_chunk, band, planes); else None."""
    import glob

    sha = kernel_source_sha()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", f"{prefix}_{name}*.json"))):
        try:
            with open(path) as f:
                rec = json.load(f)
        except (OSError, ValueError):
            continue
        if rec.get("workload") != name or rec.get("kernel_source_sha") != sha:
            continue
        if not str(rec.get("kernel", "")).startswith(f"sg::k_{kind}<"):
            continue
        if tile is not None and [str(v) for v in rec.get("tile", [])] != [str(v) for v in tile]:
            continue
        return rec.get(field)
    return None


def load_traffic(name: str, kind: str, tile=None):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, scaled by a device copy)."""
    return _load_record("traffic_sweep_fused", "hbm_bytes_per_launch", name, kind, tile)


def load_valu(name: str, kind: str, tile=None):
    """VALU wave instructions per launch (SQ_INSTS_VALU over the device)."""
    return _load_record("valu_sweep_fused", "valu_wave_insts_per_launch", name, kind, tile)


# VALU issue peak: 256 CUs x 4 SIMDs, each issuing one wave64 instruction every 4
# cycles (16 lanes) at 2.4 GHz: 614.4 G wave instructions/s, i.e. 39.3 T lane-ops/s
# of 32-bit integer and bitwise work.
VALU_PEAK_WAVE_INSTS = 256 * 4 * 2.4e9 / 4


def alu_roofline(insts: float, launch_ms: float) -> dict:
    rate = insts / (launch_ms * 1e-3)
    return {"bound": "alu", "achieved": round(rate / 1e9, 1), "peak": round(VALU_PEAK_WAVE_INSTS / 1e9, 1),
            "unit": "G wave64 VALU instr/s", "frac": round(rate / VALU_PEAK_WAVE_INSTS, 4),
            "valu_wave_insts_per_launch": insts}


def kernel_label(kind: str, sweeps_per_launch: int) -> str:
    if sweeps_per_launch == 2:
        return "sg::k_fused2 (two sweeps per launch)"
    if kind == "fused2":
        return "sg::k_fused2 and a last sg::k_fused (odd sweep count; figures per sweep)"
    if kind == "twopass":
        return "sg::k_twopass (one launch per colour)"
    return "sg::k_fused (one sweep per launch)"


def host_threads() -> int:
    """Host threads this job may use: OMP_NUM_THREADS when set, else the cores the
    process may run on, at most 16."""
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return int(env)
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


# ---------------------------------------------------------------------------
# single lattice (c0, c1, c2)
# ---------------------------------------------------------------------------
class Marker:
    """A one-workgroup fill of 16 bytes queued before and after the timed region,
    so that a kernel trace of this program can be cut to the timed launches."""

    def __init__(self, torch, sg, stream):
        self.sg, self.stream = sg, stream
        self.buf = torch.empty(256, dtype=torch.uint8, device="cuda:0")

    def __call__(self):
        self.sg.probe_bandwidth("fill", self.buf, None, 16, self.stream, blocks=1)


def run_single(args, wl, prng=None, steps=None, warmup=None, marker=None, depth1=False):
    import torch

    from paper_1411_0127_amd import sg

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    prng = prng or wl["prng"]
    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    L, R, beta, nsw = wl["L"], wl["replicas"], wl["beta"], args.sweeps or wl["sweeps"]
    S = wl.get("samples", 64)  # coded samples per word; flips are counted for these only
    V = L**3
    base = sg.Lattice(L, S, prng, coupling_seed=1, spin_seed=2, replica=0, device=dev, stream=stream)
    lats = [base] + [sg.Lattice.replica_of(base, spin_seed=2, replica=r) for r in range(1, R)]
    if args.tile:
        parts = args.tile.split(",")
        kind = parts[0] if not parts[0].isdigit() else "fused"
        nums = tuple(int(v) for v in (parts[1:] if not parts[0].isdigit() else parts))
        buffered = prng in ("mt19937", "parisi_rapuano")
        for l in lats:
            l.set_kernel(kind, *nums[:4])
            if len(nums) > 4:
                l.set_ring(5 if buffered else nums[4])  # buffered draws: five planes in flight
    elif args.kernel == "auto" and L >= 32:
        # pick the kernel and tile on these lattices, before the timed region
        sg.autotune(lats[:2], reps=5)
        shape = lats[0].kernel()
        for l in lats[2:]:
            l.set_kernel(shape[0], *shape[1:5])
    elif args.kernel != "auto":
        for l in lats:
            l.set_kernel(args.kernel)
    shape = lats[0].kernel()  # kind, tile_x, tile_y, z_chunk, band, planes in flight
    per_launch = 2 if shape[0] == "fused2" and nsw % 2 == 0 else 1
    every = wl.get("energy_every_sweep", False)

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        if every:
            # the energy after every sweep, kept on the device and read back at the end
            U = lats[0].sweep_energies(nsw, beta)
            if ev is not None:
                ev[1].record(stream)
            return [(U[-1], (2.0 * U[-1] - 3.0 * V) / V)]
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

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    if marker is not None:
        marker()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        last = step(events[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if marker is not None:
        marker()
    sweep_ms = [a.elapsed_time(b) for a, b in events]
    flips = R * S * V * nsw
    res = dict(
        wall_s=wall,
        ms_per_step=wall * 1e3 / steps,
        sweep_ms_per_step=sweep_ms,
        launches_per_step=nsw // per_launch if per_launch == 2 else nsw,
        launch_ms=sum(sweep_ms) / (steps * nsw / per_launch),
        sweeps_per_launch=per_launch,
        kind=shape[0],
        tile=shape,
        energy_per_spin=[float(x) for x in last[0][1][:4]],
    )
    res["ps_per_flip"] = res["ms_per_step"] * 1e9 / flips
    res["sweep_ps_per_flip"] = (sum(sweep_ms) / steps) * 1e9 / flips
    if depth1 and R == 1:
        # the one-sweep kernel on the same lattice: bandwidth at temporal depth 1
        lats[0].set_kernel("fused")
        lats[0].sweep(2, beta)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        n1 = 6
        a.record(stream)
        lats[0].sweep(n1, beta)
        b.record(stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / n1
        k1 = lats[0].kernel()
        gbs = 40 * V / (ms * 1e-3) / 1e9
        res["depth1"] = {"kernel": "sg::k_fused<0, 1> (one sweep per launch)", "tile": list(k1), "ms_per_sweep":
                         round(ms, 4), "alg_gbs": round(gbs, 1), "frac_of_spec": round(gbs / HBM_PEAK_GBS, 4),
                         "bytes_per_site": 40}
    for l in lats:
        l.close()
    del lats, base
    torch.cuda.empty_cache()
    return res


def measure_peaks(nbytes: int = 4 << 30, reps: int = 5):
    """GB/s of the read, copy and fill probes over nbytes (best of reps), each the
    faster of its cached and its streaming (non-temporal) form."""
    import torch

    from paper_1411_0127_amd import sg

    stream = torch.cuda.current_stream()
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    dst = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    sg.probe_bandwidth("fill", src, None, nbytes, stream)
    sg.probe_bandwidth("fill", dst, None, nbytes, stream)
    out = {"bytes": nbytes}
    for kind, moved in (("read", nbytes), ("copy", 2 * nbytes), ("fill", nbytes)):
        rate = {}
        for form, name in ((kind, "cached"), (kind + "_nt", "streaming")):
            best = None
            for _ in range(reps + 1):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(stream)
                sg.probe_bandwidth(form, dst, src, nbytes, stream)
                b.record(stream)
                torch.cuda.synchronize()
                ms = a.elapsed_time(b)
                best = ms if best is None else min(best, ms)
            rate[name] = round(moved / (best * 1e-3) / 1e9, 1)
        out[f"{kind}_gbs"] = max(rate.values())
        out[f"{kind}_forms_gbs"] = rate
    del src, dst
    torch.cuda.empty_cache()
    return out


# ---------------------------------------------------------------------------
# batched (c3) and served (c4) mixes
# ---------------------------------------------------------------------------
def _budget_bytes(torch, frac=0.8):
    return int(torch.cuda.get_device_properties(0).total_memory * frac)


def solo_sweep_ms(sg, torch, L, nsw=20, repeats=3):
    """(ms per sweep, ms per job outside its sweeps) of one lattice alone (autotuned
    kernel), on its own stream: the best of `repeats` timings of `nsw` sweeps, and
    the best of `repeats` of what a job costs besides: creating the lattice
    (couplings and spins initialised on the device) and reading its energies back
    (count, sum and copy to the host), as the server does for every job."""
    stream = torch.cuda.Stream(torch.device("cuda:0"))
    c_best = float("inf")
    for k in range(repeats):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tmp = sg.Lattice(L, 64, "minstd", coupling_seed=5 + k, spin_seed=6 + k, stream=stream)
        torch.cuda.synchronize()
        c_best = min(c_best, (time.perf_counter() - t0) * 1e3)
        tmp.close()
        del tmp
    lat = sg.Lattice(L, 64, "minstd", coupling_seed=3, spin_seed=4, stream=stream)
    if L >= 64:
        sg.autotune([lat], reps=3)
    lat.sweep(2, 1.0)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(repeats):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        lat.sweep(nsw, 1.0)
        b.record(stream)
        torch.cuda.synchronize()
        best = min(best, a.elapsed_time(b) / nsw)
    e_best = float("inf")
    for _ in range(repeats):
        t0 = time.perf_counter()
        lat.energy()
        e_best = min(e_best, (time.perf_counter() - t0) * 1e3)
    lat.close()
    return best, c_best + e_best


def run_mix(kind: str, jobs_n: int, sweep_scale: float, seed: int, persistent: bool = False,
            group_bytes=None):
    """Batched (c3) or served (c4) mix through the continuous-batching server."""
    import torch

    from paper_1411_0127_amd import sg
    from paper_1411_0127_amd.serve import GpuBackend, Server, trace_batch, trace_served

    # memory cached by torch for earlier sections belongs to their streams, which this
    # mix does not use: hand it back first, so that the mix's lattices are allocated
    # without synchronising frees in the middle of serving
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    budget = _budget_bytes(torch)
    out = {"workload": MIX_DESC[kind], "sweep_scale": sweep_scale, "seed": seed}
    if kind == "c3":
        jobs = trace_batch(jobs_n or 256, seed=seed, sweep_scale=sweep_scale)
        be = GpuBackend(rounds_per_graph=8, persistent=persistent, group_bytes=group_bytes)
        be.pretune(j.L for j in jobs)  # one-time per side, outside the measured span
        rep = Server(be, budget, chunk_rounds=200, min_rounds=8).serve(jobs)
        s = rep.summary()
        sizes = sorted({j.L for j in jobs})
        t_solo = {L: solo_sweep_ms(sg, torch, L) for L in sizes}
        plain_s = sum(j.nsweeps * t_solo[j.L][0] + t_solo[j.L][1] for j in jobs) / 1e3
        out["ps_per_flip"] = s["ps_per_flip_makespan"]
        out["plain_ps_per_flip"] = plain_s * 1e12 / s["flips"]
        out["batched_over_plain"] = out["ps_per_flip"] / out["plain_ps_per_flip"]
        out["solo_ms_per_sweep"] = {str(L): round(v[0], 4) for L, v in t_solo.items()}
        out["solo_ms_per_job_outside_sweeps"] = {str(L): round(v[1], 4) for L, v in t_solo.items()}
        out["seconds"] = s["makespan_s"]
    else:
        jobs = trace_served(jobs_n or 64, rate=50.0, seed=seed, sweep_scale=sweep_scale)
        be = GpuBackend(rounds_per_graph=8, persistent=persistent, group_bytes=group_bytes)
        be.pretune(j.L for j in jobs)
        rep = Server(be, budget, chunk_rounds=100).serve(jobs)
        s = rep.summary()
        mean_job_s = s["busy_s"] / max(1, s["jobs"])
        rate = 0.7 / max(mean_job_s, 1e-6)
        jobs2 = trace_served(max(8, (jobs_n or 64) // 2), rate=rate, seed=seed + 1, sweep_scale=sweep_scale)
        rep2 = Server(be, budget, chunk_rounds=100).serve(jobs2)
        s2 = rep2.summary()
        out["ps_per_flip"] = s["ps_per_flip_busy"]
        t_solo = {L: solo_sweep_ms(sg, torch, L) for L in sorted({j.L for j in jobs})}
        plain_s = sum(j.nsweeps * t_solo[j.L][0] + t_solo[j.L][1] for j in jobs) / 1e3
        out["plain_ps_per_flip"] = plain_s * 1e12 / s["flips"]
        out["served_over_plain"] = out["ps_per_flip"] / out["plain_ps_per_flip"]
        out["p50_latency_s"] = s["p50_latency_s"]
        out["p99_latency_s"] = s["p99_latency_s"]
        out["sub_saturating"] = dict(rate_jobs_per_s=rate, **s2)
        out["seconds"] = s["busy_s"]
    out["summary"] = s
    out["compulsory_bytes"] = batch_bytes(jobs)
    gbs = out["compulsory_bytes"] / out["seconds"] / 1e9
    out["alg_gbs"] = round(gbs, 1)
    out["frac_of_spec"] = round(gbs / HBM_PEAK_GBS, 4)
    out["batch_kernel"] = ("sg::k_batch_persistent (one launch per run, rounds ordered by per-lattice counters)"
                           if persistent else "sg::k_fused_batch (one launch per round)")
    be.close()
    torch.cuda.empty_cache()
    return out


# ---------------------------------------------------------------------------
# CPU baseline: the oracle as it stands, on the host's cores
# ---------------------------------------------------------------------------
def cpu_baseline(wl_name: str = "c2", nsweeps: int = 1, threads: int = 0):
    """The oracle on bit-planes 0 and 63 of the workload's lattice (MINSTD, the
    shared numbers of the coded samples), threaded over the host's cores, timed
    for nsweeps sweeps; plus the L=16 one-sample configuration (1000 sweeps) on
    one core and on all cores."""
    import numpy as np

    import oracle
    import seeded_inputs as si

    wl = WORKLOADS[wl_name]
    threads = threads or host_threads()
    L, beta = wl["L"], wl["beta"]
    planes = [0, 63]
    J = si.coupling_bits(L, 1, planes, threads=threads)
    S0 = si.spin_bits(L, 2, 0, planes, threads=threads)
    seeds = si.minstd_seeds_threaded(L, 2, 0, threads=threads)
    lat = oracle.OracleLattice.from_bits((L, L, L), J, S0, oracle.MINSTD, seeds)
    del J, S0, seeds
    t0 = time.perf_counter()
    lat.run(nsweeps, beta, threads=threads)
    dt = time.perf_counter() - t0
    flips = len(planes) * L**3 * nsweeps
    del lat
    rec = dict(value=dt * 1e12 / flips, unit="ps/flip", cores=threads, kind="oracle",
               sample=f"{wl_name} lattice (L={L}, T={1 / beta:.2f}, MINSTD), bit-planes 0 and 63 of the 64 coded "
                      f"samples, {nsweeps} sweep(s), one byte per spin, {threads} threads over sites "
                      f"({dt:.1f} s wall)",
               cpu_model=cpu_model(), nproc=os.cpu_count())
    # the L=16 single-sample configuration in full, on one core and on all
    w0 = WORKLOADS["c0"]
    c0 = {}
    for n in (1, threads):
        L0 = w0["L"]
        l0 = oracle.OracleLattice((L0, L0, L0), 1, si.coupling_words(L0, 1) & np.uint64(1),
                                  si.spin_words(L0, 2, 0) & np.uint64(1), oracle.MINSTD, si.minstd_seeds(L0, 2, 0))
        t0 = time.perf_counter()
        l0.run(w0["sweeps"], w0["beta"], record=True, threads=n)  # energy after every sweep
        d = time.perf_counter() - t0
        c0[f"threads_{n}"] = {"ps_per_flip": d * 1e12 / (L0**3 * w0["sweeps"]), "seconds": round(d, 3)}
    rec["c0_L16_1000_sweeps"] = c0
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--sweeps", type=int, default=0, help="sweeps per step (default: the workload's)")
    ap.add_argument("--prng", default="", choices=["", "minstd", "mt19937", "parisi_rapuano", "philox"],
                    help="generator of the main run (default: the workload's)")
    ap.add_argument("--kernel", default="auto", choices=["auto", "fused", "fused2", "twopass"])
    ap.add_argument("--tile", default="",
                    help="kernel and tile [fused|fused2,]tile_x,tile_y,z_chunk,band[,planes] (skips the autotuner)")
    ap.add_argument("--extras", default="peak,depth1,c1,c3,c4,cpu",
                    help="comma list of extra sections: peak, depth1, c1, c3, c4, cpu ('' for none)")
    ap.add_argument("--cpu-sweeps", type=int, default=1, help="sweeps of the oracle in cpu_baseline")
    ap.add_argument("--sweep-scale", type=float, default=0.1, help="c3: sweep counts x this (c4: x this / 2)")
    ap.add_argument("--jobs", type=int, default=0, help="c3/c4: number of jobs (default 256 / 64)")
    ap.add_argument("--seed", type=int, default=1, help="c3/c4: trace seed")
    ap.add_argument("--group-gib", type=float, default=-1,
                    help="batched and served mixes: GiB of lattices per persistent launch (0: all; default: the "
                         "library's)")
    ap.add_argument("--persistent", type=int, default=1,
                    help="c3/c4: 1 = one persistent launch per run, 0 = one launch per round")
    ap.add_argument("--scan", default="",
                    help="also time one MINSTD lattice (64 samples, autotuned) at each of these comma-separated sides")
    ap.add_argument("--layout-ab", action="store_true",
                    help="also time the two-pass kernel on the cube, colour-separated and sliced layouts")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="also make 3 device copies of BYTES bytes, for counter calibration")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only; --gpus {args.gpus} is not supported "
              "(independent lattices and replicas would shard by job placement, one GPU each).",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1411_0127_amd import sg

    extras = {e.strip() for e in args.extras.split(",") if e.strip()}
    wl = dict(WORKLOADS[args.workload])
    if args.prng and args.prng != wl["prng"]:
        wl["prng"] = args.prng
        wl["desc"] = wl["desc"].replace("MINSTD per-site streams", f"{args.prng} numbers")
    torch.cuda.set_device(0)
    marker = Marker(torch, sg, torch.cuda.current_stream())
    main_res = run_single(args, wl, marker=marker, depth1="depth1" in extras)
    print(f"[bench] {args.workload}: {main_res['ps_per_flip']:.5f} ps/flip, launch {main_res['launch_ms']:.4f} ms",
          file=sys.stderr, flush=True)
    L, R = wl["L"], wl["replicas"]
    V = L**3
    bps = algorithmic_bytes_per_site(wl["prng"], R, main_res["sweeps_per_launch"])
    achieved = bps * V / (main_res["launch_ms"] * 1e-3) / 1e9
    # counters are taken with the workload's own generator
    main_kind = "fused2" if main_res["sweeps_per_launch"] == 2 else main_res["kind"]
    traffic = (load_traffic(args.workload, main_kind, main_res["tile"])
               if wl["prng"] == WORKLOADS[args.workload]["prng"] else None)
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
        "ms_per_sweep": round(sum(main_res["sweep_ms_per_step"]) / (args.steps * (args.sweeps or wl["sweeps"])), 5),
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "kernel": kernel_label(main_res["kind"], main_res["sweeps_per_launch"]),
            "bytes_per_site": bps,
            "sites_per_launch": V,
            "sweeps_per_launch": main_res["sweeps_per_launch"],
            "launch_ms": round(main_res["launch_ms"], 5),
            "launches_timed": args.steps * main_res["launches_per_step"],
        },
    }
    if traffic:
        line["roofline"]["traffic_gbs"] = round(traffic / (main_res["launch_ms"] * 1e-3) / 1e9, 1)
    insts = (load_valu(args.workload, main_kind, main_res["tile"])
             if wl["prng"] == WORKLOADS[args.workload]["prng"] else None)
    if insts:
        line["alu_roofline"] = alu_roofline(insts, main_res["launch_ms"])
    if "depth1" in main_res:
        line["depth1"] = main_res["depth1"]
        t1 = load_traffic(f"{args.workload}_depth1", "fused", line["depth1"]["tile"])
        if t1 and wl["prng"] == WORKLOADS[args.workload]["prng"]:
            g1 = t1 / (line["depth1"]["ms_per_sweep"] * 1e-3) / 1e9
            line["depth1"].update(traffic=t1, traffic_gbs=round(g1, 1), traffic_frac_of_spec=round(g1 / HBM_PEAK_GBS, 4))
    if "peak" in extras:
        pk = measure_peaks()
        line["measured_peak"] = pk
        line["roofline"]["frac_of_measured_read"] = round(achieved / pk["read_gbs"], 4)
        if "depth1" in line:
            line["depth1"]["frac_of_measured_copy"] = round(line["depth1"]["alg_gbs"] / pk["copy_gbs"], 4)
            line["depth1"]["frac_of_measured_read"] = round(line["depth1"]["alg_gbs"] / pk["read_gbs"], 4)
        print(f"[bench] peaks: {pk}", file=sys.stderr, flush=True)
    if args.layout_ab:
        line["layout_ab"] = layout_ab(sg, torch, wl)
    if args.scan:
        line["scan"] = scan_sides(sg, torch, [int(v) for v in args.scan.split(",")])
    if "c1" in extras and args.workload != "c1":
        c1 = {}
        for prng in ("minstd", "mt19937", "parisi_rapuano", "philox"):
            r = run_single(args, WORKLOADS["c1"], prng=prng, steps=3, warmup=1)
            c1[prng] = {"ps_per_flip": round(r["ps_per_flip"], 6), "launch_ms": round(r["launch_ms"], 5),
                        "sweeps_per_launch": r["sweeps_per_launch"], "tile": r["tile"]}
            if prng == "minstd":
                b1 = algorithmic_bytes_per_site("minstd", 2, r["sweeps_per_launch"])
                c1[prng]["alg_gbs_per_launch"] = round(b1 * 256**3 / (r["launch_ms"] * 1e-3) / 1e9, 1)
                k1 = "fused2" if r["sweeps_per_launch"] == 2 else r["kind"]
                insts = load_valu("c1", k1, r["tile"])
                if insts:
                    c1[prng]["alu_roofline"] = alu_roofline(insts, r["launch_ms"])
        line["c1"] = {"workload": WORKLOADS["c1"]["desc"], **c1}
        print(f"[bench] c1 done", file=sys.stderr, flush=True)
    for kind in ("c3", "c4"):
        if kind in extras:
            scale = args.sweep_scale if kind == "c3" else args.sweep_scale / 2
            line[kind] = run_mix(kind, args.jobs, scale, args.seed, persistent=bool(args.persistent),
                                 group_bytes=None if args.group_gib < 0 else int(args.group_gib * (1 << 30)))
            print(f"[bench] {kind} done", file=sys.stderr, flush=True)
    if args.calibrate_copy:
        src = torch.empty(args.calibrate_copy, dtype=torch.uint8, device="cuda:0").fill_(1)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if "cpu" in extras:
        line["cpu_baseline"] = cpu_baseline("c2" if args.workload == "c2" else args.workload, args.cpu_sweeps)
    print(json.dumps(line), flush=True)


def scan_sides(sg, torch, sides, beta=1 / 0.9):
    """ms per sweep and psFlip of one MINSTD lattice of 64 samples at each side,
    autotuned, HIP events around one call (200 sweeps up to L=256, 20 above)."""
    stream = torch.cuda.current_stream()
    out = []
    for L in sides:
        lat = sg.Lattice(L, 64, "minstd", coupling_seed=1, spin_seed=2, stream=stream)
        if L >= 32:
            sg.autotune([lat], reps=3)
        nsw = 200 if L <= 256 else 20
        lat.sweep(4, beta)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        lat.sweep(nsw, beta)
        b.record(stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / nsw
        out.append({"L": L, "kernel": list(lat.kernel()), "ms_per_sweep": round(ms, 5),
                    "ps_per_flip": round(ms * 1e9 / (64 * L**3), 5)})
        lat.close()
        torch.cuda.empty_cache()
        print(f"[bench] scan L={L}: {ms:.4f} ms per sweep", file=sys.stderr, flush=True)
    return out


def layout_ab(sg, torch, wl, nsw=4):
    """ms per sweep of the two-pass kernel on the cube, the colour-separated and
    the sliced layout (conversions excluded: the difference of nsw sweeps and
    none), and of the default fused kernel, all on the same lattice."""
    L, beta = wl["L"], wl["beta"]
    stream = torch.cuda.current_stream()
    lat = sg.Lattice(L, 64, wl["prng"], coupling_seed=1, spin_seed=2, stream=stream)
    work = torch.empty(sg.sliced_footprint(L), dtype=torch.uint8, device="cuda:0")
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

    out = {"lattice": f"L={L}, 64 samples, one replica"}
    out["twopass_cube_ms_per_sweep"] = round(timed(lambda: lat.sweep(nsw, beta)) / nsw, 4)
    for name, fn in (("separated", lat.sweep_separated), ("sliced", lat.sweep_sliced)):
        full = timed(lambda: fn(nsw, beta, work))
        conv = timed(lambda: fn(0, beta, work))
        out[f"twopass_{name}_ms_per_sweep"] = round((full - conv) / nsw, 4)
        out[f"{name}_conversion_ms"] = round(conv, 4)
    lat.set_kernel("auto")
    out["fused_default_ms_per_sweep"] = round(timed(lambda: lat.sweep(nsw, beta)) / nsw, 4)
    lat.close()
    del work
    torch.cuda.empty_cache()
    return out


if __name__ == "__main__":
    main()
