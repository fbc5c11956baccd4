"""Continuous batching of spin-glass simulation jobs on one GPU.

A job is a lattice (side L, 64 coded samples, couplings and spins from its own
seeds) to be swept n times at inverse temperature beta, then its energies read
back.  The server admits jobs in arrival order when their lattice fits in an HBM
budget, keeps every admitted lattice and its random streams resident, and
advances all of them together: one launch per round sweeps every active lattice
(``sg.Batch``).  Jobs join and leave at round boundaries, so work that arrives
while others run overlaps with them on the device.  Each job's result is the
same as running it alone, since every lattice uses its own keyed streams.

The scheduling logic is written against a small backend interface; ``GpuBackend``
drives libsg, ``SimBackend`` models the device with a cost per site-sweep on a
virtual clock so admission, budgets and latency accounting can be tested on the
CPU.

Workload generators follow the two mixes this engine is measured on: a batch of
lattices all present at time 0 (sides from {32,...,512}, T in [0.5, 1.5], 100 to
2000 sweeps) and a Poisson stream of jobs (sides from {64,...,512}, T in
[0.6, 1.4], sweeps log-uniform in 10^2 .. 10^4).
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import Dict, List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Job:
    jid: int
    L: int
    nsweeps: int
    beta: float
    coupling_seed: int
    spin_seed: int
    arrival: float = 0.0

    @property
    def flips(self) -> int:
        return 64 * self.L**3 * self.nsweeps


def trace_batch(n: int, seed: int, sizes=(32, 64, 128, 256, 512), temps=(0.5, 1.5), sweeps=(100, 2000),
                sweep_scale: float = 1.0) -> List[Job]:
    """n jobs present at time 0: L uniform over sizes, T uniform, sweeps uniform."""
    rng = np.random.default_rng(seed)
    jobs = []
    for k in range(n):
        L = int(rng.choice(sizes))
        T = float(rng.uniform(*temps))
        ns = max(1, int(round(int(rng.integers(sweeps[0], sweeps[1] + 1)) * sweep_scale)))
        jobs.append(Job(k, L, ns, 1.0 / T, 1000 + 2 * k, 1001 + 2 * k, 0.0))
    return jobs


def trace_served(n: int, rate: float, seed: int, sizes=(64, 128, 256, 512), temps=(0.6, 1.4),
                 log_sweeps=(2.0, 4.0), sweep_scale: float = 1.0) -> List[Job]:
    """n jobs with Poisson arrivals at `rate` per second: L uniform over sizes,
    T uniform, sweeps = 10^U(log_sweeps)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    jobs = []
    for k in range(n):
        t += float(rng.exponential(1.0 / rate))
        L = int(rng.choice(sizes))
        T = float(rng.uniform(*temps))
        ns = max(1, int(round(10 ** float(rng.uniform(*log_sweeps)) * sweep_scale)))
        jobs.append(Job(k, L, ns, 1.0 / T, 5000 + 2 * k, 5001 + 2 * k, t))
    return jobs


# ---------------------------------------------------------------------------
# Backends
# ---------------------------------------------------------------------------
class GpuBackend:
    """libsg batches on one GPU; every lattice lives in its own torch buffer.  A run
    is one persistent launch (persistent=True) or one launch per round."""

    def __init__(self, device="cuda:0", max_lattices: int = 512, max_items: int = 1 << 20,
                 rounds_per_graph: int = 0, autotune: bool = True, persistent: bool = True,
                 group_bytes: Optional[int] = None):
        import torch

        from paper_1411_0127_amd import sg

        self.sg = sg
        self.torch = torch
        self.device = torch.device(device)
        self.stream = torch.cuda.Stream(self.device)
        self.batch = sg.Batch(max_lattices, max_items, self.stream, device=self.device)
        self.rounds_per_graph = rounds_per_graph
        self.autotune = autotune
        self.persistent = bool(persistent)
        self.batch.set_persistent(self.persistent)
        if group_bytes is not None:  # else the library's default
            self.batch.set_group_bytes(group_bytes)
        self._inflight = []  # events of queued runs; at most two are kept in flight
        self._tuned = set()

    def footprint(self, job: Job) -> int:
        return self.sg.footprint(job.L, "minstd", True)

    def now(self) -> float:
        return time.perf_counter()

    def wait(self, dt: float):
        if dt > 0:
            time.sleep(min(dt, 0.05))

    def pretune(self, sizes):
        """Autotune the fused tile for each side once (cached in the library)."""
        for L in sorted(set(sizes)):
            if L >= 64 and L not in self._tuned:
                lat = self.sg.Lattice(L, 64, "minstd", device=self.device, stream=self.stream)
                self.sg.autotune([lat], reps=3)
                self._tuned.add(L)
                lat.close()
        self.torch.cuda.synchronize()

    def start(self, job: Job):
        lat = self.sg.Lattice(job.L, 64, "minstd", coupling_seed=job.coupling_seed, spin_seed=job.spin_seed,
                              device=self.device, stream=self.stream)
        if self.autotune and job.L not in self._tuned and job.L >= 64:
            self.sg.autotune([lat], reps=3)  # cached per L inside the library
            self._tuned.add(job.L)
        elif self.autotune and job.L in self._tuned:
            self.sg.autotune([lat], reps=3)  # cache hit: sets the tuned tile
        self.batch.add(lat, job.nsweeps, job.beta)
        return lat

    def rounds_to_first_finish(self) -> int:
        return self.batch.rounds_left()[0]

    def run(self, rounds: int) -> int:
        done = self.batch.run(rounds, self.rounds_per_graph)
        ev = self.torch.cuda.Event()
        ev.record(self.stream)
        self._inflight.append(ev)
        while len(self._inflight) > 2:
            self._inflight.pop(0).synchronize()
        return done

    def finished(self):
        return self.batch.take_finished()

    def result(self, lat):
        self.batch.check()  # synchronises the stream; raises if a persistent run gave up
        U, e = lat.energy()
        return {"unsat": U, "e": e}

    def release(self, lat):
        lat.close()
        del lat

    def close(self):
        self.torch.cuda.synchronize()
        self.batch.close()


class SimBackend:
    """A model of the device: a round advances every active lattice by two sweeps
    (one for an odd last sweep), as the GPU batch does, and costs `sec_per_site` x
    (site sweeps done) + `round_overhead`, on a virtual clock."""

    def __init__(self, sec_per_site: float = 1.0e-11, round_overhead: float = 20e-6):
        self.t = 0.0
        self.sec_per_site = sec_per_site
        self.round_overhead = round_overhead
        self.active: Dict[int, List] = {}
        self._done: List = []
        self._next = 0

    def footprint(self, job: Job) -> int:
        return 44 * job.L**3 + (1 << 20)

    def now(self) -> float:
        return self.t

    def wait(self, dt: float):
        self.t += max(dt, 1e-9)

    def start(self, job: Job):
        h = self._next
        self._next += 1
        self.active[h] = [job, job.nsweeps]
        return h

    def rounds_to_first_finish(self) -> int:
        return min((v[1] + 1) // 2 for v in self.active.values()) if self.active else 0

    def run(self, rounds: int) -> int:
        if not self.active:
            return 0
        R = min(rounds, max((v[1] + 1) // 2 for v in self.active.values()))
        for _ in range(R):
            site_sweeps = sum(v[0].L**3 * min(2, v[1]) for v in self.active.values() if v[1] > 0)
            self.t += self.round_overhead + site_sweeps * self.sec_per_site
            for h, v in list(self.active.items()):
                if v[1] > 0:
                    v[1] -= min(2, v[1])
                    if v[1] == 0:
                        self._done.append(h)
        return R

    def finished(self):
        out, self._done = self._done, []
        for h in out:
            self.active.pop(h)
        return out

    def result(self, h):
        return {}

    def release(self, h):
        pass


# ---------------------------------------------------------------------------
# Server
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class Record:
    job: Job
    admitted: float
    finished: float
    result: dict

    @property
    def latency(self) -> float:
        return self.finished - self.job.arrival

    @property
    def wait(self) -> float:
        return self.admitted - self.job.arrival


@dataclasses.dataclass
class Report:
    records: List[Record]
    rejected: List[Job]
    makespan: float
    idle: float
    peak_bytes: int
    rounds: int
    runs: int

    def latency_percentile(self, q: float) -> float:
        lat = sorted(r.latency for r in self.records)
        if not lat:
            return float("nan")
        k = min(len(lat) - 1, max(0, int(math.ceil(q / 100.0 * len(lat))) - 1))
        return lat[k]

    @property
    def flips(self) -> int:
        return sum(r.job.flips for r in self.records)

    @property
    def busy(self) -> float:
        return self.makespan - self.idle

    def summary(self) -> dict:
        return {
            "jobs": len(self.records),
            "rejected": len(self.rejected),
            "p50_latency_s": self.latency_percentile(50),
            "p99_latency_s": self.latency_percentile(99),
            "makespan_s": self.makespan,
            "busy_s": self.busy,
            "flips": self.flips,
            "ps_per_flip_makespan": self.makespan * 1e12 / max(1, self.flips),
            "ps_per_flip_busy": self.busy * 1e12 / max(1, self.flips),
            "peak_hbm_bytes": self.peak_bytes,
            "rounds": self.rounds,
            "runs": self.runs,
        }


class Server:
    """FIFO admission under an HBM budget, continuous batching of admitted jobs.

    chunk_rounds bounds the rounds queued per run, so arrivals wait at most one
    chunk to be admitted; a run also stops when the first active job finishes (but
    lasts at least min_rounds), so finished jobs are read back and their memory
    freed promptly.  A round is one launch over all active lattices (two sweeps
    each on the GPU's two-sweep march)."""

    def __init__(self, backend, budget_bytes: int, chunk_rounds: int = 50, min_rounds: int = 1):
        self.b = backend
        self.budget = int(budget_bytes)
        self.chunk = int(chunk_rounds)
        self.min_rounds = max(1, int(min_rounds))

    def serve(self, jobs: Sequence[Job], on_finish=None) -> Report:
        queue = sorted(jobs, key=lambda j: (j.arrival, j.jid))
        live = {}  # handle -> (job, admitted time, bytes)
        records: List[Record] = []
        rejected: List[Job] = []
        used = peak = 0
        rounds = runs = 0
        idle = 0.0
        t0 = self.b.now()
        while queue or live:
            now = self.b.now() - t0
            while queue and queue[0].arrival <= now:
                job = queue[0]
                need = self.b.footprint(job)
                if need > self.budget:
                    rejected.append(queue.pop(0))
                    continue
                if used + need > self.budget:
                    break  # head of line waits for memory
                queue.pop(0)
                h = self.b.start(job)
                used += need
                peak = max(peak, used)
                live[h] = (job, self.b.now() - t0, need)
            if not live:
                if queue:
                    w0 = self.b.now()
                    self.b.wait(queue[0].arrival - (w0 - t0))
                    if records or rejected:  # idle time inside the served span
                        idle += self.b.now() - w0
                continue
            r = min(self.chunk, max(self.min_rounds, self.b.rounds_to_first_finish()))
            rounds += self.b.run(r)
            runs += 1
            for h in self.b.finished():
                job, adm, need = live.pop(h)
                res = self.b.result(h)
                fin = self.b.now() - t0
                rec = Record(job, adm, fin, res)
                records.append(rec)
                if on_finish is not None:
                    on_finish(rec, h)
                self.b.release(h)
                used -= need
        makespan = max((r.finished for r in records), default=0.0) - min((j.arrival for j in jobs), default=0.0)
        return Report(records, rejected, makespan, idle, peak, rounds, runs)
