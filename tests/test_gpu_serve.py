"""The continuous-batching server on the GPU: jobs that arrive while others run
join the same launches, and every job's final spins equal the job run alone."""
import sys

import numpy as np
import pytest

from paper_1411_0127_amd.serve import Job, Server

pytestmark = pytest.mark.gpu


def test_served_results_equal_solo_runs():
    import torch

    from paper_1411_0127_amd import sg
    from paper_1411_0127_amd.serve import GpuBackend

    print("[case] serve small trace", flush=True)
    sys.stdout.flush()
    rng = np.random.default_rng(11)
    # a long first job (about a thousand rounds) that the later arrivals overlap
    jobs = [Job(0, 32, 2001, 1 / 0.9, 700, 800, 0.0)]
    t = 0.0
    for k in range(1, 14):
        t += float(rng.exponential(0.002))
        L = int(rng.choice([8, 16, 24, 32]))
        jobs.append(Job(k, L, int(rng.integers(3, 60)), float(1 / rng.uniform(0.6, 1.4)), 700 + k, 800 + k, t))
    be = GpuBackend(max_lattices=16, max_items=100000, rounds_per_graph=2, autotune=False)
    budget = 3 * sg.footprint(32)
    words = {}

    def keep(rec, lat):
        words[rec.job.jid] = lat.words()

    rep = Server(be, budget, chunk_rounds=4).serve(jobs, on_finish=keep)
    assert len(rep.records) == len(jobs) and not rep.rejected
    assert rep.peak_bytes <= budget
    recs = sorted(rep.records, key=lambda r: r.admitted)
    overlap = any(b.admitted < a.finished for a, b in zip(recs, recs[1:]))
    assert overlap, "no job was admitted while another was running"
    stream = torch.cuda.Stream(torch.device("cuda:0"))
    for j in jobs:
        solo = sg.Lattice(j.L, 64, "minstd", coupling_seed=j.coupling_seed, spin_seed=j.spin_seed, stream=stream)
        solo.sweep(j.nsweeps, j.beta)
        assert np.array_equal(words[j.jid], solo.words()), f"job {j.jid} L={j.L}"
        solo.close()
