"""The continuous-batching server on the GPU: jobs that arrive while others run
join the same launches, and every job's final spins equal the job run alone and
the oracle's."""
import sys

import numpy as np
import pytest

import oracle
import seeded_inputs as si
from paper_1411_0127_amd.serve import Job, Server

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("persistent", [True, False])
def test_served_results_equal_solo_runs(persistent):
    import torch

    from paper_1411_0127_amd import sg
    from paper_1411_0127_amd.serve import GpuBackend

    print("[case] serve small trace", persistent, flush=True)
    sys.stdout.flush()
    rng = np.random.default_rng(11)
    # a long first job (about a thousand rounds) that the later arrivals overlap
    jobs = [Job(0, 32, 2001, 1 / 0.9, 700, 800, 0.0)]
    t = 0.0
    for k in range(1, 14):
        t += float(rng.exponential(0.002))
        L = int(rng.choice([8, 16, 24, 32]))
        jobs.append(Job(k, L, int(rng.integers(3, 60)), float(1 / rng.uniform(0.6, 1.4)), 700 + k, 800 + k, t))
    be = GpuBackend(max_lattices=16, max_items=100000, rounds_per_graph=2, autotune=False, persistent=persistent)
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
        if j.L <= 16 or j.jid % 4 == 1:  # the oracle on a share of the jobs (all small ones)
            ref = oracle.OracleLattice((j.L,) * 3, 64, si.coupling_words(j.L, j.coupling_seed),
                                       si.spin_words(j.L, j.spin_seed, 0), oracle.MINSTD,
                                       si.minstd_seeds(j.L, j.spin_seed, 0))
            ref.run(j.nsweeps, j.beta)
            assert np.array_equal(words[j.jid], ref.words()), f"job {j.jid} L={j.L} vs oracle"
    be.close()


def test_served_tuned_sides_match_the_oracle():
    """Served jobs of L = 64 and 128 with autotuned tiles (the benchmark's setting),
    each against the oracle."""
    from paper_1411_0127_amd import sg
    from paper_1411_0127_amd.serve import GpuBackend

    print("[case] serve tuned sides", flush=True)
    jobs = [Job(0, 128, 9, 1 / 1.2, 901, 902, 0.0), Job(1, 64, 13, 1 / 0.8, 903, 904, 0.001),
            Job(2, 64, 4, 1 / 1.0, 905, 906, 0.002)]
    be = GpuBackend(max_lattices=8, max_items=200000, rounds_per_graph=2, autotune=True)
    be.pretune([64, 128])
    words = {}
    rep = Server(be, 4 * sg.footprint(128), chunk_rounds=3).serve(jobs, on_finish=lambda r, lat: words.update(
        {r.job.jid: lat.words()}))
    assert len(rep.records) == 3
    for j in jobs:
        ref = oracle.OracleLattice((j.L,) * 3, 64, si.coupling_words(j.L, j.coupling_seed),
                                   si.spin_words(j.L, j.spin_seed, 0), oracle.MINSTD, si.minstd_seeds(j.L, j.spin_seed, 0))
        ref.run(j.nsweeps, j.beta, threads=8)
        assert np.array_equal(words[j.jid], ref.words()), f"job {j.jid} L={j.L} vs oracle"
    be.close()
