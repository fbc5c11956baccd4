"""Scheduling logic of the continuous-batching server, on the simulated backend
(CPU): budgets, admission order, overlap, latency accounting."""
import pytest

from paper_1411_0127_amd.serve import Job, Server, SimBackend, trace_batch, trace_served


def test_all_jobs_finish_within_budget():
    jobs = trace_served(60, rate=50.0, seed=3, sweep_scale=0.05)
    be = SimBackend(sec_per_site=1e-11)
    budget = 3 * be.footprint(Job(0, 512, 1, 1.0, 0, 0))
    rep = Server(be, budget, chunk_rounds=20).serve(jobs)
    assert len(rep.records) == 60 and not rep.rejected
    assert rep.peak_bytes <= budget
    for r in rep.records:
        assert r.admitted >= r.job.arrival - 1e-12
        assert r.finished > r.admitted
    assert rep.latency_percentile(50) <= rep.latency_percentile(99)
    s = rep.summary()
    assert s["flips"] == sum(j.flips for j in jobs)
    assert s["busy_s"] <= s["makespan_s"] + 1e-12


def test_fifo_admission_and_head_of_line():
    be = SimBackend()
    fp = be.footprint(Job(0, 64, 1, 1.0, 0, 0))
    jobs = [Job(0, 64, 100, 1.0, 0, 0, 0.0), Job(1, 64, 5, 1.0, 0, 0, 0.0), Job(2, 64, 5, 1.0, 0, 0, 0.0)]
    rep = Server(be, budget_bytes=2 * fp, chunk_rounds=1000).serve(jobs)
    rec = {r.job.jid: r for r in rep.records}
    # two fit at once: 0 and 1 start together, 2 starts when 1 leaves
    assert rec[0].admitted == rec[1].admitted == 0.0
    assert rec[2].admitted >= rec[1].finished - 1e-12
    assert rep.peak_bytes == 2 * fp


def test_oversize_jobs_are_rejected():
    be = SimBackend()
    jobs = [Job(0, 512, 10, 1.0, 0, 0, 0.0), Job(1, 32, 10, 1.0, 0, 0, 0.0)]
    rep = Server(be, budget_bytes=be.footprint(Job(0, 256, 1, 1.0, 0, 0)), chunk_rounds=10).serve(jobs)
    assert [j.jid for j in rep.rejected] == [0]
    assert [r.job.jid for r in rep.records] == [1]


def test_arrivals_overlap_running_work():
    """A job that arrives while another runs is admitted before that one ends."""
    be = SimBackend(sec_per_site=1e-9)
    jobs = [Job(0, 64, 400, 1.0, 0, 0, 0.0), Job(1, 32, 10, 1.0, 0, 0, 0.01)]
    rep = Server(be, budget_bytes=1 << 40, chunk_rounds=10).serve(jobs)
    rec = {r.job.jid: r for r in rep.records}
    assert rec[1].admitted < rec[0].finished
    assert rec[1].finished < rec[0].finished


def test_traces_are_seeded_and_follow_their_mix():
    a = trace_batch(256, seed=7)
    b = trace_batch(256, seed=7)
    assert [(j.L, j.nsweeps, j.beta) for j in a] == [(j.L, j.nsweeps, j.beta) for j in b]
    assert {j.L for j in a} <= {32, 64, 128, 256, 512}
    assert all(100 <= j.nsweeps <= 2000 and 0.5 <= 1 / j.beta <= 1.5 for j in a)
    s = trace_served(500, rate=50.0, seed=1)
    gaps = [b.arrival - a.arrival for a, b in zip(s, s[1:])]
    assert abs(sum(gaps) / len(gaps) - 1 / 50.0) < 0.004
    assert all(100 <= j.nsweeps <= 10000 for j in s)
