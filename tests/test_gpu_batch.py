"""Batched sweeps (sg_batch_*): every lattice of a mixed batch must end bit-identical
to the same lattice swept alone, and small ones to the oracle; graph replays are
checked one by one against eager runs."""
import sys

import numpy as np
import pytest

import oracle
import seeded_inputs as si

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch

    assert torch.cuda.is_available()
    from paper_1411_0127_amd import sg

    stream = torch.cuda.Stream(torch.device("cuda:0"))
    return sg, stream


JOBS = [  # L, coupling seed, spin seed, beta, sweeps
    (8, 11, 12, 0.5, 7),
    (16, 13, 14, 0.8, 12),
    (24, 15, 16, 1.2, 3),
    (32, 17, 18, 1.5, 9),
    (48, 19, 20, 2.0, 5),
    (16, 21, 22, 1 / 0.7, 1),
]


def solo_words(sg, stream, L, cs, ss, beta, n):
    lat = sg.Lattice(L, 64, "minstd", coupling_seed=cs, spin_seed=ss, stream=stream)
    lat.sweep(n, beta)
    w = lat.words()
    lat.close()
    return w


def oracle_words(L, cs, ss, beta, n):
    ref = oracle.OracleLattice((L, L, L), 64, si.coupling_words(L, cs), si.spin_words(L, ss, 0), oracle.MINSTD,
                               si.minstd_seeds(L, ss, 0))
    ref.sweep(n, beta)
    return ref.words()


@pytest.mark.parametrize("graph", [0, 2, 3])
def test_batch_matches_solo_and_oracle(env, graph):
    sg, stream = env
    say("batch", graph)
    b = sg.Batch(16, 100000, stream)
    lats = []
    for (L, cs, ss, beta, n) in JOBS:
        lat = sg.Lattice(L, 64, "minstd", coupling_seed=cs, spin_seed=ss, stream=stream)
        b.add(lat, n, beta)
        lats.append(lat)
    first, last = b.rounds_left()
    # two-sweep rounds: a lattice of n sweeps takes ceil(n / 2) of them
    assert (first, last) == (min((j[4] + 1) // 2 for j in JOBS), max((j[4] + 1) // 2 for j in JOBS))
    done = b.run(1000, graph)
    assert done == last
    assert b.rounds_left() == (0, 0)
    fin = b.take_finished()
    assert sorted(id(x) for x in fin) == sorted(id(x) for x in lats)
    for lat, (L, cs, ss, beta, n) in zip(lats, JOBS):
        assert lat.t == n
        w = lat.words()
        assert np.array_equal(w, solo_words(sg, stream, L, cs, ss, beta, n)), f"L={L} vs solo"
        if L <= 24:
            assert np.array_equal(w, oracle_words(L, cs, ss, beta, n)), f"L={L} vs oracle"
    b.close()


def test_batch_small_sides_and_kernel_choices(env):
    """Sides below the two-sweep march's minimum take one-sweep rounds; a lattice set
    to the two-pass kernel (which a batch has no form of) takes the default march, one
    set to the one-sweep kernel one-sweep rounds.  Every result matches the oracle."""
    sg, stream = env
    say("batch small sides and kernels")
    specs = [  # L, coupling seed, spin seed, beta, sweeps, kernel
        (2, 41, 42, 0.7, 5, "auto"), (4, 43, 44, 0.9, 4, "auto"), (6, 45, 46, 1.1, 3, "auto"),
        (16, 47, 48, 0.8, 5, "twopass"), (16, 49, 50, 0.8, 4, "fused"), (10, 51, 52, 1.3, 6, "fused2"),
    ]
    b = sg.Batch(16, 100000, stream)
    lats = []
    for (L, cs, ss, beta, n, kind) in specs:
        lat = sg.Lattice(L, 64, "minstd", coupling_seed=cs, spin_seed=ss, stream=stream)
        lat.set_kernel(kind)
        b.add(lat, n, beta)
        lats.append(lat)
    b.run(1000, 2)
    assert b.rounds_left() == (0, 0)
    for lat, (L, cs, ss, beta, n, kind) in zip(lats, specs):
        assert lat.t == n
        assert np.array_equal(lat.words(), oracle_words(L, cs, ss, beta, n)), f"L={L} {kind}"
    b.close()


def test_batch_join_leave_in_chunks(env):
    sg, stream = env
    say("batch join/leave")
    b = sg.Batch(16, 100000, stream)
    pending = list(JOBS)
    live = {}
    rnd = 0
    while pending or b.size()[0]:
        if pending:  # one lattice joins at every run boundary
            L, cs, ss, beta, n = pending.pop(0)
            lat = sg.Lattice(L, 64, "minstd", coupling_seed=cs, spin_seed=ss, stream=stream)
            b.add(lat, n, beta)
            live[id(lat)] = (lat, (L, cs, ss, beta, n))
        b.run(2, 2 if rnd % 2 else 0)
        rnd += 1
        for lat in b.take_finished():
            lat_, (L, cs, ss, beta, n) = live.pop(id(lat))
            assert lat.t == n
            assert np.array_equal(lat.words(), solo_words(sg, stream, L, cs, ss, beta, n)), f"L={L}"
            lat.close()
    assert not live
    b.close()


def test_graph_replays_one_by_one(env):
    sg, stream = env
    say("graph replays")
    b = sg.Batch(4, 100000, stream)
    specs = [(16, 31, 32, 0.9), (32, 33, 34, 1.1), (24, 35, 36, 0.6)]
    lats = []
    for (L, cs, ss, beta) in specs:
        lat = sg.Lattice(L, 64, "minstd", coupling_seed=cs, spin_seed=ss, stream=stream)
        b.add(lat, 24, beta)
        lats.append(lat)
    solos = [sg.Lattice(L, 64, "minstd", coupling_seed=cs, spin_seed=ss, stream=stream) for (L, cs, ss, _) in specs]
    for rep in range(6):  # six replays of the same 2-round graph, 4 sweeps each
        assert b.run(2, 2) == 2
        for lat, solo, (L, cs, ss, beta) in zip(lats, solos, specs):
            solo.sweep(4, beta)
            lat.energy()  # eager work and a synchronisation between replays
            assert np.array_equal(lat.words(), solo.words()), f"replay {rep} L={L}"
    b.close()


def test_batch_argument_checks(env):
    sg, stream = env
    b = sg.Batch(1, 1000, stream)
    lat = sg.Lattice(8, 64, "minstd", stream=stream)
    with pytest.raises(sg.SGError):
        b.add(lat, 0, 1.0)
    b.add(lat, 2, 1.0)
    with pytest.raises(sg.SGError):
        b.add(lat, 2, 1.0)  # already queued
    mt = sg.Lattice(8, 64, "mt19937", stream=stream)
    with pytest.raises(sg.SGError):
        b.add(mt, 2, 1.0)  # MINSTD only
    other = sg.Lattice(8, 64, "minstd")  # default stream
    with pytest.raises(sg.SGError):
        b.add(other, 2, 1.0)
    b.close()
