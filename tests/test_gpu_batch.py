"""Batched sweeps (sg_batch_*): every lattice of a mixed batch must end bit-identical
to the same lattice swept alone, and small ones to the oracle; graph replays are
checked one by one against eager runs.  Both forms of a run are covered: one
persistent launch per run (the default) and one launch per round."""
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


MODES = ["persistent", "per_round"]


def make_batch(sg, stream, mode, max_lat=16, max_items=100000):
    b = sg.Batch(max_lat, max_items, stream)
    b.set_persistent(mode == "persistent")
    return b


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("graph", [0, 2, 3])
def test_batch_matches_solo_and_oracle(env, graph, mode):
    sg, stream = env
    say("batch", graph, mode)
    b = make_batch(sg, stream, mode)
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
    b.check()
    fin = b.take_finished()
    assert sorted(id(x) for x in fin) == sorted(id(x) for x in lats)
    for lat, (L, cs, ss, beta, n) in zip(lats, JOBS):
        assert lat.t == n
        w = lat.words()
        assert np.array_equal(w, solo_words(sg, stream, L, cs, ss, beta, n)), f"L={L} vs solo"
        if L <= 24:
            assert np.array_equal(w, oracle_words(L, cs, ss, beta, n)), f"L={L} vs oracle"
    b.close()


@pytest.mark.parametrize("mode", MODES)
def test_batch_small_sides_and_kernel_choices(env, mode):
    """Sides below the two-sweep march's minimum take one-sweep rounds; a lattice set
    to the two-pass kernel (which a batch has no form of) takes the default march, one
    set to the one-sweep kernel one-sweep rounds.  Every result matches the oracle."""
    sg, stream = env
    say("batch small sides and kernels", mode)
    specs = [  # L, coupling seed, spin seed, beta, sweeps, kernel
        (2, 41, 42, 0.7, 5, "auto"), (4, 43, 44, 0.9, 4, "auto"), (6, 45, 46, 1.1, 3, "auto"),
        (16, 47, 48, 0.8, 5, "twopass"), (16, 49, 50, 0.8, 4, "fused"), (10, 51, 52, 1.3, 6, "fused2"),
    ]
    b = make_batch(sg, stream, mode)
    lats = []
    for (L, cs, ss, beta, n, kind) in specs:
        lat = sg.Lattice(L, 64, "minstd", coupling_seed=cs, spin_seed=ss, stream=stream)
        lat.set_kernel(kind)
        b.add(lat, n, beta)
        lats.append(lat)
    b.run(1000, 2)
    assert b.rounds_left() == (0, 0)
    b.check()
    for lat, (L, cs, ss, beta, n, kind) in zip(lats, specs):
        assert lat.t == n
        assert np.array_equal(lat.words(), oracle_words(L, cs, ss, beta, n)), f"L={L} {kind}"
    b.close()


@pytest.mark.parametrize("mode", MODES)
def test_batch_join_leave_in_chunks(env, mode):
    sg, stream = env
    say("batch join/leave", mode)
    b = make_batch(sg, stream, mode)
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


@pytest.mark.parametrize("mode", MODES)
def test_graph_replays_one_by_one(env, mode):
    sg, stream = env
    say("graph replays", mode)
    b = make_batch(sg, stream, mode, max_lat=4)
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
    b.check()
    b.close()


GROUP_JOBS = [(8, 11, 12, 0.5, 71), (16, 13, 14, 0.8, 100), (24, 15, 16, 1.2, 66), (32, 17, 18, 1.5, 90),
              (48, 19, 20, 2.0, 64), (16, 21, 22, 1 / 0.7, 129)]


@pytest.mark.parametrize("graph", [0, 2])
@pytest.mark.parametrize("cap_sites", [1, 20000, 60000])
def test_grouped_persistent_runs(env, graph, cap_sites):
    """Persistent runs of 4 rounds or more launch the lattices in groups of bounded
    memory, one after another: a cap of one site puts each lattice in a group of its
    own, the others form groups of several.  A short first run stays one launch;
    every lattice must equal the same lattice swept alone, and L = 8 and 16 the
    oracle."""
    sg, stream = env
    say("grouped persistent", graph, cap_sites)
    b = make_batch(sg, stream, "persistent")
    b.set_group_bytes(40 * cap_sites)
    lats = []
    for (L, cs, ss, beta, n) in GROUP_JOBS:
        lat = sg.Lattice(L, 64, "minstd", coupling_seed=cs, spin_seed=ss, stream=stream)
        b.add(lat, n, beta)
        lats.append(lat)
    # runs of 32 rounds (grouped launches while at least 4 are left), after a short
    # first run (one launch)
    b.run(2, graph)
    runs = 1
    while b.rounds_left()[1] > 0:
        b.run(32, graph)
        runs += 1
    assert runs >= 2
    b.check()
    done = b.take_finished()
    assert len(done) == len(GROUP_JOBS)
    for lat, (L, cs, ss, beta, n) in zip(lats, GROUP_JOBS):
        assert lat.t == n
        w = lat.words()
        assert np.array_equal(w, solo_words(sg, stream, L, cs, ss, beta, n)), f"L={L} vs solo"
        if L <= 16:
            assert np.array_equal(w, oracle_words(L, cs, ss, beta, n)), f"L={L} vs oracle"
        lat.close()
    b.close()


@pytest.mark.parametrize("mode", MODES)
def test_large_sides_with_tuned_tiles(env, mode):
    """One lattice each of L = 64, 128, 256, 512 and 544 with the autotuned tiles the
    benchmark uses (pretuned as the server does), odd sweep counts, and runs replayed
    from a graph at least twice: whole columns of the two-sweep march up to L = 512,
    two z chunks of it at L = 544, four of the one-sweep march for a lattice set to
    it at L = 256.  Each lattice must equal the same lattice swept alone, L = 64
    also the oracle."""
    sg, stream = env
    from paper_1411_0127_amd.serve import GpuBackend

    say("batch large sides", mode)
    be = GpuBackend(max_lattices=8, max_items=200000, rounds_per_graph=2, persistent=(mode == "persistent"))
    be.pretune([64, 128, 256, 512, 544])
    specs = [  # L, coupling seed, spin seed, beta, sweeps, kernel
        (64, 61, 62, 0.9, 7, None), (128, 63, 64, 1.1, 5, None), (256, 65, 66, 0.7, 9, None),
        (512, 67, 68, 1.3, 5, None), (256, 69, 70, 1.0, 5, "fused"), (544, 71, 72, 0.8, 3, None),
    ]
    b = make_batch(sg, be.stream, mode, max_lat=8, max_items=200000)
    lats = []
    for (L, cs, ss, beta, n, kind) in specs:
        lat = sg.Lattice(L, 64, "minstd", coupling_seed=cs, spin_seed=ss, stream=be.stream)
        if kind is None:
            sg.autotune([lat], reps=3)  # cache hit: the pretuned shape
        else:
            lat.set_kernel(kind)
        b.add(lat, n, beta)
        lats.append(lat)
    runs = 0
    while b.rounds_left()[1] > 0:
        b.run(2, 2)  # two-round runs: the graph of a run shape is replayed
        runs += 1
    assert runs >= 3
    b.check()
    for lat, (L, cs, ss, beta, n, kind) in zip(lats, specs):
        assert lat.t == n
        w = lat.words()
        solo = sg.Lattice(L, 64, "minstd", coupling_seed=cs, spin_seed=ss, stream=be.stream)
        if kind is None:
            sg.autotune([solo], reps=3)
        solo.sweep(n, beta)
        assert np.array_equal(w, solo.words()), f"L={L} {kind} vs solo"
        solo.close()
        if L == 64:
            assert np.array_equal(w, oracle_words(L, cs, ss, beta, n)), "L=64 vs oracle"
        lat.close()
    b.close()
    be.close()


def test_persistent_wait_limit_is_reported(env):
    """A spin limit of one poll, forced from the host, makes a persistent run give
    up at its first wait for a previous round: every workgroup leaves, the kernel
    ends normally and sg_batch_check reports the failure."""
    sg, stream = env
    say("persistent wait limit")
    b = make_batch(sg, stream, "persistent", max_lat=2)
    b.set_persistent(True, spin_cap=1)
    lat = sg.Lattice(16, 64, "minstd", coupling_seed=3, spin_seed=4, stream=stream)
    b.add(lat, 40, 1.0)  # twenty rounds of one work item each, every one waiting for the last
    b.run(100, 0)
    with pytest.raises(sg.SGError) as e:
        b.check()
    assert e.value.code == sg.SG_EDEVICE
    # the batch keeps working with the default limit
    b.set_persistent(True)
    lat2 = sg.Lattice(16, 64, "minstd", coupling_seed=5, spin_seed=6, stream=stream)
    b.add(lat2, 6, 1.0)
    b.run(100, 0)
    b.check()
    assert np.array_equal(lat2.words(), oracle_words(16, 5, 6, 1.0, 6))
    b.close()


def test_batch_argument_checks(env):
    sg, stream = env
    b = sg.Batch(1, 1000, stream)
    with pytest.raises(sg.SGError):
        sg._check(sg.lib.sg_batch_set_persistent(b.handle, 2, 0))
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


def test_error_flag_starts_cleared_on_a_dirty_buffer(env):
    """A batch built on a caller buffer full of ones reports no error after runs
    of the per-round form, which never touch the flag: creation clears it."""
    import ctypes

    import torch

    sg, stream = env
    say("batch error flag on a dirty buffer")
    n = ctypes.c_size_t()
    sg._check(sg.lib.sg_batch_footprint(4, 1000, ctypes.byref(n)))
    with torch.cuda.stream(stream):
        buf = torch.full((int(n.value),), 0xFF, dtype=torch.uint8, device="cuda:0")
    h = ctypes.c_void_p()
    sg._check(sg.lib.sg_batch_create(4, 1000, ctypes.c_void_p(buf.data_ptr()), int(n.value),
                                     ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)))
    try:
        sg._check(sg.lib.sg_batch_set_persistent(h, 0, 0))
        lat = sg.Lattice(16, 64, "minstd", coupling_seed=7, spin_seed=8, stream=stream)
        sg._check(sg.lib.sg_batch_add(h, lat.handle, 4, ctypes.c_double(1.0)))
        done = ctypes.c_int64()
        sg._check(sg.lib.sg_batch_run(h, 100, 0, ctypes.byref(done)))
        sg._check(sg.lib.sg_batch_check(h))
        assert np.array_equal(lat.words(), oracle_words(16, 7, 8, 1.0, 4))
        lat.close()
    finally:
        sg.lib.sg_batch_destroy(h)
        torch.cuda.synchronize()
        del buf
