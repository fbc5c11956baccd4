"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Spins are compared bit for bit (integer work: the tolerance is zero), energies and
overlaps as exact integers.  Each test prints the case it runs before touching the
GPU, so that a failing run names it.
"""
import math
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
def sg():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1411_0127_amd import sg as mod

    return mod


PRNG = {"minstd": oracle.MINSTD, "mt19937": oracle.MT19937, "philox": oracle.PHILOX,
        "parisi_rapuano": oracle.PARISI_RAPUANO}


def stream_seeds(L, prng, sseed, r):
    if PRNG[prng] == oracle.MINSTD:
        return si.minstd_seeds(L, sseed, r)
    if PRNG[prng] == oracle.MT19937:
        return si.mt_seeds(L, sseed, r)
    if PRNG[prng] == oracle.PARISI_RAPUANO:
        return si.pr_seeds(L, sseed, r)
    return si.philox_key(sseed, r)


def oracle_for(L, S, prng, cseed, sseed, r=0, J=None, words=None):
    seeds = stream_seeds(L, prng, sseed, r)
    return oracle.OracleLattice((L, L, L), S, si.coupling_words(L, cseed) if J is None else J,
                                si.spin_words(L, sseed, r) if words is None else words, PRNG[prng], seeds)


def mask(S):
    return np.uint64((1 << S) - 1) if S < 64 else np.uint64(0xFFFFFFFFFFFFFFFF)


def assert_same(gpu_words, ref, S, what):
    m = mask(S)
    got = gpu_words & m
    want = ref.words() & m
    if not np.array_equal(got, want):
        bad = np.flatnonzero(got != want)
        raise AssertionError(f"{what}: {bad.size} site words differ, first at site {bad[0]}")


# ---------------------------------------------------------------------------
# inputs and random numbers
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("L", [2, 4, 16, 18])
@pytest.mark.parametrize("prng", ["minstd", "mt19937"])
def test_device_inputs_and_draws_match(sg, L, prng):
    say("inputs", L, prng)
    lat = sg.Lattice(L, 64, prng, coupling_seed=5, spin_seed=6, replica=3)
    assert np.array_equal(lat.couplings(), si.coupling_words(L, 5))
    assert np.array_equal(lat.words(), si.spin_words(L, 6, 3))
    ref = oracle_for(L, 64, prng, 5, 6, 3)
    for t in range(3):
        lat.sweep(1, 0.8)
        R = ref.draws()
        ref.sweep_with(R, 0.8)
        assert np.array_equal(lat.randoms(), R), f"draws of sweep {t}"


@pytest.mark.parametrize("L,nsweeps", [(8, 170), (18, 80)])
def test_mt19937_streams_across_twists(sg, L, nsweeps):
    # 8 or 18 draws per column per sweep: the 624-word blocks end inside sweeps
    say("mt twists", L, nsweeps)
    lat = sg.Lattice(L, 64, "mt19937", coupling_seed=1, spin_seed=9)
    ref = oracle_for(L, 64, "mt19937", 1, 9)
    for t in range(nsweeps):
        lat.sweep(1, 0.6)
        ref.sweep(1, 0.6)
    assert np.array_equal(lat.randoms(), ref.last_R)
    assert_same(lat.words(), ref, 64, f"MT19937 L={L} after {nsweeps} sweeps")


# ---------------------------------------------------------------------------
# the small configuration: L=16, one sample, energy after every sweep
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kernel", ["fused", "twopass"])
def test_single_sample_L16_1000_sweeps_every_sweep(sg, kernel):
    say("L16 1 sample 1000 sweeps", kernel)
    L, beta = 16, 1 / 0.7
    lat = sg.Lattice(L, 1, "minstd", coupling_seed=1, spin_seed=2)
    lat.set_kernel(kernel)
    ref = oracle_for(L, 1, "minstd", 1, 2)
    for t in range(1000):
        lat.sweep(1, beta)
        ref.sweep(1, beta)
        U, e = lat.energy()
        Uo = ref.unsatisfied()
        assert U[0] == Uo[0], f"energy differs after sweep {t + 1}"
        assert e[0] == (2.0 * Uo[0] - 3 * L**3) / L**3
        assert_same(lat.words(), ref, 1, f"sweep {t + 1}")


# ---------------------------------------------------------------------------
# 64 samples, both kernels, both generators, every sweep
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("L", [2, 4, 8, 16, 18, 32])
@pytest.mark.parametrize("prng", ["minstd", "mt19937", "parisi_rapuano"])
@pytest.mark.parametrize("kernel", ["fused", "twopass"])
def test_64_samples_every_sweep(sg, L, prng, kernel):
    say("64 samples", L, prng, kernel)
    lat = sg.Lattice(L, 64, prng, coupling_seed=3, spin_seed=4)
    lat.set_kernel(kernel)
    ref = oracle_for(L, 64, prng, 3, 4)
    for t, beta in enumerate([0.9, 0.9, 0.9, 0.3, 2.0, 1 / 1.1]):
        lat.sweep(1, beta)
        ref.sweep(1, beta)
        assert_same(lat.words(), ref, 64, f"L={L} {prng} {kernel} sweep {t + 1}")
    assert np.array_equal(lat.energy()[0], ref.unsatisfied())


@pytest.mark.parametrize("L,tiles", [
    (24, (12, 24, 24)), (24, (5, 7, 5)), (26, (4, 9, 6)), (34, (17, 3, 34)), (34, (16, 20, 11)), (34, (17, 21, 34)),
    (20, (1, 1, 1)), (22, (11, 22, 3)), (36, (6, 10, 36)),
])
@pytest.mark.parametrize("prng", ["minstd", "mt19937", "parisi_rapuano"])
def test_fused_tile_shapes_and_ragged_edges(sg, L, tiles, prng):
    say("tiles", L, tiles, prng)
    lat = sg.Lattice(L, 64, prng, coupling_seed=8, spin_seed=21)
    lat.set_kernel("fused", *tiles)
    ref = oracle_for(L, 64, prng, 8, 21)
    for t in range(4):
        lat.sweep(1, 0.75)
        ref.sweep(1, 0.75)
        assert_same(lat.words(), ref, 64, f"L={L} tiles={tiles} sweep {t + 1}")


# ---------------------------------------------------------------------------
# two sweeps per launch (MINSTD): calls of 2, 3 and 4 sweeps run two-sweep
# launches and, for an odd count, one one-sweep launch
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("L", [8, 10, 16, 18, 32, 34])
@pytest.mark.parametrize("ring", [5, 6])
def test_two_sweeps_per_launch_every_call(sg, L, ring):
    say("fused2 64 samples", L, ring)
    lat = sg.Lattice(L, 64, "minstd", coupling_seed=3, spin_seed=4)
    lat.set_kernel("fused2")
    lat.set_ring(ring)
    assert lat.kernel()[0] == "fused2" and lat.kernel()[5] == ring
    ref = oracle_for(L, 64, "minstd", 3, 4)
    t = 0
    for n, beta in [(2, 0.9), (3, 0.3), (4, 2.0), (2, 1 / 1.1), (1, 0.9), (2, 0.7)]:
        lat.sweep(n, beta)
        ref.sweep(n, beta)
        t += n
        assert lat.t == t
        assert_same(lat.words(), ref, 64, f"L={L} fused2 after {t} sweeps")
    assert np.array_equal(lat.energy()[0], ref.unsatisfied())


@pytest.mark.parametrize("L,tiles", [
    (24, (12, 20, 24)), (24, (5, 7, 5)), (26, (4, 9, 6)), (34, (17, 3, 34)), (34, (16, 16, 11)),
    (20, (1, 1, 1)), (22, (11, 22, 3)), (36, (6, 10, 36)), (40, (20, 6, 0)), (16, (8, 16, 5)),
])
@pytest.mark.parametrize("ring", [5, 6])
def test_two_sweep_tile_shapes_and_ragged_edges(sg, L, tiles, ring):
    say("fused2 tiles", L, tiles, ring)
    lat = sg.Lattice(L, 64, "minstd", coupling_seed=8, spin_seed=21)
    lat.set_kernel("fused2", *tiles)
    lat.set_ring(ring)
    ref = oracle_for(L, 64, "minstd", 8, 21)
    for k in range(3):
        lat.sweep(2, 0.75)
        ref.sweep(2, 0.75)
        assert_same(lat.words(), ref, 64, f"L={L} fused2 tiles={tiles} after {2 * k + 2} sweeps")


@pytest.mark.parametrize("L", [8, 16, 30])
def test_two_sweeps_two_replicas(sg, L):
    say("fused2 replicas", L)
    a = sg.Lattice(L, 64, "minstd", coupling_seed=7, spin_seed=100, replica=0)
    a.set_kernel("fused2")
    b = sg.Lattice.replica_of(a, spin_seed=100, replica=1)
    b.set_kernel("fused2")
    ra = oracle_for(L, 64, "minstd", 7, 100, 0)
    rb = oracle_for(L, 64, "minstd", 7, 100, 1)
    for n in (2, 3, 2):
        sg.sweep_replicas([a, b], n, 1 / 0.7)
        ra.sweep(n, 1 / 0.7)
        rb.sweep(n, 1 / 0.7)
        assert_same(a.words(), ra, 64, f"replica 0 after {a.t}")
        assert_same(b.words(), rb, 64, f"replica 1 after {b.t}")
    nd, _ = sg.overlap(a, b)
    assert np.array_equal(nd, oracle.ndiff(ra, rb))


# ---------------------------------------------------------------------------
# two sweeps per launch with buffered draws (MT19937, Parisi-Rapuano): the fill
# writes both sweeps' numbers, and the march reads them with the planes
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("L", [8, 10, 16, 18, 32, 34])
@pytest.mark.parametrize("prng", ["mt19937", "parisi_rapuano"])
def test_two_sweeps_buffered_draws_every_call(sg, L, prng):
    say("fused2 buffered", L, prng)
    lat = sg.Lattice(L, 64, prng, coupling_seed=3, spin_seed=4)
    lat.set_kernel("fused2")
    assert lat.kernel()[0] == "fused2" and lat.kernel()[5] == 5
    ref = oracle_for(L, 64, prng, 3, 4)
    t = 0
    for n, beta in [(2, 0.9), (3, 0.3), (4, 2.0), (2, 1 / 1.1), (1, 0.9), (2, 0.7)]:
        lat.sweep(n, beta)
        ref.sweep(n, beta)
        t += n
        assert lat.t == t
        assert_same(lat.words(), ref, 64, f"L={L} {prng} fused2 after {t} sweeps")
        assert np.array_equal(lat.randoms(), ref.last_R), f"draws of sweep {t}"
    assert np.array_equal(lat.energy()[0], ref.unsatisfied())


@pytest.mark.parametrize("L,tiles", [(24, (5, 7, 5)), (26, (4, 9, 6)), (34, (17, 3, 34)), (20, (1, 1, 1)),
                                     (36, (6, 10, 36)), (16, (8, 16, 5))])
@pytest.mark.parametrize("prng", ["mt19937", "parisi_rapuano"])
def test_two_sweeps_buffered_tile_shapes(sg, L, tiles, prng):
    say("fused2 buffered tiles", L, tiles, prng)
    lat = sg.Lattice(L, 64, prng, coupling_seed=8, spin_seed=21)
    lat.set_kernel("fused2", *tiles)
    ref = oracle_for(L, 64, prng, 8, 21)
    for k in range(3):
        lat.sweep(2, 0.75)
        ref.sweep(2, 0.75)
        assert_same(lat.words(), ref, 64, f"L={L} {prng} fused2 tiles={tiles} after {2 * k + 2} sweeps")


@pytest.mark.parametrize("prng", ["mt19937", "parisi_rapuano"])
def test_two_sweeps_buffered_two_replicas(sg, prng):
    say("fused2 buffered replicas", prng)
    L = 18
    a = sg.Lattice(L, 64, prng, coupling_seed=7, spin_seed=100, replica=0)
    a.set_kernel("fused2")
    b = sg.Lattice.replica_of(a, spin_seed=100, replica=1)
    b.set_kernel("fused2")
    ra = oracle_for(L, 64, prng, 7, 100, 0)
    rb = oracle_for(L, 64, prng, 7, 100, 1)
    for n in (2, 3, 2):
        sg.sweep_replicas([a, b], n, 1 / 0.7)
        ra.sweep(n, 1 / 0.7)
        rb.sweep(n, 1 / 0.7)
        assert_same(a.words(), ra, 64, f"replica 0 after {a.t}")
        assert_same(b.words(), rb, 64, f"replica 1 after {b.t}")
        assert np.array_equal(b.randoms(), rb.last_R)
    with pytest.raises(sg.SGError):
        a.set_ring(6)


def test_mt19937_two_sweeps_across_twists(sg):
    # 2 x 18 numbers per column per launch: 624-word blocks end inside launches
    say("mt twists fused2")
    L = 18
    lat = sg.Lattice(L, 64, "mt19937", coupling_seed=1, spin_seed=9)
    lat.set_kernel("fused2")
    ref = oracle_for(L, 64, "mt19937", 1, 9)
    lat.sweep(80, 0.6)
    ref.sweep(80, 0.6)
    assert np.array_equal(lat.randoms(), ref.last_R)
    assert_same(lat.words(), ref, 64, "MT19937 L=18 after 80 sweeps, two per launch")


def test_two_sweeps_L16_single_sample_every_second_sweep(sg):
    say("fused2 L16 1 sample 1000 sweeps")
    L, beta = 16, 1 / 0.7
    lat = sg.Lattice(L, 1, "minstd", coupling_seed=1, spin_seed=2)
    lat.set_kernel("fused2")
    ref = oracle_for(L, 1, "minstd", 1, 2)
    for t in range(500):
        lat.sweep(2, beta)
        ref.sweep(2, beta)
        assert lat.energy()[0][0] == ref.unsatisfied()[0], f"energy differs after sweep {2 * t + 2}"
    assert_same(lat.words(), ref, 1, "after 1000 sweeps")


def test_two_sweeps_beta_zero_and_infinite(sg):
    say("fused2 beta 0 and inf")
    lat = sg.Lattice(20, 64, "minstd", coupling_seed=1, spin_seed=2)
    lat.set_kernel("fused2")
    w0 = lat.words()
    lat.sweep(2, 0.0)
    assert np.array_equal(lat.words(), w0)  # every spin flipped twice
    lat.sweep(3, 0.0)
    assert np.array_equal(lat.words(), ~w0)
    prev = lat.energy()[0]
    for _ in range(3):
        lat.sweep(2, math.inf)
        U = lat.energy()[0]
        assert np.all(U <= prev)
        prev = U


def test_two_sweep_kernel_argument_checks(sg):
    lat = sg.Lattice(16, 64, "minstd", coupling_seed=1, spin_seed=2)
    for bad in (1, 4, 7):
        with pytest.raises(sg.SGError):
            lat.set_ring(bad)
    assert lat.kernel()[5] == 5  # default below L = 512
    mt = sg.Lattice(16, 64, "mt19937", coupling_seed=1, spin_seed=2)
    mt.set_kernel("fused2")
    with pytest.raises(sg.SGError) as e:  # buffered draws: five planes in flight only
        mt.set_ring(6)
    assert e.value.code == sg.SG_EINVAL
    assert mt.kernel()[5] == 5
    small = sg.Lattice(6, 64, "minstd", coupling_seed=1, spin_seed=2)
    with pytest.raises(sg.SGError):
        small.set_kernel("fused2", 3, 3, 0)
    small.set_kernel("auto")  # falls back to the one-sweep kernel below L = 8
    ref = oracle_for(6, 64, "minstd", 1, 2)
    small.sweep(4, 0.8)
    ref.sweep(4, 0.8)
    assert_same(small.words(), ref, 64, "L=6 auto")
    lat = sg.Lattice(16, 64, "minstd", coupling_seed=1, spin_seed=2)
    with pytest.raises(sg.SGError):
        lat.set_kernel("fused2", 9, 40, 0)  # more lanes than a workgroup holds


# ---------------------------------------------------------------------------
# Parisi-Rapuano column streams: the device's numbers and a resumed lattice
# ---------------------------------------------------------------------------
def test_parisi_rapuano_device_numbers_and_forward_moves(sg):
    say("parisi-rapuano numbers")
    L = 18
    lat = sg.Lattice(L, 64, "parisi_rapuano", coupling_seed=2, spin_seed=3)
    seeds = si.pr_seeds(L, 3, 0)
    for t in range(4):
        lat.sweep(1, 0.9)
        got = lat.randoms()
        for c in (0, 1, 17, 100, L * L - 1):
            want = oracle.pr_outputs(seeds[c], (t + 1) * L)[t * L:]
            assert np.array_equal(got[c::L * L], want), (t, c)
    a = sg.Lattice(L, 64, "parisi_rapuano", coupling_seed=2, spin_seed=3)
    a.sweep(5, 0.9)
    b = sg.Lattice(L, 64, "parisi_rapuano", coupling_seed=2, spin_seed=3)
    b.sweep(2, 0.9)
    w = b.words()
    c = sg.Lattice(L, 64, "parisi_rapuano", coupling_seed=2, spin_seed=3)
    c.set_sweep_count(2)  # regenerates the column streams forward
    c.set_spins(w)
    c.sweep(3, 0.9)
    assert np.array_equal(c.words(), a.words())
    with pytest.raises(sg.SGError):
        c.set_ring(6)


# ---------------------------------------------------------------------------
# one number per sample (SG_PHILOX): every kernel, every sweep split
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("L", [8, 16, 18, 32])
@pytest.mark.parametrize("kernel", ["fused2", "fused", "twopass", "auto"])
def test_per_sample_numbers_every_call(sg, L, kernel):
    say("philox", L, kernel)
    lat = sg.Lattice(L, 64, "philox", coupling_seed=3, spin_seed=4)
    lat.set_kernel(kernel)
    ref = oracle_for(L, 64, "philox", 3, 4)
    t = 0
    for n, beta in [(1, 0.9), (2, 0.9), (3, 0.3), (2, 2.0), (1, 1 / 1.1), (2, math.inf), (2, 0.0)]:
        lat.sweep(n, beta)
        ref.sweep(n, beta)
        t += n
        assert_same(lat.words(), ref, 64, f"L={L} philox {kernel} after {t} sweeps")
    assert np.array_equal(lat.energy()[0], ref.unsatisfied())


@pytest.mark.parametrize("kernel", ["fused2", "fused"])
def test_per_sample_numbers_two_replicas(sg, kernel):
    say("philox replicas", kernel)
    L = 16
    a = sg.Lattice(L, 64, "philox", coupling_seed=7, spin_seed=100, replica=0)
    a.set_kernel(kernel)
    b = sg.Lattice.replica_of(a, spin_seed=100, replica=1)
    b.set_kernel(kernel)
    ra = oracle_for(L, 64, "philox", 7, 100, 0)
    rb = oracle_for(L, 64, "philox", 7, 100, 1)
    for n in (2, 1, 2):
        sg.sweep_replicas([a, b], n, 1 / 0.7)
        ra.sweep(n, 1 / 0.7)
        rb.sweep(n, 1 / 0.7)
        assert_same(a.words(), ra, 64, f"replica 0 after {a.t}")
        assert_same(b.words(), rb, 64, f"replica 1 after {b.t}")


def test_per_sample_numbers_split_identical_samples_on_the_gpu(sg):
    """Identical samples (same couplings, same start) stay identical under one
    number per site and evolve apart under one number per sample."""
    say("philox identical samples")
    L = 16
    V = L**3
    rng = np.random.default_rng(3)
    J = rng.integers(0, 2, size=(3, V)).astype(np.uint64) * np.uint64(0xFFFFFFFFFFFFFFFF)
    w0 = rng.integers(0, 2, size=V).astype(np.uint64) * np.uint64(0xFFFFFFFFFFFFFFFF)
    shared = sg.Lattice(L, 64, "minstd", couplings=J, spin_seed=5)
    own = sg.Lattice(L, 64, "philox", couplings=J, spin_seed=5)
    shared.set_spins(w0)
    own.set_spins(w0)
    shared.sweep(4, 0.8)
    own.sweep(4, 0.8)
    ws = shared.words()
    assert np.all((ws == 0) | (ws == np.uint64(0xFFFFFFFFFFFFFFFF)))
    wo = own.words()
    assert np.mean((wo != 0) & (wo != np.uint64(0xFFFFFFFFFFFFFFFF))) > 0.2
    with pytest.raises(sg.SGError):
        own.randoms()  # 64 numbers per site: no single number to return


# ---------------------------------------------------------------------------
# layout study: the colour-separated ("standard") layout and the sliced layout
# of the coordinate transformation give the same spins as the cube kernels
# ---------------------------------------------------------------------------
def _layout_sweep(lat, layout, n, beta, work):
    return lat.sweep_sliced(n, beta, work) if layout == "sliced" else lat.sweep_separated(n, beta, work)


@pytest.mark.parametrize("layout", ["sliced", "separated"])
@pytest.mark.parametrize("L", [2, 4, 8, 18, 32])
@pytest.mark.parametrize("prng", ["minstd", "mt19937", "parisi_rapuano", "philox"])
def test_layout_sweeps_match_the_oracle(sg, layout, L, prng):
    say("layout", layout, L, prng)
    lat = sg.Lattice(L, 64, prng, coupling_seed=5, spin_seed=6)
    ref = oracle_for(L, 64, prng, 5, 6)
    work = None
    t = 0
    for n, beta in [(1, 0.9), (2, 0.4), (3, 1.6), (0, 0.9)]:
        work = _layout_sweep(lat, layout, n, beta, work)
        ref.sweep(n, beta)
        t += n
        assert lat.t == t
        assert_same(lat.words(), ref, 64, f"L={L} {prng} {layout} after {t} sweeps")


@pytest.mark.parametrize("layout", ["sliced", "separated"])
def test_layouts_equal_the_cube_kernels_at_L64(sg, layout):
    say("layout vs cube L64", layout)
    L = 64
    a = sg.Lattice(L, 64, "minstd", coupling_seed=9, spin_seed=10)
    b = sg.Lattice(L, 64, "minstd", coupling_seed=9, spin_seed=10)
    a.sweep(3, 0.8)      # fused kernels
    _layout_sweep(b, layout, 3, 0.8, None)
    assert np.array_equal(a.words(), b.words())
    a.sweep(2, 1.3)
    b.set_kernel("twopass")
    b.sweep(1, 1.3)      # mixing layouts between calls keeps the trajectory
    _layout_sweep(b, layout, 1, 1.3, None)
    assert np.array_equal(a.words(), b.words())
    fn = sg.lib.sg_sweep_sliced if layout == "sliced" else sg.lib.sg_sweep_separated
    with pytest.raises(sg.SGError):
        sg._check(fn(b.handle, 1, 1.0, None, 0))


def test_sliced_layout_mt19937_at_L64_against_the_cube(sg):
    say("sliced mt19937 L64")
    a = sg.Lattice(64, 64, "mt19937", coupling_seed=3, spin_seed=4)
    b = sg.Lattice(64, 64, "mt19937", coupling_seed=3, spin_seed=4)
    a.sweep(5, 0.9)
    b.sweep_sliced(5, 0.9)
    assert np.array_equal(a.words(), b.words())


# ---------------------------------------------------------------------------
# replicas, overlap, energies
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("L", [8, 16, 30])
@pytest.mark.parametrize("prng", ["minstd", "mt19937", "parisi_rapuano"])
@pytest.mark.parametrize("kernel", ["fused", "twopass"])
def test_two_replicas_in_one_pass(sg, L, prng, kernel):
    say("replicas", L, prng, kernel)
    a = sg.Lattice(L, 64, prng, coupling_seed=7, spin_seed=100, replica=0)
    a.set_kernel(kernel)
    b = sg.Lattice.replica_of(a, spin_seed=100, replica=1)
    ra = oracle_for(L, 64, prng, 7, 100, 0)
    rb = oracle_for(L, 64, prng, 7, 100, 1)
    for t in range(5):
        sg.sweep_replicas([a, b], 1, 1 / 0.7)
        ra.sweep(1, 1 / 0.7)
        rb.sweep(1, 1 / 0.7)
        assert_same(a.words(), ra, 64, f"replica 0 sweep {t + 1}")
        assert_same(b.words(), rb, 64, f"replica 1 sweep {t + 1}")
    nd, q = sg.overlap(a, b)
    assert np.array_equal(nd, oracle.ndiff(ra, rb))
    assert np.array_equal(q, 1.0 - 2.0 * oracle.ndiff(ra, rb) / L**3)
    nd, q = sg.overlap(a, a)
    assert np.all(nd == 0) and np.all(q == 1.0)
    assert np.array_equal(a.energy()[0], ra.unsatisfied())
    assert np.array_equal(b.energy()[0], rb.unsatisfied())


def test_overlap_of_a_spin_flipped_copy(sg):
    say("overlap -1")
    a = sg.Lattice(12, 64, "minstd", coupling_seed=1, spin_seed=2)
    b = sg.Lattice.replica_of(a, spin_seed=2, replica=0)
    b.set_spins(~a.words())
    nd, q = sg.overlap(a, b)
    assert np.all(nd == 12**3) and np.all(q == -1.0)


def test_overlap_rejects_different_couplings(sg):
    a = sg.Lattice(8, 64, "minstd", coupling_seed=1, spin_seed=2)
    b = sg.Lattice(8, 64, "minstd", coupling_seed=3, spin_seed=2)
    with pytest.raises(sg.SGError) as e:
        sg.overlap(a, b)
    assert e.value.code == sg.SG_EMISMATCH


# ---------------------------------------------------------------------------
# edge cases: sample counts between 1 and 64, empty calls, invalid arguments
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("S", [1, 7, 33, 63])
@pytest.mark.parametrize("kernel", ["fused2", "fused", "twopass"])
def test_partial_sample_counts(sg, S, kernel):
    say("samples", S, kernel)
    L = 10
    lat = sg.Lattice(L, S, "minstd", coupling_seed=3, spin_seed=4)
    lat.set_kernel(kernel)
    ref = oracle_for(L, S, "minstd", 3, 4)
    for n in (1, 2, 3):
        lat.sweep(n, 0.8)
        ref.sweep(n, 0.8)
        assert_same(lat.words(), ref, S, f"{S} samples, {kernel}, after {lat.t} sweeps")
    U, e = lat.energy()
    assert U.shape == (S,) and np.array_equal(U, ref.unsatisfied())
    assert np.array_equal(e, (2.0 * U - 3 * L**3) / L**3)
    sp = lat.spins()  # int8 +-1 per sample and site, against the oracle's own spins
    assert sp.shape == (S, L**3) and np.array_equal(sp, ref.s)


def test_empty_calls_and_invalid_arguments(sg):
    say("edge arguments")
    lat = sg.Lattice(8, 64, "minstd", coupling_seed=1, spin_seed=2)
    w = lat.words()
    lat.sweep(0, 0.5)
    sg.sweep_replicas([lat], 0, 0.5)
    assert lat.t == 0 and np.array_equal(lat.words(), w)
    for n, beta in ((1, float("nan")), (1, -0.1), (-1, 0.5)):
        with pytest.raises(sg.SGError) as e:
            lat.sweep(n, beta)
        assert e.value.code == sg.SG_EINVAL
    assert lat.t == 0 and np.array_equal(lat.words(), w)
    for L, S in ((15, 64), (0, 64), (8, 0), (8, 65)):
        with pytest.raises(sg.SGError):
            sg.Lattice(L, S, "minstd")


# ---------------------------------------------------------------------------
# limits and properties
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kernel", ["fused", "twopass"])
def test_beta_zero_flips_every_spin(sg, kernel):
    say("beta 0", kernel)
    lat = sg.Lattice(20, 64, "minstd", coupling_seed=1, spin_seed=2)
    lat.set_kernel(kernel)
    w0 = lat.words()
    U0 = lat.energy()[0]
    for t in range(1, 4):
        lat.sweep(1, 0.0)
        assert np.array_equal(lat.words(), w0 if t % 2 == 0 else ~w0)
        assert np.array_equal(lat.energy()[0], U0)


def test_zero_temperature_monotone_and_stream_free(sg):
    say("T=0")
    a = sg.Lattice(24, 64, "mt19937", coupling_seed=4, spin_seed=5, replica=0)
    b = sg.Lattice.replica_of(a, spin_seed=999, replica=7)
    b.set_spins(a.words())
    prev = a.energy()[0]
    for _ in range(5):
        a.sweep(1, math.inf)
        b.sweep(1, math.inf)
        U = a.energy()[0]
        assert np.all(U <= prev)
        prev = U
        assert np.array_equal(a.words(), b.words())


def test_sweep_splitting_kernels_and_resume(sg):
    say("splitting")
    L = 64
    ref = sg.Lattice(L, 64, "minstd", coupling_seed=2, spin_seed=3)
    ref.sweep(9, 0.85)
    two = sg.Lattice(L, 64, "minstd", coupling_seed=2, spin_seed=3)
    two.set_kernel("twopass")
    two.sweep(4, 0.85)
    mid = two.words()
    two.set_kernel("fused")
    two.sweep(5, 0.85)
    assert np.array_equal(two.words(), ref.words())
    # resume from a checkpoint of spins and the sweep count
    res = sg.Lattice(L, 64, "minstd", coupling_seed=2, spin_seed=3)
    res.set_spins(mid)
    res.set_sweep_count(4)
    res.sweep(5, 0.85)
    assert np.array_equal(res.words(), ref.words())
    # MT19937: a fresh lattice can be moved forward, regenerating its streams
    m1 = sg.Lattice(16, 64, "mt19937", coupling_seed=2, spin_seed=3)
    m1.sweep(6, 0.85)
    m2 = sg.Lattice(16, 64, "mt19937", coupling_seed=2, spin_seed=3)
    m2.sweep(2, 0.85)
    w = m2.words()
    m3 = sg.Lattice(16, 64, "mt19937", coupling_seed=2, spin_seed=3)
    m3.set_sweep_count(2)
    m3.set_spins(w)
    m3.sweep(4, 0.85)
    assert np.array_equal(m3.words(), m1.words())


@pytest.mark.parametrize("prng", ["mt19937", "parisi_rapuano", "minstd"])
def test_mid_run_checkpoint_of_stream_states(sg, prng):
    """Spins, stream states and sweep count taken mid-run resume a new lattice
    bit-exactly (the column states of MT19937 / Parisi-Rapuano included)."""
    say("checkpoint", prng)
    L = 18
    a = sg.Lattice(L, 64, prng, coupling_seed=2, spin_seed=3)
    a.sweep(7, 0.85)
    words, state, t = a.words(), a.stream_state(), a.t
    assert state.size == {"mt19937": 4 * 624 * L * L, "parisi_rapuano": 4 * 64 * L * L, "minstd": 0}[prng]
    a.sweep(5, 0.85)
    b = sg.Lattice(L, 64, prng, coupling_seed=2, spin_seed=3)
    b.sweep(1, 0.85)  # a lattice that has swept: its own streams are overwritten
    b.set_spins(words)
    b.set_stream_state(state, t)
    assert b.t == 7
    b.sweep(5, 0.85)
    assert np.array_equal(a.words(), b.words())
    ref = oracle_for(L, 64, prng, 2, 3)
    ref.sweep(12, 0.85)
    assert_same(b.words(), ref, 64, f"{prng} resumed at sweep 7")
    with pytest.raises(sg.SGError):
        b.set_stream_state(np.zeros(3, dtype=np.uint8), 1)


def test_gauge_symmetry_at_L64(sg):
    say("gauge")
    L = 64
    J = si.coupling_words(L, 13)
    g = si.gauge_words(L, 14)
    z, y, x = np.meshgrid(np.arange(L), np.arange(L), np.arange(L), indexing="ij")
    x, y, z = x.ravel(), y.ravel(), z.ravel()
    nb = [((x + 1) % L) + L * (y + L * z), x + L * (((y + 1) % L) + L * z), x + L * (y + L * ((z + 1) % L))]
    Jg = np.stack([J[d] ^ g ^ g[nb[d]] for d in range(3)])
    a = sg.Lattice(L, 64, "minstd", couplings=J, spin_seed=15)
    b = sg.Lattice(L, 64, "minstd", couplings=Jg, spin_seed=15)
    b.set_spins(a.words() ^ g)
    for _ in range(6):
        a.sweep(1, 0.9)
        b.sweep(1, 0.9)
    assert np.array_equal(b.words(), a.words() ^ g)


# ---------------------------------------------------------------------------
# the L=256 configuration on bit planes the oracle can afford
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("prng", ["minstd", "mt19937"])
def test_L256_two_replicas_on_two_bit_planes(sg, prng):
    say("L256", prng)
    L, beta, nsweeps = 256, 1 / 0.7, 2
    a = sg.Lattice(L, 64, prng, coupling_seed=1, spin_seed=2, replica=0)
    b = sg.Lattice.replica_of(a, spin_seed=2, replica=1)
    sg.sweep_replicas([a, b], nsweeps, beta)
    J = si.coupling_words(L, 1)
    for lat, r in ((a, 0), (b, 1)):
        w = lat.words()
        S0 = si.spin_words(L, 2, r)
        for j in (0, 63):
            sh = np.uint64(j)
            seeds = si.minstd_seeds(L, 2, r) if prng == "minstd" else si.mt_seeds(L, 2, r)
            one = oracle.OracleLattice((L, L, L), 1, (J >> sh) & np.uint64(1), (S0 >> sh) & np.uint64(1),
                                       PRNG[prng], seeds)
            one.sweep(nsweeps, beta)
            assert np.array_equal((w >> sh) & np.uint64(1), one.words()), f"replica {r} plane {j}"


@pytest.mark.parametrize("prng", ["minstd", "mt19937", "philox"])
def test_autotune_leaves_state_and_parity(sg, prng):
    say("autotune", prng)
    L, beta = 32, 0.9
    a = sg.Lattice(L, 64, prng, coupling_seed=5, spin_seed=6, replica=0)
    b = sg.Lattice.replica_of(a, spin_seed=6, replica=1)
    ra = oracle_for(L, 64, prng, 5, 6, 0)
    rb = oracle_for(L, 64, prng, 5, 6, 1)
    sg.sweep_replicas([a, b], 2, beta)
    ra.sweep(2, beta)
    rb.sweep(2, beta)
    wa, wb = a.words(), b.words()
    shape, ms = sg.autotune([a, b], reps=2)
    assert shape[0] in ("twopass", "fused", "fused2")
    assert a.kernel()[:5] == shape and b.kernel()[:5] == shape
    assert ms > 0 and (shape[0] == "twopass" or (shape[1] > 0 and shape[2] > 0))
    assert a.t == 2 and b.t == 2
    assert np.array_equal(a.words(), wa) and np.array_equal(b.words(), wb)
    again, ms2 = sg.autotune([a, b], reps=2)
    assert again == shape and ms2 < 0  # taken from the cache
    for n in (1, 2, 3):
        sg.sweep_replicas([a, b], n, beta)
        ra.sweep(n, beta)
        rb.sweep(n, beta)
    assert_same(a.words(), ra, 64, "after autotune, replica 0")
    assert_same(b.words(), rb, 64, "after autotune, replica 1")


# ---------------------------------------------------------------------------
# energies after every sweep in one call (sg_sweep_energies)
# ---------------------------------------------------------------------------
# sides up to 16 with MINSTD or per-sample numbers take the one-workgroup kernel with
# the lattice in LDS (its counts taken per sample up to 4 samples, read by ballots up
# to 16, by a butterfly of bit-sliced additions above), the others a sweep, a count
# and a reduction per sweep;
# the L=16 one-sample case is the benchmark's smallest configuration as it runs
@pytest.mark.parametrize("L,S,prng,n", [(2, 64, "minstd", 40), (4, 1, "minstd", 50), (6, 64, "philox", 12),
                                        (8, 64, "minstd", 30), (12, 64, "philox", 9), (16, 1, "minstd", 1000),
                                        (16, 64, "minstd", 30), (10, 33, "philox", 7), (14, 17, "minstd", 11),
                                        (12, 16, "minstd", 9), (8, 4, "philox", 13), (6, 3, "minstd", 20),
                                        (10, 5, "minstd", 8),
                                        (20, 64, "minstd", 15), (20, 64, "philox", 4), (16, 64, "mt19937", 25),
                                        (18, 64, "parisi_rapuano", 21), (22, 64, "minstd", 7)])
def test_energy_after_every_sweep_in_one_call(sg, L, S, prng, n):
    say("sweep energies", L, S, prng, n)
    lat = sg.Lattice(L, S, prng, coupling_seed=31, spin_seed=32)
    ref = oracle_for(L, S, prng, 31, 32)
    U = lat.sweep_energies(n, 0.8)
    assert U.shape == (n, S) and lat.t == n
    for k in range(n):
        ref.sweep(1, 0.8)
        assert np.array_equal(U[k], ref.unsatisfied()), f"energies after sweep {k + 1}"
    assert_same(lat.words(), ref, S, f"L={L} {prng} after {n} sweeps")
    assert lat.sweep_energies(0, 0.8).shape == (0, S)
    lat.close()


def test_small_lattice_energy_records_across_launches(sg):
    # one launch of the small-lattice kernel covers up to 2049 sweeps: 2100 take two,
    # and a call that follows continues the same trajectory
    say("small-lattice sweep energies in two launches")
    L, n, beta = 4, 2100, 0.7
    lat = sg.Lattice(L, 64, "minstd", coupling_seed=35, spin_seed=36)
    ref = oracle_for(L, 64, "minstd", 35, 36)
    U = lat.sweep_energies(n, beta)
    U2 = lat.sweep_energies(3, beta)
    for k in range(n):
        ref.sweep(1, beta)
        assert np.array_equal(U[k], ref.unsatisfied()), f"energies after sweep {k + 1}"
    for k in range(3):
        ref.sweep(1, beta)
        assert np.array_equal(U2[k], ref.unsatisfied()), f"energies after sweep {n + k + 1}"
    assert lat.t == n + 3
    assert_same(lat.words(), ref, 64, f"L={L} after {n + 3} sweeps")
    lat.close()


def test_energy_records_across_read_back_chunks(sg):
    # at L=320 the reduction area holds 49 sweeps' totals: 100 sweeps take three chunks
    say("sweep energies in chunks")
    L, n, beta = 320, 100, 0.9
    a = sg.Lattice(L, 64, "minstd", coupling_seed=33, spin_seed=34)
    b = sg.Lattice(L, 64, "minstd", coupling_seed=33, spin_seed=34)
    U = a.sweep_energies(n, beta)
    for k in range(n):
        b.sweep(1, beta)
        assert np.array_equal(U[k], b.energy()[0]), f"energies after sweep {k + 1}"
    assert np.array_equal(a.words(), b.words())
    a.close()
    b.close()


# ---------------------------------------------------------------------------
# the flip rule on every local configuration (sg_flip_words)
# ---------------------------------------------------------------------------
def _oracle_decisions(beta, prng, rs):
    """accept[v][k]: the oracle's Metropolis decision for a red site with v of its
    six bonds satisfied (dE = 4v - 12) and R = rs[k], read off one oracle sweep of a
    4x4x4 lattice whose other sites cannot flip."""
    from test_oracle_pins import _site_bonds

    ext, V = (4, 4, 4), 64
    T = oracle.thresholds(beta, prng)
    site = (1, 2, 1)
    i0 = site[0] + 4 * (site[1] + 4 * site[2])
    acc = np.zeros((7, len(rs)), dtype=bool)
    top = 0x7FFFFFFE if prng == oracle.MINSTD else 0xFFFFFFFF
    for v in range(7):
        s = np.ones(V, dtype=np.int8)
        J = np.ones((3, V), dtype=np.int8)
        for k, (d, owner) in enumerate(_site_bonds(ext, *site)):
            J[d, owner] = 1 if k < v else -1  # all spins +1: J = +1 is a satisfied bond
        for k, r in enumerate(rs):
            R = np.full(V, top, dtype=np.uint32)
            R[i0] = r
            acc[v, k] = oracle.sweep_once(ext, s, J, R, T)[i0] != s[i0]
    return acc


@pytest.mark.parametrize("form", [0, 1, 2, 3])
def test_flip_rule_on_every_local_configuration(sg, form):
    """All 2^13 patterns of (s, n0..n5, j0..j5), 64 per word, at R on both sides of
    every threshold, through each compiled form of the bit-sliced rule; each bit
    must follow the oracle's Metropolis decision for its number of satisfied
    bonds (a bond is satisfied when J s_i s_k = +1, i.e. when its three bits XOR to
    0 under the bit mapping of Sec. 4)."""
    say("flip rule", form)
    prng_name = "minstd" if form < 2 else "mt19937"
    prng = oracle.MINSTD if form < 2 else oracle.MT19937
    beta = 0.37
    T = [int(v) for v in oracle.thresholds(beta, prng)]
    top = 0x7FFFFFFE if form < 2 else 0xFFFFFFFF
    rs = sorted({0, T[2] - 1, T[2], T[1] - 1, T[1], T[0] - 1, T[0], top} - {-1})
    acc = _oracle_decisions(beta, prng, rs)
    c = np.arange(1 << 13, dtype=np.uint64).reshape(128, 64)  # config 64w + j in bit j of word w
    bit = lambda b: (((c >> np.uint64(b)) & np.uint64(1)) << np.arange(64, dtype=np.uint64)).sum(
        axis=1, dtype=np.uint64)
    base = np.stack([bit(b) for b in range(13)], axis=1)  # [128][13]: s, n0..n5, j0..j5
    words = np.repeat(base, len(rs), axis=0)
    R = np.tile(np.array(rs, dtype=np.uint32), 128)
    got = sg.flip_words(form, words, R, beta, prng_name)
    sb = (c & np.uint64(1)).astype(np.int64)
    v = np.zeros(c.shape, dtype=np.int64)
    for k in range(6):
        nb = ((c >> np.uint64(1 + k)) & np.uint64(1)).astype(np.int64)
        jb = ((c >> np.uint64(7 + k)) & np.uint64(1)).astype(np.int64)
        v += (sb ^ nb ^ jb) == 0
    for w in range(128):
        for k, r in enumerate(rs):
            flip = acc[v[w], k]
            want = int(base[w, 0]) ^ int((flip.astype(np.uint64) << np.arange(64, dtype=np.uint64)).sum(
                dtype=np.uint64))
            assert int(got[w * len(rs) + k]) == want, (form, w, r)
    # forms with 32-bit comparisons take MINSTD's thresholds only
    if form < 2:
        with pytest.raises(sg.SGError):
            sg.flip_words(form, words[:1], R[:1], beta, "mt19937")
