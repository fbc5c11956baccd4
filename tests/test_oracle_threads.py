"""CPU checks of the oracle's threaded run and of the bit-plane inputs used at
large sizes: both must give exactly what the plain forms give."""
import numpy as np
import pytest

import oracle
import seeded_inputs as si

PRNGS = [oracle.MINSTD, oracle.MT19937, oracle.PHILOX, oracle.PARISI_RAPUANO]


def _seeds(L, prng, sseed, r):
    if prng == oracle.MINSTD:
        return si.minstd_seeds(L, sseed, r)
    if prng == oracle.MT19937:
        return si.mt_seeds(L, sseed, r)
    if prng == oracle.PARISI_RAPUANO:
        return si.pr_seeds(L, sseed, r)
    return si.philox_key(sseed, r)


@pytest.mark.parametrize("prng", PRNGS)
@pytest.mark.parametrize("L,threads", [(2, 3), (6, 4), (10, 7), (16, 5)])
def test_threaded_run_equals_the_serial_run(prng, L, threads):
    J, S0 = si.coupling_words(L, 3), si.spin_words(L, 4, 1)
    a = oracle.OracleLattice((L, L, L), 5, J, S0, prng, _seeds(L, prng, 4, 1))
    b = oracle.OracleLattice((L, L, L), 5, J, S0, prng, _seeds(L, prng, 4, 1))
    Ua = a.run(7, 0.8, record=True)
    Ub = b.run(7, 0.8, record=True, threads=threads)
    assert np.array_equal(a.s, b.s)
    assert np.array_equal(Ua, Ub)
    assert np.array_equal(a.state, b.state)


@pytest.mark.parametrize("L", [4, 18, 32])
def test_bit_planes_equal_the_words(L):
    J = si.coupling_words(L, 7)
    S = si.spin_words(L, 8, 1)
    planes = [0, 5, 63]
    cb = si.coupling_bits(L, 7, planes, threads=3)
    sb = si.spin_bits(L, 8, 1, planes, threads=5)
    for k, p in enumerate(planes):
        sh = np.uint64(p)
        assert np.array_equal(cb[k], ((J >> sh) & np.uint64(1)).astype(np.uint8))
        assert np.array_equal(sb[k], ((S >> sh) & np.uint64(1)).astype(np.uint8))
    assert np.array_equal(si.minstd_seeds_threaded(L, 8, 1, threads=4), si.minstd_seeds(L, 8, 1))


@pytest.mark.parametrize("prng", [oracle.MINSTD, oracle.MT19937])
def test_lattice_from_bit_planes_follows_the_same_trajectory(prng):
    """Samples given as bit planes 0 and 63 evolve like bits 0 and 63 of the
    64-sample lattice (they share the site's numbers)."""
    L = 8
    J, S0 = si.coupling_words(L, 1), si.spin_words(L, 2, 0)
    full = oracle.OracleLattice((L, L, L), 64, J, S0, prng, _seeds(L, prng, 2, 0))
    pl = oracle.OracleLattice.from_bits((L, L, L), si.coupling_bits(L, 1, [0, 63]), si.spin_bits(L, 2, 0, [0, 63]),
                                        prng, _seeds(L, prng, 2, 0))
    full.run(5, 0.9)
    pl.run(5, 0.9, threads=3)
    w = full.words()
    for k, p in enumerate((0, 63)):
        want = ((w >> np.uint64(p)) & np.uint64(1)).astype(np.int8) * 2 - 1
        assert np.array_equal(pl.s[k], want)
