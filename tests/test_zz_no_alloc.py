"""The allocation-free sliced sweep (sg_sweep_sliced_static) against the sliced
sweep with a caller work buffer (sg_sweep_sliced), through the C ABI.

Spins are integer words: the bar is bit-exactness.  Two calls in a row on the
static work area, the second on a smaller lattice, so that a stale word left by
the first call would show.  Each case is printed before it touches the GPU."""
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


def _pair(sg, L, prng, cseed, sseed):
    return (sg.Lattice(L, 64, prng, coupling_seed=cseed, spin_seed=sseed),
            sg.Lattice(L, 64, prng, coupling_seed=cseed, spin_seed=sseed))


@pytest.mark.parametrize("prng", ["minstd", "mt19937"])
def test_static_sweep_equals_the_buffered_one_on_two_calls(sg, prng):
    # first call: the largest side the static area takes; second: a smaller one
    for L, n, beta, cseed, sseed in ((64, 3, 0.9, 21, 22), (16, 2, 1.4, 23, 24)):
        say("static sliced", prng, "L", L, "sweeps", n)
        a, b = _pair(sg, L, prng, cseed, sseed)
        a.sweep_sliced(n, beta)          # caller work buffer
        b.sweep_sliced_static(n, beta)   # static work area
        wa, wb = a.words(), b.words()
        assert b.t == a.t == n
        assert np.array_equal(wa, wb), f"L={L} {prng}: static and buffered sliced sweeps differ"
        if L == 16:
            seeds = si.minstd_seeds(L, sseed, 0) if prng == "minstd" else si.mt_seeds(L, sseed, 0)
            ref = oracle.OracleLattice((L, L, L), 64, si.coupling_words(L, cseed), si.spin_words(L, sseed, 0),
                                       oracle.MINSTD if prng == "minstd" else oracle.MT19937, seeds)
            ref.sweep(n, beta)
            assert np.array_equal(wb, ref.words()), f"L={L} {prng}: static sliced sweep differs from the oracle"
        a.close()
        b.close()


def test_static_sweep_rejects_sides_beyond_its_area(sg):
    say("static sliced size limit")
    lat = sg.Lattice(66, 64, "minstd", coupling_seed=1, spin_seed=2)
    before = lat.words()
    with pytest.raises(sg.SGError) as e:
        lat.sweep_sliced_static(1, 1.0)
    assert e.value.code == sg.SG_EINVAL
    assert "64" in str(e.value)
    assert lat.t == 0 and np.array_equal(lat.words(), before)
    lat.close()
