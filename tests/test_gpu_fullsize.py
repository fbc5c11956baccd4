"""Parity at the full benchmark sizes, on sampled sites.

After n sweeps a site's spin depends only on the old spins within Manhattan
distance 2n (a red site reads its neighbours, a blue site reads new red
neighbours).  The oracle therefore reproduces any sampled site exactly from a
window of the global lattice of side 2h+2, h = 2n+1, around it: the wrap of the
window corrupts only sites within 2n of its faces.  The window keeps the global
colour parity, and every site in it gets its global couplings, spins and random
numbers.  All 64 samples of each sampled site are compared bit for bit, in the
launch configuration the benchmark times (autotuned fused tile)."""
import sys

import numpy as np
import pytest

import oracle
import seeded_inputs as si

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def window_check(L, prng, cseed, sseed, replica, words, nsweeps, beta, centers):
    h = 2 * nsweeps + 1
    W = 2 * h + 2
    bad = []
    for (cx, cy, cz) in centers:
        o = [cx - h, cy - h, cz - h]
        if (o[0] + o[1] + o[2]) % 2:
            o[0] -= 1  # keep the global colour of every window site
        lz, ly, lx = np.meshgrid(np.arange(W), np.arange(W), np.arange(W), indexing="ij")
        gx = (o[0] + lx.ravel()) % L
        gy = (o[1] + ly.ravel()) % L
        gz = (o[2] + lz.ravel()) % L
        gsite = gx + L * (gy + L * gz)
        J = si.coupling_words_at(L, cseed, gsite)
        # local bond (i, i+d) must be the global bond (g, g+d): identical inside the window
        S0 = si.spin_words_at(L, sseed, replica, gsite)
        if prng == "philox":
            key = si.philox_key(sseed, replica)
            ref = oracle.OracleLattice((W, W, W), 64, J, S0, oracle.PHILOX, key)
            for t in range(nsweeps):  # every window site draws the numbers of its global site
                R = np.stack([oracle.sample_draws(key, int(g), t) for g in gsite], axis=1)  # [64][W^3]
                ref.sweep_with(R, beta)
        elif prng == "parisi_rapuano":
            cols = (gx + L * gy).reshape(W, W, W)[0].ravel()
            seeds = si.pr_seeds_at(L, sseed, replica, cols)
            outs = np.stack([oracle.pr_outputs(s_, nsweeps * L) for s_ in seeds])
            ref = oracle.OracleLattice((W, W, W), 64, J, S0, oracle.PARISI_RAPUANO, seeds)
            zg = gz.reshape(W, W, W)
            for t in range(nsweeps):
                R = outs[np.tile(np.arange(W * W), W), (t * L + zg.ravel())].astype(np.uint32)
                ref.sweep_with(R, beta)
        elif prng == "minstd":
            ref = oracle.OracleLattice((W, W, W), 64, J, S0, oracle.MINSTD,
                                       si.minstd_seeds_at(L, sseed, replica, gsite))
            ref.sweep(nsweeps, beta)
        else:
            cols = (gx + L * gy).reshape(W, W, W)[0].ravel()  # window column -> global column
            seeds = si.mt_seeds_at(L, sseed, replica, cols)
            outs = np.stack([oracle.mt19937_outputs(int(s), nsweeps * L) for s in seeds])  # [W*W, n*L]
            ref = oracle.OracleLattice((W, W, W), 64, J, S0, oracle.MT19937, seeds)
            zg = gz.reshape(W, W, W)
            for t in range(nsweeps):
                R = outs[np.tile(np.arange(W * W), W), (t * L + zg.ravel())].astype(np.uint32)
                ref.sweep_with(R, beta)
        lc = (cx - o[0]) + W * ((cy - o[1]) + W * (cz - o[2]))
        want = ref.words()[lc]
        got = words[cx + L * (cy + L * cz)]
        if got != want:
            bad.append(((cx, cy, cz), hex(int(got)), hex(int(want))))
    assert not bad, f"{len(bad)} of {len(centers)} sampled sites differ, first {bad[:3]}"


def centers_for(L, rng, n_random, tile=(32, 8)):
    tx, ty = 2 * tile[0], tile[1]
    xs = sorted({0, 1, L - 1, L - 2} | {v % L for k in (1, 2, 3) for v in (k * tx - 1, k * tx, k * tx + 1)})
    ys = sorted({0, 1, L - 1} | {v % L for k in (1, 2) for v in (k * ty - 1, k * ty)})
    zs = sorted({0, 1, L // 2 - 1, L // 2, L - 1})
    pts = [(x, y, z) for x in xs[::2] for y in ys for z in zs]
    pts += [tuple(int(v) for v in rng.integers(0, L, 3)) for _ in range(n_random)]
    return pts


def test_L1024_sampled_sites_after_two_sweeps():
    import torch

    from paper_1411_0127_amd import sg

    say("L1024 window parity")
    L, beta, n = 1024, 1 / 1.1, 2
    lat = sg.Lattice(L, 64, "minstd", coupling_seed=1, spin_seed=2)
    shape, _ = sg.autotune([lat], reps=2)
    lat.sweep(n, beta)
    words = lat.words()
    lat.close()
    del lat
    torch.cuda.empty_cache()
    window_check(L, "minstd", 1, 2, 0, words, n, beta, centers_for(L, np.random.default_rng(5), 120, shape[1:3]))


@pytest.mark.parametrize("prng", ["minstd", "mt19937", "philox", "parisi_rapuano"])
def test_L256_two_replicas_sampled_sites(prng):
    from paper_1411_0127_amd import sg

    say("L256 window parity", prng)
    L, beta, n = 256, 1 / 0.7, 3
    a = sg.Lattice(L, 64, prng, coupling_seed=1, spin_seed=2, replica=0)
    b = sg.Lattice.replica_of(a, spin_seed=2, replica=1)
    shape, _ = sg.autotune([a, b], reps=2)
    sg.sweep_replicas([a, b], n, beta)
    wa, wb = a.words(), b.words()
    rng = np.random.default_rng(9)
    window_check(L, prng, 1, 2, 0, wa, n, beta, centers_for(L, rng, 60, shape[1:3]))
    window_check(L, prng, 1, 2, 1, wb, n, beta, centers_for(L, rng, 30, shape[1:3]))


def test_beyond_two_to_the_31_sites():
    """L = 1300: V = 2.2e9 sites, past every signed 32-bit index.  Two sweeps on
    the two-sweep kernel and one on the one-sweep kernel, checked on sampled
    sites, the last rows and planes among them."""
    import torch

    from paper_1411_0127_amd import sg

    L, beta, n = 1300, 1 / 1.1, 3
    assert L**3 > 2**31
    say("L1300 window parity")
    lat = sg.Lattice(L, 64, "minstd", coupling_seed=4, spin_seed=5)
    lat.sweep(2, beta)  # one two-sweep launch
    lat.sweep(1, beta)  # one one-sweep launch
    words = lat.words()
    lat.close()
    del lat
    torch.cuda.empty_cache()
    rng = np.random.default_rng(12)
    centers = [(L - 1, L - 1, L - 1), (0, L - 1, L - 1), (L - 2, 0, L - 1), (L // 2, L - 1, L - 2), (17, 33, L - 1)]
    centers += [tuple(int(v) for v in rng.integers(0, L, 3)) for _ in range(25)]
    window_check(L, "minstd", 4, 5, 0, words, n, beta, centers)


# ---------------------------------------------------------------------------
# Whole bit-planes against the oracle at the full sizes: sample 0 and sample 63
# of every site, the oracle running those two samples (they share the site's
# numbers) threaded over the host's cores.
# ---------------------------------------------------------------------------
def _threads():
    import os

    env = os.environ.get("OMP_NUM_THREADS")
    return int(env) if env and env.isdigit() and int(env) > 0 else max(1, min(16, os.cpu_count() or 1))


def _planes_oracle(L, prng, cseed, sseed, replica):
    planes = [0, 63]
    seeds = (si.minstd_seeds_threaded(L, sseed, replica, _threads()) if prng == "minstd"
             else si.mt_seeds(L, sseed, replica))
    return oracle.OracleLattice.from_bits((L, L, L), si.coupling_bits(L, cseed, planes, _threads()),
                                          si.spin_bits(L, sseed, replica, planes, _threads()),
                                          oracle.MINSTD if prng == "minstd" else oracle.MT19937, seeds)


def _assert_planes(words, ref, what, chunk=1 << 26):
    for k, p in enumerate((0, 63)):
        sh = np.uint64(p)
        for a in range(0, words.size, chunk):
            got = ((words[a:a + chunk] >> sh) & np.uint64(1)).astype(np.int8) * 2 - 1
            if not np.array_equal(got, ref.s[k, a:a + chunk]):
                bad = a + int(np.flatnonzero(got != ref.s[k, a:a + chunk])[0])
                raise AssertionError(f"{what}: plane {p} differs, first at site {bad}")


@pytest.mark.parametrize("prng,checkpoints", [("minstd", (10, 100, 1000)), ("mt19937", (10, 100))])
def test_L256_two_replicas_bit_planes_at_10_100_1000_sweeps(prng, checkpoints):
    """The L=256 two-replica configuration as the benchmark runs it (autotuned,
    both replicas in one call), planes 0 and 63 of both replicas against the
    oracle after 10 and 100 sweeps, and (MINSTD) of replica 0 after 1000."""
    from paper_1411_0127_amd import sg

    say("L256 bit planes", prng, checkpoints)
    L, beta = 256, 1 / 0.7
    a = sg.Lattice(L, 64, prng, coupling_seed=1, spin_seed=2, replica=0)
    b = sg.Lattice.replica_of(a, spin_seed=2, replica=1)
    sg.autotune([a, b], reps=2)
    refs = [_planes_oracle(L, prng, 1, 2, r) for r in (0, 1)]
    done = 0
    for upto in checkpoints:
        sg.sweep_replicas([a, b], upto - done, beta)
        # past 100 sweeps the oracle follows replica 0 alone (its time is the cost)
        pairs = ((a, refs[0], 0), (b, refs[1], 1)) if upto <= 100 else ((a, refs[0], 0),)
        for lat, ref, r in pairs:
            ref.run(upto - done, beta, threads=_threads())
            _assert_planes(lat.words(), ref, f"{prng} replica {r} after {upto} sweeps")
        say("L256 bit planes", prng, "equal after", upto, "sweeps")
        done = upto
    a.close()
    b.close()


def test_L1024_bit_planes_after_four_sweeps():
    """The L=1024 configuration as the benchmark runs it (autotuned two-sweep
    launches), planes 0 and 63 of all 2^30 sites against the oracle after four
    sweeps."""
    import torch

    from paper_1411_0127_amd import sg

    say("L1024 bit planes")
    L, beta, n = 1024, 1 / 1.1, 4
    lat = sg.Lattice(L, 64, "minstd", coupling_seed=1, spin_seed=2)
    sg.autotune([lat], reps=2)
    lat.sweep(n, beta)
    words = lat.words()
    lat.close()
    del lat
    torch.cuda.empty_cache()
    ref = _planes_oracle(L, "minstd", 1, 2, 0)
    ref.run(n, beta, threads=_threads())
    _assert_planes(words, ref, f"L=1024 after {n} sweeps")


def test_L1024_global_flip_maps_the_whole_trajectory():
    """The energy is even in the spins and a Metropolis decision depends only on the
    products J s_i s_k (Sec. 1, Eq. (1); Sec. 4), so a start with every spin flipped,
    under the same couplings and streams, stays the complement of the original
    sweep after sweep.  Checked on all 64 samples of all 2^30 sites after four
    sweeps in the benchmark's launch configuration (autotuned two-sweep march)."""
    import torch

    from paper_1411_0127_amd import sg

    say("L1024 global flip")
    L, beta, n = 1024, 1 / 1.1, 4
    a = sg.Lattice(L, 64, "minstd", coupling_seed=1, spin_seed=2)
    b = sg.Lattice(L, 64, "minstd", coupling_seed=1, spin_seed=2)
    sg.autotune([a], reps=2)
    sg.autotune([b], reps=2)  # the cached shape
    assert a.kernel() == b.kernel()
    w = a.words()
    np.invert(w, out=w)
    b.set_spins(w)
    del w
    a.sweep(n, beta)
    b.sweep(n, beta)
    wa = a.words()
    a.close()
    wb = b.words()
    b.close()
    del a, b
    torch.cuda.empty_cache()
    np.invert(wb, out=wb)
    assert wa.shape == (L**3,)
    assert np.array_equal(wa, wb), "the flipped start does not stay the complement"
