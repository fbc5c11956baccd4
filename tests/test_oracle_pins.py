"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test would catch a plausible slip in the oracle (a dropped bond, a wrong
sign, a swapped index, a wrong colour order, a <= for a <, a wrong generator
constant).  None of them re-types the oracle's own formula: they use published
check values, an independent library implementation (numpy's MT19937), closed
forms, invariants, exact enumeration, and the table printed in Sec. 4.
"""
import math
import os

import numpy as np
import pytest

import oracle
import seeded_inputs as si

M31 = 2**31 - 1


def _rand_lattice(ext, seed):
    rng = np.random.default_rng(seed)
    V = ext[0] * ext[1] * ext[2]
    s = rng.choice(np.array([-1, 1], dtype=np.int8), V)
    J = rng.choice(np.array([-1, 1], dtype=np.int8), (3, V))
    return s, J


def _coords(ext):
    Lx, Ly, Lz = ext
    z, y, x = np.meshgrid(np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing="ij")
    return x.ravel(), y.ravel(), z.ravel()


def _site_bonds(ext, x, y, z):
    """(direction, owner index) of the six bonds of site (x, y, z)."""
    Lx, Ly, Lz = ext
    i = lambda a, b, c: (a % Lx) + Lx * ((b % Ly) + Ly * (c % Lz))
    return [(0, i(x, y, z)), (1, i(x, y, z)), (2, i(x, y, z)),
            (0, i(x - 1, y, z)), (1, i(x, y - 1, z)), (2, i(x, y, z - 1))]


# ---------------------------------------------------------------------------
# Generators
# ---------------------------------------------------------------------------
def test_minstd_published_check_value():
    # Park & Miller (CACM 1988): from seed 1 the 10000th state is 1043618065.
    r = 1
    for _ in range(10000):
        r = oracle.minstd_next(r)
    assert r == 1043618065


def test_minstd_per_site_streams_jump_ahead():
    # The draw of sweep t at a site with seed s is 16807^(t+1) s mod (2^31 - 1):
    # computed here by modular exponentiation, not by iterating.
    L = 4
    seeds = si.minstd_seeds(L, 11, 0)
    lat = oracle.OracleLattice((L, L, L), 1, si.coupling_words(L, 1), si.spin_words(L, 11, 0),
                               oracle.MINSTD, seeds)
    for t in range(5):
        R = lat.draws()
        a = pow(16807, t + 1, M31)
        expect = (a * seeds.astype(object)) % M31
        assert np.array_equal(R.astype(object), expect)


def test_mt19937_published_check_values():
    # init_genrand(5489): first output 3499211612; the 10000th is 4123659995
    # (the check value the C++ standard library specifies for mt19937).
    out = oracle.mt19937_outputs(5489, 10000)
    assert int(out[0]) == 3499211612
    assert int(out[9999]) == 4123659995


@pytest.mark.parametrize("seed", [0, 1, 12345, 2**31 + 7, 2**32 - 1])
def test_mt19937_matches_numpy_legacy(seed):
    # numpy's legacy RandomState seeds MT19937 with init_genrand for an integer
    # seed: an independent implementation; 2000 outputs cross three twists.
    ref = np.random.RandomState(seed)._bit_generator.random_raw(2000).astype(np.uint32)
    assert np.array_equal(oracle.mt19937_outputs(seed, 2000), ref)


def test_mt19937_column_stream_layout():
    # Site (x, y, z) takes output t*Lz + z of its column's stream at sweep t.
    ext = (4, 2, 6)
    Lx, Ly, Lz = ext
    seeds = np.array([17, 99, 3, 12345, 7, 8, 2**32 - 5, 42], dtype=np.uint32)
    V = Lx * Ly * Lz
    lat = oracle.OracleLattice(ext, 1, np.zeros((3, V), np.uint64), np.zeros(V, np.uint64),
                               oracle.MT19937, seeds)
    Rs = [lat.draws() for _ in range(3)]
    for c, sd in enumerate(seeds):
        ref = np.random.RandomState(int(sd))._bit_generator.random_raw(3 * Lz).astype(np.uint32)
        x, y = c % Lx, c // Lx
        for t in range(3):
            for z in range(Lz):
                assert Rs[t][x + Lx * (y + Ly * z)] == ref[t * Lz + z]


# ---------------------------------------------------------------------------
# Thresholds
# ---------------------------------------------------------------------------
def test_thresholds_edge_cases():
    assert list(oracle.thresholds(0.0, oracle.MINSTD)) == [M31] * 3
    assert list(oracle.thresholds(0.0, oracle.MT19937)) == [2**32] * 3
    assert list(oracle.thresholds(math.inf, oracle.MINSTD)) == [0, 0, 0]
    # exp(-4 beta) = 1/2 exactly in binary64 for beta = ln2/4
    b = math.log(2.0) / 4
    assert int(oracle.thresholds(b, oracle.MT19937)[0]) == 2**31
    assert int(oracle.thresholds(b, oracle.MINSTD)[0]) == 2**30  # ceil((2^31-1)/2)
    assert int(oracle.thresholds(b, oracle.MT19937)[1]) == 2**30
    for beta in (0.1, 0.5, 1 / 0.7, 1 / 1.1, 3.0):
        T = [int(v) for v in oracle.thresholds(beta, oracle.MINSTD)]
        assert T[0] >= T[1] >= T[2] >= 0
        for k in range(3):
            p = math.exp(-4 * (k + 1) * beta)
            assert abs(T[k] - M31 * p) <= 1.0


# ---------------------------------------------------------------------------
# Update rule: ΔE table of Sec. 4, the printed mask, and energy differences
# ---------------------------------------------------------------------------
def _load_dE_table(golden_dir):
    rows = []
    with open(os.path.join(golden_dir, "paper_dE_table.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                a, b = line.split()
                rows.append((int(a), int(b)))
    return dict(rows)


def _paper_mask(v, r, T):
    """The flip mask printed in Sec. 4, evaluated on one bit: v = sum of bond bits."""
    s2, s1, s0 = (v >> 2) & 1, (v >> 1) & 1, v & 1
    c12, c8, c4 = int(r < T[2]), int(r < T[1]), int(r < T[0])
    return c12 | (1 - s2) | ((s2 & (s2 ^ s1)) & (c8 | (c4 & (1 - s0))))


def test_dE_table_and_mask_against_oracle(golden_dir):
    table = _load_dE_table(golden_dir)
    assert sorted(table) == list(range(7))
    ext = (4, 4, 4)
    V = 64
    beta = 0.4
    T = [int(v) for v in oracle.thresholds(beta, oracle.MINSTD)]
    site = (1, 2, 1)  # x+y+z even: red
    i0 = site[0] + 4 * (site[1] + 4 * site[2])
    bonds = _site_bonds(ext, *site)
    for v in range(7):
        s = np.ones(V, dtype=np.int8)
        J = np.ones((3, V), dtype=np.int8)
        for k, (d, owner) in enumerate(bonds):
            J[d, owner] = 1 if k < v else -1  # all spins +1: J=+1 satisfied
        # the table's dE is the oracle's energy difference of the flip
        U0 = oracle.unsatisfied(ext, s, J)
        s2 = s.copy()
        s2[i0] = -1
        assert 2 * (oracle.unsatisfied(ext, s2, J) - U0) == table[v]
        # the oracle's decision equals the paper's mask in every R region
        for r in (0, T[2] - 1, T[2], T[1] - 1, T[1], T[0] - 1, T[0], M31 - 1):
            R = np.full(V, M31 - 1, dtype=np.uint32)
            R[i0] = r
            new = oracle.sweep_once(ext, s, J, R, np.array(T, dtype=np.uint64))
            assert int(new[i0] != s[i0]) == _paper_mask(v, r, T), (v, r)


@pytest.mark.parametrize("ext,beta,seed", [((4, 4, 6), 0.9, 5), ((2, 4, 4), 0.3, 6), ((6, 2, 2), 2.0, 7)])
def test_update_rule_is_metropolis_on_energy_differences(ext, beta, seed):
    """Red sites decide on the old state, blue sites on the state after the red
    pass; each flips iff dE <= 0 or R < T(dE), dE from the energy function."""
    s, J = _rand_lattice(ext, seed)
    V = s.size
    T = [int(v) for v in oracle.thresholds(beta, oracle.MINSTD)]
    rng = np.random.default_rng(seed + 100)
    cand = np.array([1, max(T[2] - 1, 1), T[2] + 1, T[1] - 1, T[1], T[0] - 1, T[0], M31 - 1], dtype=np.int64)
    R = rng.choice(cand, V).astype(np.uint32)
    new = oracle.sweep_once(ext, s, J, R, np.array(T, dtype=np.uint64))
    x, y, z = _coords(ext)
    red = (x + y + z) % 2 == 0

    def expect(state, i):
        U0 = oracle.unsatisfied(ext, state, J)
        s2 = state.copy()
        s2[i] = -s2[i]
        dE = 2 * (oracle.unsatisfied(ext, s2, J) - U0)
        return dE <= 0 or R[i] < T[dE // 4 - 1]

    for i in np.flatnonzero(red):
        assert (new[i] != s[i]) == expect(s, i)
    mid = s.copy()
    mid[red] = new[red]
    for i in np.flatnonzero(~red):
        assert (new[i] != mid[i]) == expect(mid, i)


# ---------------------------------------------------------------------------
# Energy function: closed forms and symmetries
# ---------------------------------------------------------------------------
def test_energy_closed_forms():
    ext = (4, 6, 2)
    V = 48
    up = np.ones(V, dtype=np.int8)
    ferro = np.ones((3, V), dtype=np.int8)
    assert oracle.unsatisfied(ext, up, ferro) == 0
    assert oracle.unsatisfied(ext, up, -ferro) == 3 * V
    x, y, z = _coords(ext)
    neel = np.where((x + y + z) % 2 == 0, 1, -1).astype(np.int8)
    assert oracle.unsatisfied(ext, neel, ferro) == 3 * V
    # one flipped spin in a ferromagnet breaks its six bonds
    one = up.copy()
    one[7] = -1
    assert oracle.unsatisfied(ext, one, ferro) == 6


def test_energy_symmetries():
    ext = (4, 4, 4)
    s, J = _rand_lattice(ext, 3)
    U = oracle.unsatisfied(ext, s, J)
    assert oracle.unsatisfied(ext, (-s).astype(np.int8), J) == U          # global flip
    assert oracle.unsatisfied(ext, s, (-J).astype(np.int8)) == 3 * 64 - U  # J -> -J: E -> -E
    g = np.random.default_rng(4).choice(np.array([-1, 1], dtype=np.int8), 64)
    Lx, Ly, Lz = ext
    x, y, z = _coords(ext)
    nb = [((x + 1) % Lx) + Lx * (y + Ly * z), x + Lx * (((y + 1) % Ly) + Ly * z), x + Lx * (y + Ly * ((z + 1) % Lz))]
    Jg = np.stack([J[d] * g * g[nb[d]] for d in range(3)]).astype(np.int8)
    assert oracle.unsatisfied(ext, (s * g).astype(np.int8), Jg) == U     # gauge invariance


# ---------------------------------------------------------------------------
# Dynamics: beta = 0, T = 0, gauge, splitting, bit planes
# ---------------------------------------------------------------------------
def _seeded(L, S, prng, cseed=1, sseed=2, r=0):
    seeds = si.minstd_seeds(L, sseed, r) if prng == oracle.MINSTD else si.mt_seeds(L, sseed, r)
    return oracle.OracleLattice((L, L, L), S, si.coupling_words(L, cseed), si.spin_words(L, sseed, r), prng, seeds)


@pytest.mark.parametrize("prng", [oracle.MINSTD, oracle.MT19937])
def test_beta_zero_accepts_everything(prng):
    lat = _seeded(6, 64, prng)
    s0 = lat.s.copy()
    U0 = lat.unsatisfied()
    for t in range(1, 4):
        lat.sweep(1, 0.0)
        assert np.array_equal(lat.s, s0 if t % 2 == 0 else -s0)
        assert np.array_equal(lat.unsatisfied(), U0)


def test_zero_temperature_is_monotone_and_stream_independent():
    a = _seeded(8, 16, oracle.MINSTD, sseed=2)
    b = _seeded(8, 16, oracle.MINSTD, sseed=2)
    b.state = si.minstd_seeds(8, 999, 3).copy()  # other random numbers, same start
    prev = a.unsatisfied()
    for _ in range(6):
        a.sweep(1, math.inf)
        b.sweep(1, math.inf)
        U = a.unsatisfied()
        assert np.all(U <= prev)
        prev = U
        assert np.array_equal(a.s, b.s)


@pytest.mark.parametrize("prng", [oracle.MINSTD, oracle.MT19937])
def test_gauge_symmetry_of_the_dynamics(prng):
    L = 6
    Jw = si.coupling_words(L, 5)
    Sw = si.spin_words(L, 6, 0)
    g = si.gauge_words(L, 77)
    x, y, z = _coords((L, L, L))
    nb = [((x + 1) % L) + L * (y + L * z), x + L * (((y + 1) % L) + L * z), x + L * (y + L * ((z + 1) % L))]
    Jg = np.stack([Jw[d] ^ g ^ g[nb[d]] for d in range(3)])
    seeds = si.minstd_seeds(L, 6, 0) if prng == oracle.MINSTD else si.mt_seeds(L, 6, 0)
    a = oracle.OracleLattice((L, L, L), 64, Jw, Sw, prng, seeds)
    b = oracle.OracleLattice((L, L, L), 64, Jg, Sw ^ g, prng, seeds)
    for _ in range(4):
        a.sweep(1, 0.8)
        b.sweep(1, 0.8)
        assert np.array_equal(b.words(), a.words() ^ g)


def test_call_splitting_and_run_agree():
    a = _seeded(6, 8, oracle.MT19937)
    b = _seeded(6, 8, oracle.MT19937)
    a.sweep(5, 1.2)
    for _ in range(5):
        b.sweep(1, 1.2)
    c = _seeded(6, 8, oracle.MT19937)
    c.run(2, 1.2)
    c.run(3, 1.2)
    assert np.array_equal(a.s, b.s) and np.array_equal(a.s, c.s)


def test_sample_is_its_bit_plane():
    L = 6
    full = _seeded(L, 64, oracle.MINSTD)
    full.sweep(3, 0.9)
    for j in (0, 17, 63):
        Jw = (si.coupling_words(L, 1) >> np.uint64(j)) & np.uint64(1)
        Sw = (si.spin_words(L, 2, 0) >> np.uint64(j)) & np.uint64(1)
        one = oracle.OracleLattice((L, L, L), 1, Jw, Sw, oracle.MINSTD, si.minstd_seeds(L, 2, 0))
        one.sweep(3, 0.9)
        assert np.array_equal(one.s[0], full.s[j])


def test_overlap_limits():
    a = _seeded(4, 64, oracle.MINSTD)
    b = _seeded(4, 64, oracle.MINSTD)
    assert np.all(oracle.overlap(a, b) == 1.0)
    b.s = (-b.s).astype(np.int8)
    assert np.all(oracle.overlap(a, b) == -1.0)


# ---------------------------------------------------------------------------
# Exact enumeration and the Gibbs law of the dynamics (Eq. 3)
# ---------------------------------------------------------------------------
def test_enumeration_closed_forms():
    ext = (2, 2, 4)
    V = 16
    _, J = _rand_lattice(ext, 8)
    # beta = 0: <E> = 0 and <E^2> = sum over pairs of bonds joining the same two sites
    e1, e2, hist = oracle.gibbs(ext, J, 0.0)
    assert abs(e1) < 1e-12
    Lx, Ly, Lz = ext
    x, y, z = _coords(ext)
    ends = []
    for d, (dx, dy, dz) in enumerate([(1, 0, 0), (0, 1, 0), (0, 0, 1)]):
        k = ((x + dx) % Lx) + Lx * (((y + dy) % Ly) + Ly * ((z + dz) % Lz))
        for i in range(V):
            ends.append((frozenset((i, int(k[i]))), int(J[d, i])))
    expect = sum(ja * jb for (pa, ja) in ends for (pb, jb) in ends if pa == pb)
    assert abs(e2 - expect) < 1e-9
    assert abs(hist.sum() - 1) < 1e-12
    # an unfrustrated (gauge-ferromagnetic) coupling set has E_min = -3V
    g = np.random.default_rng(9).choice(np.array([-1, 1], dtype=np.int8), V)
    nb = [((x + 1) % Lx) + Lx * (y + Ly * z), x + Lx * (((y + 1) % Ly) + Ly * z), x + Lx * (y + Ly * ((z + 1) % Lz))]
    Jg = np.stack([g * g[nb[d]] for d in range(3)]).astype(np.int8)
    e1, _, hist = oracle.gibbs(ext, Jg, 8.0)
    assert abs(e1 + 3 * V) < 1e-6 and hist[0] > 1 - 1e-6
    # gauge invariance of the whole distribution
    _, _, h1 = oracle.gibbs(ext, J, 0.7)
    Jgg = np.stack([J[d] * g * g[nb[d]] for d in range(3)]).astype(np.int8)
    _, _, h2 = oracle.gibbs(ext, Jgg, 0.7)
    assert np.allclose(h1, h2, atol=1e-14)


def _binned_mean_err(series, nbins=40):
    n = len(series) // nbins * nbins
    b = series[:n].reshape(nbins, -1).mean(axis=1)
    return series[:n].mean(), b.std(ddof=1) / math.sqrt(nbins)


@pytest.mark.parametrize("beta", [0.5, 1 / 0.7, 2.0])
def test_metropolis_reaches_the_gibbs_law_on_2x2x4(beta):
    """Time averages of E and E^2 of the oracle's dynamics agree with exact
    enumeration within 5 standard errors (binned), for 8 coupling samples."""
    ext = (2, 2, 4)
    V = 16
    S = 8
    rng = np.random.default_rng(2024)
    Jw = rng.integers(0, 2**63, size=(3, V), dtype=np.uint64)
    Sw = rng.integers(0, 2**63, size=V, dtype=np.uint64)
    seeds = rng.integers(1, M31 - 1, size=V, dtype=np.uint32)
    lat = oracle.OracleLattice(ext, S, Jw, Sw, oracle.MINSTD, seeds)
    lat.run(2000, beta)
    U = lat.run(60000, beta, record=True)
    E = 2.0 * U - 3.0 * V
    n = E.shape[0]
    for j in range(S):
        e1, e2, hist = oracle.gibbs(ext, lat.J[j], beta)
        # the binned error cannot be smaller than that of n independent draws
        var1 = e2 - e1 * e1
        Eu = 2.0 * np.arange(3 * V + 1) - 3.0 * V
        var2 = float((hist * Eu**4).sum()) - e2 * e2
        m, err = _binned_mean_err(E[:, j])
        err = max(err, math.sqrt(max(var1, 0.0) / n))
        assert abs(m - e1) < 5 * err, (j, m, e1, err)
        m2, err2 = _binned_mean_err(E[:, j] ** 2)
        err2 = max(err2, math.sqrt(max(var2, 0.0) / n))
        assert abs(m2 - e2) < 5 * err2, (j, m2, e2, err2)


# ---------------------------------------------------------------------------
# per-sample numbers (one 32-bit draw per coded sample, per site and sweep)
# ---------------------------------------------------------------------------
PHILOX_KAT = [  # known-answer vectors of the Philox4x32-10 definition (Salmon et al., SC'11)
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


def test_philox_known_answers():
    for ctr, key, want in PHILOX_KAT:
        assert tuple(int(v) for v in oracle.philox4x32_10(ctr, key)) == want


def _rocrand_philox_tool(tmp_path):
    """A host program computing Philox4x32-10 with rocRAND's own implementation
    (a header shipped with ROCm), to compare the oracle against."""
    import shutil
    import subprocess

    hdr = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hdr) or not os.path.exists(hipcc):
        pytest.skip("rocRAND headers or hipcc not available")
    src = tmp_path / "philox_ref.cpp"
    src.write_text(
        "#include <cstdio>\n#include <rocrand/rocrand_philox4x32_10.h>\n"
        "struct Raw : rocrand_device::philox4x32_10_engine {\n"
        "  uint4 run(uint4 c, uint2 k) { return ten_rounds(c, k); }\n};\n"
        "int main() { Raw r; unsigned v[6];\n"
        "  while (scanf(\"%x %x %x %x %x %x\", v, v + 1, v + 2, v + 3, v + 4, v + 5) == 6) {\n"
        "    uint4 o = r.run(uint4{v[0], v[1], v[2], v[3]}, uint2{v[4], v[5]});\n"
        "    printf(\"%x %x %x %x\\n\", o.x, o.y, o.z, o.w); } }\n")
    exe = tmp_path / "philox_ref"
    r = subprocess.run([hipcc, "-O1", "-o", str(exe), str(src)], capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("cannot build the rocRAND reference: " + r.stderr[-300:])
    return exe


def test_philox_matches_rocrand(tmp_path):
    import subprocess

    exe = _rocrand_philox_tool(tmp_path)
    rng = np.random.default_rng(77)
    cases = rng.integers(0, 2**32, size=(300, 6), dtype=np.uint64)
    inp = "\n".join(" ".join(f"{int(v):x}" for v in row) for row in cases) + "\n"
    out = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True).stdout.split("\n")
    for row, line in zip(cases, out):
        want = [int(v, 16) for v in line.split()]
        got = oracle.philox4x32_10(row[:4], row[4:])
        assert [int(v) for v in got] == want, row


def test_per_sample_numbers_are_uniform_and_distinct_across_samples():
    key = si.philox_key(5, 0)
    R = np.stack([oracle.sample_draws(key, i, t) for i in range(300) for t in (0, 1, 7)])  # [900][64]
    # top 4 bits of 57600 draws: chi-square with 15 degrees of freedom
    h = np.bincount((R >> np.uint32(28)).ravel(), minlength=16)
    e = R.size / 16
    chi2 = float(((h - e) ** 2 / e).sum())
    assert chi2 < 45.0, chi2  # p ~ 1e-4
    # neighbouring samples, sites and sweeps draw different numbers
    assert (R[:, 1:] != R[:, :-1]).mean() > 0.999
    assert (R[1:] != R[:-1]).mean() > 0.999
    # every bit of every sample is used: each of the 32 bit positions is set about half the time
    bits = ((R[..., None] >> np.arange(32, dtype=np.uint32)) & np.uint32(1)).mean(axis=(0, 1))
    assert np.all(np.abs(bits - 0.5) < 0.02)


def test_per_sample_numbers_split_identical_samples():
    """With one number per site (asynchronous multispin coding) samples with the
    same couplings and start stay identical; with one number per sample they
    evolve apart."""
    ext = (6, 6, 6)
    V = 216
    rng = np.random.default_rng(3)
    J1 = rng.integers(0, 2, size=(3, V)).astype(np.uint64) * np.uint64(0xFFFFFFFFFFFFFFFF)
    S1 = rng.integers(0, 2, size=V).astype(np.uint64) * np.uint64(0xFFFFFFFFFFFFFFFF)
    shared = oracle.OracleLattice(ext, 64, J1, S1, oracle.MINSTD, si.minstd_seeds(6, 9, 0))
    own = oracle.OracleLattice(ext, 64, J1, S1, oracle.PHILOX, si.philox_key(9, 0))
    shared.sweep(4, 0.8)
    own.sweep(4, 0.8)
    assert len({w.tobytes() for w in shared.s}) == 1
    assert len({w.tobytes() for w in own.s}) > 32


def test_per_sample_beta_zero_and_zero_temperature():
    ext = (4, 4, 4)
    V = 64
    rng = np.random.default_rng(8)
    Jw = rng.integers(0, 2**63, size=(3, V), dtype=np.uint64)
    Sw = rng.integers(0, 2**63, size=V, dtype=np.uint64)
    lat = oracle.OracleLattice(ext, 64, Jw, Sw, oracle.PHILOX, 12345)
    lat.sweep(1, 0.0)
    assert np.array_equal(lat.words(), ~Sw)  # every proposal accepted
    prev = lat.unsatisfied()
    for _ in range(4):
        lat.sweep(1, math.inf)
        U = lat.unsatisfied()
        assert np.all(U <= prev)
        prev = U


@pytest.mark.parametrize("beta", [0.5, 1 / 0.7])
def test_per_sample_metropolis_reaches_the_gibbs_law_on_2x2x4(beta):
    """The per-sample variant is Metropolis for every sample on its own: time
    averages of E and E^2 agree with exact enumeration within 5 standard errors."""
    ext = (2, 2, 4)
    V = 16
    S = 6
    rng = np.random.default_rng(2025)
    Jw = rng.integers(0, 2**63, size=(3, V), dtype=np.uint64)
    Sw = rng.integers(0, 2**63, size=V, dtype=np.uint64)
    lat = oracle.OracleLattice(ext, S, Jw, Sw, oracle.PHILOX, si.philox_key(4, 0))
    lat.run(1000, beta)
    U = lat.run(30000, beta, record=True)
    E = 2.0 * U - 3.0 * V
    n = E.shape[0]
    for j in range(S):
        e1, e2, hist = oracle.gibbs(ext, lat.J[j], beta)
        var1 = e2 - e1 * e1
        Eu = 2.0 * np.arange(3 * V + 1) - 3.0 * V
        var2 = float((hist * Eu**4).sum()) - e2 * e2
        m, err = _binned_mean_err(E[:, j])
        err = max(err, math.sqrt(max(var1, 0.0) / n))
        assert abs(m - e1) < 5 * err, (j, m, e1, err)
        m2, err2 = _binned_mean_err(E[:, j] ** 2)
        err2 = max(err2, math.sqrt(max(var2, 0.0) / n))
        assert abs(m2 - e2) < 5 * err2, (j, m2, e2, err2)


# ---------------------------------------------------------------------------
# Parisi-Rapuano (Sec. 3).  No independent implementation or published values of
# its 32-bit words are at hand.  The pins are the linear recurrence of the lowest
# bit, which follows from addition mod 2 (a wrong lag breaks it); the words
# recovered through the lag-61 output rule, which must add with carries bit by bit
# (XOR in place of + breaks it, a wrong output lag too); uniformity; and the Gibbs
# law of the dynamics it drives.
# ---------------------------------------------------------------------------
def test_parisi_rapuano_lowest_bit_obeys_the_lagged_xor_recurrence():
    seeds = si.pr_seeds(4, 11, 0)
    for c in (0, 5, 15):
        R = oracle.pr_outputs(seeds[c], 20000)
        b = (R & np.uint32(1)).astype(np.uint8)
        n = np.arange(116, b.size)
        assert np.array_equal(b[n], b[n - 24] ^ b[n - 55])
        # the neighbouring lags do not hold
        assert not np.array_equal(b[n], b[n - 23] ^ b[n - 55])
        assert not np.array_equal(b[n], b[n - 24] ^ b[n - 54])


def _pr_recover_x(seed, R):
    """Undo the output rule R_n = x_n XOR x_{n-61}: starting from the 61 seed words
    x_{-61} .. x_{-1}, x_n = R_n XOR x_{n-61} gives every later x_n from the numbers
    alone.  Returns x_{-61} .. x_{N-1}."""
    x = np.empty(61 + R.size, dtype=np.uint32)
    x[:61] = seed
    for n in range(R.size):
        x[61 + n] = R[n] ^ x[n]
    return x


def test_parisi_rapuano_recovered_words_add_with_carries():
    """The words recovered through the lag-61 output rule must obey the additive
    recurrence bit by bit: bit 0 of x_n is the XOR of bit 0 of x_{n-24} and x_{n-55},
    bit 1 adds the carry out of bit 0, and a ripple-carry adder written out with
    boolean operations reproduces all 32 bits.  A generator that XORs instead of
    adding fails the carry checks, and one whose output lag is not 61 makes the
    recovered words fail even the lowest-bit recurrence."""
    seeds = si.pr_seeds(4, 11, 0)
    for c in (0, 6, 13):
        R = oracle.pr_outputs(seeds[c], 5000)
        x = _pr_recover_x(seeds[c], R)
        n = np.arange(61, x.size)  # positions of x_0, x_1, ...
        a, b, s = x[n - 24], x[n - 55], x[n]
        bit = lambda w, k: ((w >> np.uint32(k)) & np.uint32(1)).astype(np.uint8)
        assert np.array_equal(bit(s, 0), bit(a, 0) ^ bit(b, 0))
        assert np.array_equal(bit(s, 1), bit(a, 1) ^ bit(b, 1) ^ (bit(a, 0) & bit(b, 0)))
        carry = np.zeros(n.size, dtype=np.uint8)
        for k in range(32):
            ak, bk = bit(a, k), bit(b, k)
            assert np.array_equal(bit(s, k), ak ^ bk ^ carry), k
            carry = (ak & bk) | (carry & (ak ^ bk))
        # the carries matter: XOR alone differs from the recovered words
        assert (s != (a ^ b)).mean() > 0.7


def test_parisi_rapuano_output_lag_is_61():
    """The recovery above only closes at lag 61: undoing the output with lag 60 or
    62 leaves words that break the lowest-bit recurrence."""
    seeds = si.pr_seeds(4, 5, 1)
    R = oracle.pr_outputs(seeds[3], 3000)
    for lag in (60, 62):
        x = np.empty(lag + R.size, dtype=np.uint32)
        x[:lag] = np.resize(seeds[3], lag)
        for k in range(R.size):
            x[lag + k] = R[k] ^ x[k]
        n = np.arange(lag + 61, x.size)
        b0 = x & np.uint32(1)
        assert not np.array_equal(b0[n], b0[n - 24] ^ b0[n - 55]), lag


def test_parisi_rapuano_outputs_are_uniform_and_streams_differ():
    seeds = si.pr_seeds(8, 3, 0)
    R = np.stack([oracle.pr_outputs(seeds[c], 4000) for c in range(16)])
    h = np.bincount((R >> np.uint32(28)).ravel(), minlength=16)
    e = R.size / 16
    chi2 = float(((h - e) ** 2 / e).sum())
    assert chi2 < 45.0, chi2
    bits = ((R[..., None] >> np.arange(32, dtype=np.uint32)) & np.uint32(1)).mean(axis=(0, 1))
    assert np.all(np.abs(bits - 0.5) < 0.02)
    assert (R[1:] != R[:-1]).mean() > 0.999  # columns draw different numbers
    # lag-1 serial correlation of the normalised numbers
    u = R.astype(np.float64) / 2**32
    corr = float(np.mean((u[:, 1:] - 0.5) * (u[:, :-1] - 0.5)) / np.var(u))
    assert abs(corr) < 0.02


def test_parisi_rapuano_column_streams_in_sweep_order():
    """Site (x, y, z) takes number t*L + z of column x + L*y in sweep t."""
    L = 4
    seeds = si.pr_seeds(L, 7, 1)
    rng = np.random.default_rng(1)
    Jw = rng.integers(0, 2**63, size=(3, L**3), dtype=np.uint64)
    Sw = rng.integers(0, 2**63, size=L**3, dtype=np.uint64)
    lat = oracle.OracleLattice((L, L, L), 1, Jw, Sw, oracle.PARISI_RAPUANO, seeds)
    got = np.stack([lat.draws() for _ in range(3)])  # [t][V]
    for c in (0, 3, 9, 15):
        want = oracle.pr_outputs(seeds[c], 3 * L).reshape(3, L)
        assert np.array_equal(got[:, c::L * L], want)


@pytest.mark.parametrize("beta", [0.5, 1 / 0.7])
def test_parisi_rapuano_metropolis_reaches_the_gibbs_law_on_2x2x4(beta):
    ext = (2, 2, 4)
    V = 16
    S = 6
    rng = np.random.default_rng(2026)
    Jw = rng.integers(0, 2**63, size=(3, V), dtype=np.uint64)
    Sw = rng.integers(0, 2**63, size=V, dtype=np.uint64)
    lat = oracle.OracleLattice(ext, S, Jw, Sw, oracle.PARISI_RAPUANO, si.pr_seeds(2, 4, 0))
    lat.run(2000, beta)
    U = lat.run(60000, beta, record=True)
    E = 2.0 * U - 3.0 * V
    n = E.shape[0]
    for j in range(S):
        e1, e2, hist = oracle.gibbs(ext, lat.J[j], beta)
        var1 = e2 - e1 * e1
        Eu = 2.0 * np.arange(3 * V + 1) - 3.0 * V
        var2 = float((hist * Eu**4).sum()) - e2 * e2
        m, err = _binned_mean_err(E[:, j])
        err = max(err, math.sqrt(max(var1, 0.0) / n))
        assert abs(m - e1) < 5 * err, (j, m, e1, err)
        m2, err2 = _binned_mean_err(E[:, j] ** 2)
        err2 = max(err2, math.sqrt(max(var2, 0.0) / n))
        assert abs(m2 - e2) < 5 * err2, (j, m2, e2, err2)
