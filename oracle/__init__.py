"""CPU oracle for the checkerboard Metropolis sweep of the 3D +-J spin glass.

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the GPU library (``paper_1411_0127_amd``) and never imports it; both take
their seeded inputs from ``seeded_inputs``.

What it computes (Lulli, Bernaschi, Parisi, arXiv:1411.0127):

* the Hamiltonian H = -sum_<ik> J_ik s_i s_k with J, s in {-1, +1} (Sec. 1, Eq. 1);
* red/blue checkerboard Metropolis, red (x+y+z even) first (Sec. 1);
* Metropolis acceptance P_flip = 1 for dE <= 0, exp(-beta dE) otherwise, decided
  as an integer comparison R < R_max exp(-beta dE) (Sec. 4);
* asynchronous multispin coding: the samples coded at one site share that site's
  random number (Sec. 4) -- here every sample is simulated on its own, one byte per
  spin, with the shared number;
* MINSTD, MT19937 and Parisi-Rapuano generators (Sec. 3), one MINSTD stream per
  site, one MT19937 or Parisi-Rapuano stream per x-y column;
* a per-sample variant of the acceptance step: every coded sample draws its own
  32-bit number per site and sweep (Philox4x32-10, Salmon et al., SC'11), instead
  of sharing the site's;
* observables: unsatisfied-bond count / energy per spin, and the two-replica
  overlap q (textbook definition; the paper simulates replicas, Sec. 2).

Every function has a pin in ``tests/test_oracle_pins.py``.  The keyed input
generator and the per-site / per-column stream layout are this project's
convention: they are pinned only through determinism and GPU agreement
("parity unpinned" for the stream layout; the generators themselves are pinned).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MINSTD = 0
MT19937 = 1
PHILOX = 2  # one number per sample, per site and sweep
PARISI_RAPUANO = 3
MINSTD_RANGE = 2**31 - 1
MT19937_RANGE = 2**32
PHILOX_RANGE = 2**32
PR_RANGE = 2**32

_lib: Optional[ctypes.CDLL] = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no target-specific tuning)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-pthread", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        p = ctypes.c_void_p
        i64 = ctypes.c_int64
        ci = ctypes.c_int
        L.oc_minstd_next.argtypes = [ctypes.c_uint32]
        L.oc_minstd_next.restype = ctypes.c_uint32
        L.oc_minstd_draws.argtypes = [i64, p, p]
        L.oc_mt_init_many.argtypes = [i64, p, p]
        L.oc_mt_outputs.argtypes = [ctypes.c_uint32, i64, p]
        L.oc_mt_draws.argtypes = [ci, ci, ci, p, p]
        L.oc_mt_sizeof.restype = i64
        L.oc_thresholds.argtypes = [ctypes.c_double, ctypes.c_uint64, p]
        L.oc_sweep.argtypes = [ci, ci, ci, p, p, p, p]
        L.oc_unsatisfied.argtypes = [ci, ci, ci, p, p]
        L.oc_unsatisfied.restype = i64
        L.oc_ndiff.argtypes = [i64, p, p]
        L.oc_ndiff.restype = i64
        L.oc_gibbs.argtypes = [ci, ci, ci, p, ctypes.c_double, p, p, p]
        L.oc_gibbs.restype = ci
        L.oc_run.argtypes = [ci, ci, ci, ci, p, p, ci, p, i64, p, p]
        L.oc_run.restype = ci
        L.oc_run_threads.argtypes = [ci, ci, ci, ci, p, p, ci, p, i64, p, p, ci]
        L.oc_run_threads.restype = ci
        L.oc_philox4x32_10.argtypes = [p, p, p]
        L.oc_pr_sizeof.restype = i64
        L.oc_pr_init_many.argtypes = [i64, p, p]
        L.oc_pr_outputs.argtypes = [p, i64, p]
        L.oc_pr_draws.argtypes = [ci, ci, ci, p, p]
        L.oc_sample_draws.argtypes = [ctypes.c_uint64, i64, i64, p]
        L.oc_sample_draws_all.argtypes = [i64, ci, ctypes.c_uint64, i64, p]
        _lib = L
    return _lib


def _ptr(a: np.ndarray) -> ctypes.c_void_p:
    assert a.flags["C_CONTIGUOUS"]
    return ctypes.c_void_p(a.ctypes.data)


# ---------------------------------------------------------------------------
# Generators
# ---------------------------------------------------------------------------
def minstd_next(r: int) -> int:
    return int(lib().oc_minstd_next(r))


def mt19937_outputs(seed: int, n: int) -> np.ndarray:
    out = np.empty(n, dtype=np.uint32)
    lib().oc_mt_outputs(seed & 0xFFFFFFFF, n, _ptr(out))
    return out


def pr_outputs(seed_words, n: int) -> np.ndarray:
    """First n Parisi-Rapuano numbers from the 61 seed words x_{-61} .. x_{-1}."""
    seed = np.ascontiguousarray(np.asarray(seed_words, dtype=np.uint32))
    assert seed.shape == (61,)
    out = np.empty(n, dtype=np.uint32)
    lib().oc_pr_outputs(_ptr(seed), n, _ptr(out))
    return out


def philox4x32_10(counter, key) -> np.ndarray:
    """Philox4x32-10 of a 4-word counter under a 2-word key (uint32 words)."""
    c = np.ascontiguousarray(np.asarray(counter, dtype=np.uint32))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32))
    out = np.empty(4, dtype=np.uint32)
    lib().oc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def sample_draws(key: int, site: int, t: int) -> np.ndarray:
    """The 64 per-sample numbers of one site in sweep t (uint32[64])."""
    out = np.empty(64, dtype=np.uint32)
    lib().oc_sample_draws(int(key) & 0xFFFFFFFFFFFFFFFF, int(site), int(t), _ptr(out))
    return out


def thresholds(beta: float, prng: int) -> np.ndarray:
    rng = MINSTD_RANGE if prng == MINSTD else 2**32
    T = np.zeros(3, dtype=np.uint64)
    lib().oc_thresholds(float(beta), rng, _ptr(T))
    return T


# ---------------------------------------------------------------------------
# Bit encoding (Sec. 4): J = -1 <-> bit 1, s = +1 <-> bit 1; sample j <-> bit j.
# ---------------------------------------------------------------------------
def spins_from_words(words: np.ndarray, nsamples: int) -> np.ndarray:
    w = np.asarray(words, dtype=np.uint64)
    j = np.arange(nsamples, dtype=np.uint64)[:, None]
    bits = (w[None, :] >> j) & np.uint64(1)
    return (2 * bits.astype(np.int8) - 1).astype(np.int8)


def couplings_from_words(words: np.ndarray, nsamples: int) -> np.ndarray:
    """words: uint64 [3][V] -> int8 [S][3][V]."""
    w = np.asarray(words, dtype=np.uint64)
    j = np.arange(nsamples, dtype=np.uint64)[:, None, None]
    bits = (w[None, :, :] >> j) & np.uint64(1)
    return (1 - 2 * bits.astype(np.int8)).astype(np.int8)


def words_from_spins(s: np.ndarray) -> np.ndarray:
    """int8 [S][V] -> uint64 [V] with bit j = (s[j] == +1); bits >= S are 0."""
    S, V = s.shape
    w = np.zeros(V, dtype=np.uint64)
    for j in range(S):
        w |= (s[j] > 0).astype(np.uint64) << np.uint64(j)
    return w


# ---------------------------------------------------------------------------
# Lattice
# ---------------------------------------------------------------------------
class OracleLattice:
    """One replica of S coded samples on an even Lx x Ly x Lz periodic lattice.

    ``J_words``: uint64 [3][V]; ``spin_words``: uint64 [V];
    ``stream_seeds``: uint32 per-site MINSTD seeds [V], or per-column MT19937
    seeds [Lx*Ly], or per-column Parisi-Rapuano seed words [Lx*Ly][61], or the
    64-bit Philox key of the per-sample numbers.  Samples
    j < S are simulated, each with its own couplings (bit j of every coupling
    word) and the site's shared random number -- or, with PHILOX, its own.
    """

    def __init__(self, extents, nsamples, J_words, spin_words, prng, stream_seeds):
        Lx, Ly, Lz = extents
        assert Lx % 2 == 0 and Ly % 2 == 0 and Lz % 2 == 0, "extents must be even"
        assert 1 <= nsamples <= 64
        self.Lx, self.Ly, self.Lz = int(Lx), int(Ly), int(Lz)
        self.V = self.Lx * self.Ly * self.Lz
        self.S = int(nsamples)
        self.prng = int(prng)
        self.J = np.ascontiguousarray(couplings_from_words(J_words, self.S))
        self.s = np.ascontiguousarray(spins_from_words(spin_words, self.S))
        self.t = 0
        self._init_streams(stream_seeds)

    def _init_streams(self, stream_seeds):
        L = lib()
        if self.prng == MINSTD:
            self.state = np.ascontiguousarray(np.asarray(stream_seeds, dtype=np.uint32).copy())
            assert self.state.shape == (self.V,)
            assert int(self.state.min()) >= 1 and int(self.state.max()) <= MINSTD_RANGE - 1
        elif self.prng == PHILOX:
            self.state = np.array([int(stream_seeds) & 0xFFFFFFFFFFFFFFFF, 0], dtype=np.uint64)  # key, next sweep
        elif self.prng == PARISI_RAPUANO:
            seeds = np.ascontiguousarray(np.asarray(stream_seeds, dtype=np.uint32))
            assert seeds.shape == (self.Lx * self.Ly, 61)
            self.state = np.zeros(seeds.shape[0] * int(L.oc_pr_sizeof()), dtype=np.uint8)
            L.oc_pr_init_many(seeds.shape[0], _ptr(self.state), _ptr(seeds))
        else:
            seeds = np.ascontiguousarray(np.asarray(stream_seeds, dtype=np.uint32))
            assert seeds.shape == (self.Lx * self.Ly,)
            nbytes = int(L.oc_mt_sizeof())
            self.state = np.zeros(seeds.shape[0] * nbytes, dtype=np.uint8)
            L.oc_mt_init_many(seeds.shape[0], _ptr(self.state), _ptr(seeds))
        self.last_R = np.zeros(self.V, dtype=np.uint32)

    @classmethod
    def from_bits(cls, extents, J_bits, spin_bits, prng, stream_seeds):
        """Lattice of S = len(spin_bits) samples given as bit planes: J_bits uint8
        [S][3][V], spin_bits uint8 [S][V] (bit 1 <=> J = -1, s = +1, as in the
        words).  The arrays are converted in place to the +-1 bytes the oracle
        works on, so large lattices need no 64-bit words."""
        self = cls.__new__(cls)
        Lx, Ly, Lz = extents
        assert Lx % 2 == 0 and Ly % 2 == 0 and Lz % 2 == 0, "extents must be even"
        self.Lx, self.Ly, self.Lz = int(Lx), int(Ly), int(Lz)
        self.V = self.Lx * self.Ly * self.Lz
        J = np.ascontiguousarray(J_bits, dtype=np.uint8).view(np.int8)
        s = np.ascontiguousarray(spin_bits, dtype=np.uint8).view(np.int8)
        self.S = int(s.shape[0])
        assert 1 <= self.S <= 64 and J.shape == (self.S, 3, self.V) and s.shape == (self.S, self.V)
        for a in J:
            a *= -2
            a += 1  # bit 1 -> J = -1, bit 0 -> +1
        for a in s:
            a *= 2
            a -= 1  # bit 1 -> s = +1, bit 0 -> -1
        self.J, self.s = J, s
        self.prng = int(prng)
        self.t = 0
        self._init_streams(stream_seeds)
        return self

    def draws(self) -> np.ndarray:
        """Random numbers of the next sweep (advances the streams): uint32 [V], or
        [S][V] with PHILOX."""
        if self.prng == PHILOX:
            R = np.empty((self.S, self.V), dtype=np.uint32)
            lib().oc_sample_draws_all(self.V, self.S, int(self.state[0]), int(self.state[1]), _ptr(R))
            self.state[1] += np.uint64(1)
            return R
        R = np.empty(self.V, dtype=np.uint32)
        if self.prng == MINSTD:
            lib().oc_minstd_draws(self.V, _ptr(self.state), _ptr(R))
        elif self.prng == PARISI_RAPUANO:
            lib().oc_pr_draws(self.Lx, self.Ly, self.Lz, _ptr(self.state), _ptr(R))
        else:
            lib().oc_mt_draws(self.Lx, self.Ly, self.Lz, _ptr(self.state), _ptr(R))
        return R

    def sweep_with(self, R: np.ndarray, beta: float, samples=None):
        """One sweep with given numbers: R [V] shared by the samples, or R [S][V]."""
        T = thresholds(beta, self.prng)
        R = np.ascontiguousarray(np.asarray(R, dtype=np.uint32))
        for j in range(self.S) if samples is None else samples:
            Rj = np.ascontiguousarray(R[j]) if R.ndim == 2 else R
            lib().oc_sweep(self.Lx, self.Ly, self.Lz, _ptr(self.s[j]), _ptr(self.J[j]), _ptr(Rj), _ptr(T))

    def sweep(self, n: int, beta: float, samples=None):
        for _ in range(int(n)):
            R = self.draws()
            self.sweep_with(R, beta, samples)
            self.last_R = R
            self.t += 1

    def run(self, n: int, beta: float, record: bool = False, threads: int = 1):
        """n sweeps in one C call; returns U[t][j] after every sweep if ``record``.
        threads > 1 spreads the draws over sites or columns and each colour pass
        over planes (same result: sites of one colour are independent)."""
        n = int(n)
        T = thresholds(beta, self.prng)
        U = np.zeros((n, self.S), dtype=np.int64) if record else None
        if int(threads) > 1:
            rc = lib().oc_run_threads(self.Lx, self.Ly, self.Lz, self.S, _ptr(self.s), _ptr(self.J), self.prng,
                                      _ptr(self.state), n, _ptr(T), _ptr(U) if record else None, int(threads))
        else:
            rc = lib().oc_run(self.Lx, self.Ly, self.Lz, self.S, _ptr(self.s), _ptr(self.J), self.prng,
                              _ptr(self.state), n, _ptr(T), _ptr(U) if record else None)
        if rc != 0:
            raise MemoryError("oracle run failed")
        self.t += n
        return U

    def unsatisfied(self) -> np.ndarray:
        return np.array(
            [lib().oc_unsatisfied(self.Lx, self.Ly, self.Lz, _ptr(self.s[j]), _ptr(self.J[j])) for j in range(self.S)],
            dtype=np.int64,
        )

    def energy_per_spin(self) -> np.ndarray:
        return (2.0 * self.unsatisfied() - 3.0 * self.V) / self.V

    def words(self) -> np.ndarray:
        return words_from_spins(self.s)


def ndiff(a: OracleLattice, b: OracleLattice) -> np.ndarray:
    assert a.V == b.V and a.S == b.S
    return np.array([lib().oc_ndiff(a.V, _ptr(a.s[j]), _ptr(b.s[j])) for j in range(a.S)], dtype=np.int64)


def overlap(a: OracleLattice, b: OracleLattice) -> np.ndarray:
    return 1.0 - 2.0 * ndiff(a, b) / a.V


def unsatisfied(extents, s: np.ndarray, J: np.ndarray) -> int:
    Lx, Ly, Lz = extents
    s = np.ascontiguousarray(s, dtype=np.int8)
    J = np.ascontiguousarray(J, dtype=np.int8)
    return int(lib().oc_unsatisfied(Lx, Ly, Lz, _ptr(s), _ptr(J)))


def sweep_once(extents, s: np.ndarray, J: np.ndarray, R: np.ndarray, T: np.ndarray) -> np.ndarray:
    """One sweep of one sample on copies of the arrays (pure function form)."""
    Lx, Ly, Lz = extents
    s = np.ascontiguousarray(s, dtype=np.int8).copy()
    J = np.ascontiguousarray(J, dtype=np.int8)
    R = np.ascontiguousarray(R, dtype=np.uint32)
    T = np.ascontiguousarray(T, dtype=np.uint64)
    lib().oc_sweep(Lx, Ly, Lz, _ptr(s), _ptr(J), _ptr(R), _ptr(T))
    return s


def gibbs(extents, J: np.ndarray, beta: float):
    """Exact <E>, <E^2> and P(U) of one sample (J int8 [3][V]) by enumeration."""
    Lx, Ly, Lz = extents
    V = Lx * Ly * Lz
    J = np.ascontiguousarray(J, dtype=np.int8)
    hist = np.zeros(3 * V + 1, dtype=np.float64)
    e1 = ctypes.c_double()
    e2 = ctypes.c_double()
    rc = lib().oc_gibbs(Lx, Ly, Lz, _ptr(J), float(beta), ctypes.byref(e1), ctypes.byref(e2), _ptr(hist))
    if rc != 0:
        raise ValueError("gibbs enumeration needs V <= 24")
    return e1.value, e2.value, hist
