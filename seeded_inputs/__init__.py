"""Seeded synthetic inputs for the 3D +-J Edwards-Anderson spin glass.

This module is shared by the CPU oracle (through the tests) and by the GPU
library's callers.  It holds no part of the Metropolis method: it only turns
user seeds into the quenched couplings, the initial spins and the initial
state of the per-site / per-column random streams.  The paper draws all of
these "at random" (Sec. 1, bimodal distribution P(J)); a reproducible keyed
generator stands in for its system random pool.

Generator: SplitMix64 (G. L. Steele, D. Lea, C. H. Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014).  Its n-th output from state
``k`` is ``mix64(k + n * GAMMA)`` for n = 1, 2, ...; that definition makes it
counter-based, so any word can be produced on its own.  The GPU library
implements the same published definition in its own device code.

Conventions (this project's, stated once here):

* site index ``i = x + L*(y + L*z)``;
* ``key(seed, tag, r) = out(out(seed, 1 + tag), 1 + r)`` where
  ``out(k, n) = mix64(k + n*GAMMA)``;
* coupling word of bond (i, i + d^) for d in {x, y, z} = 0, 1, 2:
  ``out(key(coupling_seed, TAG_J, 0), 1 + 3*i + d)``; bit j set <=> J = -1 for
  sample j (bit mapping of Sec. 4);
* initial spin word of site i, replica r: ``out(key(spin_seed, TAG_SPIN, r), 1 + i)``;
  bit j set <=> sigma = +1 for sample j;
* MINSTD seed of site (x, y, z), replica r, with k = low 32 bits of
  ``key(spin_seed, TAG_MINSTD, r)``:
  ``1 + ((fmix32((x + L*y) ^ fmix32(z ^ k)) >> 1) mod (2**31 - 2))``, a value in
  [1, 2**31 - 2], i.e. a valid non-zero MINSTD state; fmix32 is the 32-bit
  finalizer of MurmurHash3 (A. Appleby), a bijection of 32-bit words;
* MT19937 seed of column c = x + L*y, replica r:
  ``out(key(spin_seed, TAG_MT, r), 1 + c) & 0xffffffff``;
* key of the per-sample (Philox4x32-10) numbers of replica r:
  ``key(spin_seed, TAG_PHILOX, r)``;
* Parisi-Rapuano seed words x_{-61+k}, k = 0..60, of column c, replica r:
  ``out(key(spin_seed, TAG_PR, r), 1 + 61*c + k) & 0xffffffff``, with the lowest
  bit of word k = 0 set (an odd word guarantees the generator's full period).
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

TAG_J = 1
TAG_SPIN = 2
TAG_MINSTD = 3
TAG_MT = 4
TAG_PHILOX = 5
TAG_PR = 6

MINSTD_MODULUS = 2**31 - 1


def fmix32(h) -> np.ndarray:
    """MurmurHash3 32-bit finalizer (wrapping uint32 arithmetic)."""
    h = np.asarray(h, dtype=np.uint32)
    with np.errstate(over="ignore"):
        h = h ^ (h >> np.uint32(16))
        h = h * np.uint32(0x85EBCA6B)
        h = h ^ (h >> np.uint32(13))
        h = h * np.uint32(0xC2B2AE35)
        return h ^ (h >> np.uint32(16))


def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function on a uint64 array (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def out(key, n) -> np.ndarray:
    """n-th SplitMix64 output (n >= 1) of a generator whose state starts at ``key``."""
    key = np.uint64(int(key) & 0xFFFFFFFFFFFFFFFF)
    n = np.asarray(n, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return mix64(key + n * GAMMA)


def out_scalar(key: int, n: int) -> int:
    return int(out(key, np.array([n], dtype=np.uint64))[0])


def key(seed: int, tag: int, replica: int) -> int:
    return out_scalar(out_scalar(seed, 1 + tag), 1 + replica)


def _chunks(total: int, chunk: int = 1 << 24):
    for start in range(0, total, chunk):
        yield start, min(total, start + chunk)


def coupling_words(L: int, coupling_seed: int) -> np.ndarray:
    """uint64 array J[3][L^3]; J[d][i] is the bond between i and i + d^ (periodic)."""
    V = L**3
    k = key(coupling_seed, TAG_J, 0)
    J = np.empty((3, V), dtype=np.uint64)
    for a, b in _chunks(V):
        i = np.arange(a, b, dtype=np.uint64)
        for d in range(3):
            J[d, a:b] = out(k, np.uint64(1 + d) + np.uint64(3) * i)
    return J


def spin_words(L: int, spin_seed: int, replica: int) -> np.ndarray:
    """uint64 array S[L^3] of initial spin words (bit j = sample j, 1 <=> +1)."""
    V = L**3
    k = key(spin_seed, TAG_SPIN, replica)
    S = np.empty(V, dtype=np.uint64)
    for a, b in _chunks(V):
        S[a:b] = out(k, np.arange(a + 1, b + 1, dtype=np.uint64))
    return S


def _minstd_seed(L: int, k: int, sites) -> np.ndarray:
    i = np.asarray(sites, dtype=np.uint64)
    LL = np.uint64(L * L)
    xy = (i % LL).astype(np.uint32)
    z = (i // LL).astype(np.uint32)
    h = fmix32(xy ^ fmix32(z ^ np.uint32(k))) >> np.uint32(1)
    h = np.where(h >= np.uint32(MINSTD_MODULUS - 1), h - np.uint32(MINSTD_MODULUS - 1), h)
    return (h + np.uint32(1)).astype(np.uint32)


def minstd_seeds(L: int, spin_seed: int, replica: int) -> np.ndarray:
    """uint32 array of per-site MINSTD seeds in [1, 2^31 - 2]."""
    V = L**3
    k = key(spin_seed, TAG_MINSTD, replica) & 0xFFFFFFFF
    s = np.empty(V, dtype=np.uint32)
    for a, b in _chunks(V):
        s[a:b] = _minstd_seed(L, k, np.arange(a, b, dtype=np.uint64))
    return s


def mt_seeds(L: int, spin_seed: int, replica: int) -> np.ndarray:
    """uint32 array of per-column MT19937 seeds, column c = x + L*y."""
    k = key(spin_seed, TAG_MT, replica)
    c = np.arange(1, L * L + 1, dtype=np.uint64)
    return (out(k, c) & np.uint64(0xFFFFFFFF)).astype(np.uint32)


def pr_seeds_at(L: int, spin_seed: int, replica: int, columns) -> np.ndarray:
    """uint32 [len(columns)][61] Parisi-Rapuano seed words of the given columns."""
    k = key(spin_seed, TAG_PR, replica)
    c = np.asarray(columns, dtype=np.uint64)[:, None]
    n = np.uint64(1) + np.uint64(61) * c + np.arange(61, dtype=np.uint64)[None, :]
    w = (out(k, n) & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    w[:, 0] |= np.uint32(1)
    return w


def pr_seeds(L: int, spin_seed: int, replica: int) -> np.ndarray:
    """uint32 [L*L][61] Parisi-Rapuano seed words of every column c = x + L*y."""
    return pr_seeds_at(L, spin_seed, replica, np.arange(L * L))


def philox_key(spin_seed: int, replica: int) -> int:
    """64-bit key of the per-sample numbers of one replica."""
    return key(spin_seed, TAG_PHILOX, replica)


def coupling_words_at(L: int, coupling_seed: int, sites: np.ndarray) -> np.ndarray:
    """Coupling words J[3][len(sites)] of the given site indices (same values as
    coupling_words(L, coupling_seed)[:, sites])."""
    k = key(coupling_seed, TAG_J, 0)
    i = np.asarray(sites, dtype=np.uint64)
    return np.stack([out(k, np.uint64(1 + d) + np.uint64(3) * i) for d in range(3)])


def spin_words_at(L: int, spin_seed: int, replica: int, sites: np.ndarray) -> np.ndarray:
    k = key(spin_seed, TAG_SPIN, replica)
    return out(k, np.asarray(sites, dtype=np.uint64) + np.uint64(1))


def minstd_seeds_at(L: int, spin_seed: int, replica: int, sites: np.ndarray) -> np.ndarray:
    return _minstd_seed(L, key(spin_seed, TAG_MINSTD, replica) & 0xFFFFFFFF, sites)


def mt_seeds_at(L: int, spin_seed: int, replica: int, columns: np.ndarray) -> np.ndarray:
    k = key(spin_seed, TAG_MT, replica)
    return (out(k, np.asarray(columns, dtype=np.uint64) + np.uint64(1)) & np.uint64(0xFFFFFFFF)).astype(np.uint32)


def gauge_words(L: int, gauge_seed: int) -> np.ndarray:
    """Random per-site gauge words g_i for the gauge-symmetry checks."""
    k = key(gauge_seed, 7, 0)
    return out(k, np.arange(1, L**3 + 1, dtype=np.uint64))


def site_index(L: int, x, y, z):
    return np.asarray(x) + L * (np.asarray(y) + L * np.asarray(z))


# ---------------------------------------------------------------------------
# Bit planes at large sizes (planes.c: the same definitions in C, threaded), for
# lattices whose 64-sample words do not fit in host memory (L = 1024: 24 GiB of
# coupling words).  Built with gcc next to this file.
# ---------------------------------------------------------------------------
import ctypes as _ct
import os as _os
import subprocess as _sp

_HERE = _os.path.dirname(_os.path.abspath(__file__))
_PSRC = _os.path.join(_HERE, "planes.c")
_PLIB = _os.path.join(_HERE, "libsi_planes.so")
_plib = None


def build_planes(force: bool = True) -> str:
    if force or not _os.path.exists(_PLIB):
        tmp = _PLIB + ".tmp"
        _sp.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-pthread", "-o", tmp, _PSRC])
        _os.replace(tmp, _PLIB)
    return _PLIB


def _planes_lib():
    global _plib
    if _plib is None:
        if not _os.path.exists(_PLIB) or _os.path.getmtime(_PLIB) < _os.path.getmtime(_PSRC):
            build_planes()
        lib = _ct.CDLL(_PLIB)
        p = _ct.c_void_p
        lib.si_coupling_bits.argtypes = [_ct.c_int64, _ct.c_uint64, p, _ct.c_int, p, _ct.c_int]
        lib.si_spin_bits.argtypes = [_ct.c_int64, _ct.c_uint64, p, _ct.c_int, p, _ct.c_int]
        lib.si_minstd_seeds.argtypes = [_ct.c_int, _ct.c_uint32, p, _ct.c_int]
        _plib = lib
    return _plib


def _threads(threads):
    return int(threads) if threads else max(1, min(16, _os.cpu_count() or 1))


def coupling_bits(L: int, coupling_seed: int, planes, threads: int = 0) -> np.ndarray:
    """uint8 [len(planes)][3][L^3]: bit p of every coupling word, for p in planes
    (the same bits as coupling_words(L, coupling_seed) >> p & 1)."""
    pl = np.ascontiguousarray(np.asarray(planes, dtype=np.int32))
    V = L**3
    bits = np.empty((pl.size, 3, V), dtype=np.uint8)
    _planes_lib().si_coupling_bits(V, key(coupling_seed, TAG_J, 0), pl.ctypes.data, pl.size, bits.ctypes.data,
                                   _threads(threads))
    return bits


def spin_bits(L: int, spin_seed: int, replica: int, planes, threads: int = 0) -> np.ndarray:
    """uint8 [len(planes)][L^3]: bit p of every initial spin word."""
    pl = np.ascontiguousarray(np.asarray(planes, dtype=np.int32))
    V = L**3
    bits = np.empty((pl.size, V), dtype=np.uint8)
    _planes_lib().si_spin_bits(V, key(spin_seed, TAG_SPIN, replica), pl.ctypes.data, pl.size, bits.ctypes.data,
                               _threads(threads))
    return bits


def minstd_seeds_threaded(L: int, spin_seed: int, replica: int, threads: int = 0) -> np.ndarray:
    """minstd_seeds(L, spin_seed, replica), computed in C on several threads."""
    s = np.empty(L**3, dtype=np.uint32)
    _planes_lib().si_minstd_seeds(L, key(spin_seed, TAG_MINSTD, replica) & 0xFFFFFFFF, s.ctypes.data,
                                  _threads(threads))
    return s
