"""Python binding of libsg (include/sg.h): argument marshalling only.

Every step of the sweep runs in the HIP library; PyTorch only provides the device
buffer each lattice lives in and the stream its work is queued on.  If the
library is missing this module raises at import: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsg.so")

SG_MINSTD = 0
SG_MT19937 = 1
SG_PHILOX = 2
SG_PARISI_RAPUANO = 3
SG_OK = 0
SG_EINVAL = -1
SG_ENOMEM = -2
SG_EDEVICE = -3
SG_EMISMATCH = -4
SG_KERNEL_AUTO = 0
SG_KERNEL_TWOPASS = 1
SG_KERNEL_FUSED = 2
SG_KERNEL_FUSED2 = 3

PRNGS = {"minstd": SG_MINSTD, "mt19937": SG_MT19937, "philox": SG_PHILOX, "parisi_rapuano": SG_PARISI_RAPUANO,
         SG_MINSTD: SG_MINSTD, SG_MT19937: SG_MT19937, SG_PHILOX: SG_PHILOX, SG_PARISI_RAPUANO: SG_PARISI_RAPUANO}
KERNELS = {"auto": SG_KERNEL_AUTO, "twopass": SG_KERNEL_TWOPASS, "fused": SG_KERNEL_FUSED, "fused2": SG_KERNEL_FUSED2}
KERNEL_NAMES = {v: k for k, v in KERNELS.items()}

# Every function the header declares, with its ctypes signature.
_p = ctypes.c_void_p
_i = ctypes.c_int
_i64 = ctypes.c_int64
_u64 = ctypes.c_uint64
_u32 = ctypes.c_uint32
_sz = ctypes.c_size_t
_d = ctypes.c_double
SIGNATURES = {
    "sg_footprint": (_i, [_i, _i, _i, ctypes.POINTER(_sz)]),
    "sg_replica_footprint": (_i, [_i, _i, _i, ctypes.POINTER(_sz)]),
    "sg_lattice_create": (_i, [_i, _i, _i, _p, _u64, _u64, _u32, _p, _sz, _p, ctypes.POINTER(_p)]),
    "sg_lattice_create_replica": (_i, [_p, _u64, _u32, _p, _sz, _p, ctypes.POINTER(_p)]),
    "sg_sweep": (_i, [_p, _i64, _d]),
    "sg_sweep_replicas": (_i, [ctypes.POINTER(_p), _i, _i64, _d]),
    "sg_energy": (_i, [_p, _p, _p]),
    "sg_overlap": (_i, [_p, _p, _p, _p]),
    "sg_get_spins": (_i, [_p, _p, _sz]),
    "sg_get_words": (_i, [_p, _p, _sz]),
    "sg_set_spins": (_i, [_p, _p, _sz]),
    "sg_get_couplings": (_i, [_p, _p, _sz]),
    "sg_get_randoms": (_i, [_p, _p, _sz]),
    "sg_thresholds": (_i, [_d, _i, _p]),
    "sg_sweep_count": (_i64, [_p]),
    "sg_set_sweep_count": (_i, [_p, _i64]),
    "sg_stream_state_bytes": (_i, [_p, ctypes.POINTER(_sz)]),
    "sg_get_stream_state": (_i, [_p, _p, _sz]),
    "sg_set_stream_state": (_i, [_p, _p, _sz, _i64]),
    "sg_set_kernel": (_i, [_p, _i, _i, _i, _i, _i]),
    "sg_set_ring": (_i, [_p, _i]),
    "sg_get_kernel": (_i, [_p, _p]),
    "sg_autotune": (_i, [ctypes.POINTER(_p), _i, _i, _p, ctypes.POINTER(_d)]),
    "sg_batch_footprint": (_i, [_i, _i, ctypes.POINTER(_sz)]),
    "sg_batch_create": (_i, [_i, _i, _p, _sz, _p, ctypes.POINTER(_p)]),
    "sg_batch_add": (_i, [_p, _p, _i64, _d]),
    "sg_batch_run": (_i, [_p, _i64, _i, ctypes.POINTER(_i64)]),
    "sg_batch_take_finished": (_i, [_p, ctypes.POINTER(_p), _i, ctypes.POINTER(_i)]),
    "sg_sliced_footprint": (_i, [_i, ctypes.POINTER(_sz)]),
    "sg_sweep_sliced": (_i, [_p, _i64, _d, _p, _sz]),
    "sg_sweep_sliced_static": (_i, [_p, _i64, _d]),
    "sg_sweep_energies": (_i, [_p, _i64, _d, _p]),
    "sg_flip_words": (_i, [_i, _p, _p, _u64, _d, _i, _p, _p]),
    "sg_sweep_separated": (_i, [_p, _i64, _d, _p, _sz]),
    "sg_batch_rounds_left": (_i, [_p, ctypes.POINTER(_i64), ctypes.POINTER(_i64)]),
    "sg_batch_size": (_i, [_p, ctypes.POINTER(_i), ctypes.POINTER(_i), ctypes.POINTER(_i)]),
    "sg_batch_destroy": (_i, [_p]),
    "sg_batch_set_persistent": (_i, [_p, _i, _u32]),
    "sg_batch_set_group_bytes": (_i, [_p, _sz]),
    "sg_batch_check": (_i, [_p]),
    "sg_probe_bandwidth": (_i, [_i, _p, _p, _sz, _i, _p]),
    "sg_destroy": (_i, [_p]),
    "sg_last_error": (ctypes.c_char_p, []),
}


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"libsg.so not found at {LIB_PATH}; build it with "
            "`python -c 'import __graft_entry__ as g; g.build()'` (hipcc, gfx950)"
        )
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


class SGError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libsg error {code}: {msg}")
        self.code = code


def _check(rc: int):
    if rc != SG_OK:
        raise SGError(rc, lib.sg_last_error().decode(errors="replace"))


def _ptr(a: np.ndarray) -> ctypes.c_void_p:
    assert a.flags["C_CONTIGUOUS"]
    return ctypes.c_void_p(a.ctypes.data)


def thresholds(beta: float, prng="minstd") -> np.ndarray:
    T = np.zeros(3, dtype=np.uint64)
    _check(lib.sg_thresholds(float(beta), PRNGS[prng], _ptr(T)))
    return T


def sliced_footprint(L: int) -> int:
    n = _sz()
    _check(lib.sg_sliced_footprint(int(L), ctypes.byref(n)))
    return int(n.value)


def probe_bandwidth(kind: str, dst, src, nbytes: int, stream, blocks: int = 0):
    """Queue a bandwidth probe (sg_probe_bandwidth): kind "read", "copy" or "fill",
    or "read_nt", "copy_nt", "fill_nt" for the streaming forms; dst / src are
    device tensors (src unused for the fills)."""
    k = {"read": 0, "copy": 1, "fill": 2, "read_nt": 3, "copy_nt": 4, "fill_nt": 5}[kind]
    _check(lib.sg_probe_bandwidth(k, _p(dst.data_ptr()), _p(src.data_ptr()) if src is not None else None,
                                  int(nbytes), int(blocks), _p(stream.cuda_stream)))


def flip_words(form: int, words: np.ndarray, R: np.ndarray, beta: float, prng="minstd", stream=None) -> np.ndarray:
    """The flip rule on given configurations (sg_flip_words): words uint64[n][13]
    (s, n0..n5, j0..j5), R uint32[n]; returns the new spin words uint64[n]."""
    torch = _torch()
    w = np.ascontiguousarray(words, dtype=np.uint64)
    r = np.ascontiguousarray(R, dtype=np.uint32)
    n = r.size
    assert w.shape == (n, 13)
    stream = stream if stream is not None else torch.cuda.current_stream()
    with torch.cuda.stream(stream):  # the copies, the kernel and the read-back in one stream order
        dw = torch.from_numpy(w.view(np.int64)).to("cuda")
        dr = torch.from_numpy(r.view(np.int32)).to("cuda")
        out = torch.empty(max(n, 1), dtype=torch.int64, device="cuda")
        _check(lib.sg_flip_words(int(form), _p(dw.data_ptr()), _p(dr.data_ptr()), n, float(beta), PRNGS[prng],
                                 _p(out.data_ptr()), _p(stream.cuda_stream)))
        res = out[:n].cpu()
    stream.synchronize()
    return res.numpy().view(np.uint64)


def footprint(L: int, prng="minstd", own_couplings: bool = True, nsamples: int = 64) -> int:
    """Device bytes of a lattice (sg_footprint), or of a replica sharing another
    lattice's couplings (sg_replica_footprint) when own_couplings is False."""
    n = _sz()
    f = lib.sg_footprint if own_couplings else lib.sg_replica_footprint
    _check(f(int(L), int(nsamples), PRNGS[prng], ctypes.byref(n)))
    return int(n.value)


def _torch():
    import torch

    return torch


class Lattice:
    """One replica of up to 64 coded samples of a cubic L^3 lattice on the GPU."""

    def __init__(self, L: int, nsamples: int = 64, prng="minstd", coupling_seed: int = 1, spin_seed: int = 2,
                 replica: int = 0, couplings: Optional[np.ndarray] = None, device=None, stream=None,
                 _base: "Optional[Lattice]" = None):
        torch = _torch()
        self.L = int(L)
        self.nsamples = int(nsamples)
        self.prng = PRNGS[prng]
        self.V = self.L ** 3
        self.device = torch.device(device if device is not None else "cuda")
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        self._base = _base
        self.nbytes = footprint(self.L, self.prng, own_couplings=_base is None, nsamples=self.nsamples)
        # allocated on the lattice's stream: the caching allocator then keeps the
        # block from other streams until work queued on this one is done
        with torch.cuda.stream(stream):
            self.buf = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
        h = _p()
        sptr = _p(stream.cuda_stream)
        if _base is None:
            jp = None
            if couplings is not None:
                self._J = np.ascontiguousarray(couplings, dtype=np.uint64)
                if self._J.size != 3 * self.V:
                    raise ValueError("couplings must hold 3*L^3 words")
                jp = _ptr(self._J)
            _check(lib.sg_lattice_create(self.L, self.nsamples, self.prng, jp, int(coupling_seed) & (2**64 - 1),
                                         int(spin_seed) & (2**64 - 1), int(replica), _p(self.buf.data_ptr()),
                                         self.nbytes, sptr, ctypes.byref(h)))
        else:
            _check(lib.sg_lattice_create_replica(_base.handle, int(spin_seed) & (2**64 - 1), int(replica),
                                                 _p(self.buf.data_ptr()), self.nbytes, sptr, ctypes.byref(h)))
        self.handle = h

    @classmethod
    def replica_of(cls, base: "Lattice", spin_seed: int, replica: int, stream=None) -> "Lattice":
        return cls(base.L, base.nsamples, base.prng, spin_seed=spin_seed, replica=replica, device=base.device,
                   stream=stream if stream is not None else base.stream, _base=base)

    # -- dynamics -----------------------------------------------------------------
    def sweep(self, n: int, beta: float):
        _check(lib.sg_sweep(self.handle, int(n), float(beta)))

    def _layout_work(self, work):
        torch = _torch()
        if work is None:
            with torch.cuda.stream(self.stream):
                work = torch.empty(sliced_footprint(self.L), dtype=torch.uint8, device=self.buf.device)
        elif work.device.type == "cuda":
            work.record_stream(self.stream)  # queued work reads it after this call returns
        return work

    def sweep_sliced(self, n: int, beta: float, work=None):
        """n sweeps on the sliced layout of Sec. 2 (sg_sweep_sliced); ``work`` is a
        uint8 device tensor of sliced_footprint(L) bytes, allocated when None."""
        work = self._layout_work(work)
        _check(lib.sg_sweep_sliced(self.handle, int(n), float(beta), _p(work.data_ptr()), int(work.numel())))
        return work

    def sweep_sliced_static(self, n: int, beta: float):
        """n sweeps on the sliced layout in the library's static work area
        (sg_sweep_sliced_static: no allocation, L <= 64)."""
        _check(lib.sg_sweep_sliced_static(self.handle, int(n), float(beta)))

    def sweep_separated(self, n: int, beta: float, work=None):
        """n sweeps on the colour-separated layout (sg_sweep_separated); ``work`` as
        for sweep_sliced."""
        work = self._layout_work(work)
        _check(lib.sg_sweep_separated(self.handle, int(n), float(beta), _p(work.data_ptr()), int(work.numel())))
        return work

    def set_kernel(self, kind="auto", tile_x: int = 0, tile_y: int = 0, z_chunk: int = 0, band: int = 0):
        _check(lib.sg_set_kernel(self.handle, KERNELS[kind] if isinstance(kind, str) else int(kind),
                                 int(tile_x), int(tile_y), int(z_chunk), int(band)))

    def set_ring(self, planes: int = 0):
        """Planes in flight of the two-sweep march: 5, 6 or 0 (default)."""
        _check(lib.sg_set_ring(self.handle, int(planes)))

    def kernel(self):
        """(kind, tile_x, tile_y, z_chunk, band, planes in flight) the next sweeps use."""
        out = np.zeros(6, dtype=np.int32)
        _check(lib.sg_get_kernel(self.handle, _ptr(out)))
        return (KERNEL_NAMES[int(out[0])],) + tuple(int(v) for v in out[1:])

    @property
    def t(self) -> int:
        return int(lib.sg_sweep_count(self.handle))

    def set_sweep_count(self, t: int):
        _check(lib.sg_set_sweep_count(self.handle, int(t)))

    # -- observables ------------------------------------------------------------------
    def energy(self):
        """(unsatisfied-bond counts int64[nsamples], energy per spin float64[nsamples])."""
        U = np.zeros(self.nsamples, dtype=np.int64)
        e = np.zeros(self.nsamples, dtype=np.float64)
        _check(lib.sg_energy(self.handle, _ptr(U), _ptr(e)))
        return U, e

    def sweep_energies(self, n: int, beta: float) -> np.ndarray:
        """n sweeps with the unsatisfied-bond counts after every one
        (sg_sweep_energies): int64[n][nsamples]."""
        U = np.zeros((int(n), self.nsamples), dtype=np.int64)
        _check(lib.sg_sweep_energies(self.handle, int(n), float(beta), _ptr(U) if U.size else None))
        return U

    def spins(self) -> np.ndarray:
        out = np.empty((self.nsamples, self.V), dtype=np.int8)
        _check(lib.sg_get_spins(self.handle, _ptr(out), out.size))
        return out

    def words(self) -> np.ndarray:
        out = np.empty(self.V, dtype=np.uint64)
        _check(lib.sg_get_words(self.handle, _ptr(out), out.size))
        return out

    def set_spins(self, w: np.ndarray):
        """Replace the spin words (uint64[L^3])."""
        w = np.ascontiguousarray(w, dtype=np.uint64)
        _check(lib.sg_set_spins(self.handle, _ptr(w), w.size))

    def stream_state(self) -> np.ndarray:
        """Per-column stream states (uint8 bytes; empty for MINSTD and Philox)."""
        n = _sz()
        _check(lib.sg_stream_state_bytes(self.handle, ctypes.byref(n)))
        out = np.empty(int(n.value), dtype=np.uint8)
        _check(lib.sg_get_stream_state(self.handle, _ptr(out) if out.size else None, out.size))
        return out

    def set_stream_state(self, state: np.ndarray, t: int):
        """Restore stream states taken at sweep count t (and set the count to t)."""
        state = np.ascontiguousarray(state, dtype=np.uint8)
        _check(lib.sg_set_stream_state(self.handle, _ptr(state) if state.size else None, state.size, int(t)))

    def couplings(self) -> np.ndarray:
        out = np.empty((3, self.V), dtype=np.uint64)
        _check(lib.sg_get_couplings(self.handle, _ptr(out), out.size))
        return out

    def randoms(self) -> np.ndarray:
        out = np.empty(self.V, dtype=np.uint32)
        _check(lib.sg_get_randoms(self.handle, _ptr(out), out.size))
        return out

    def close(self):
        if getattr(self, "handle", None) is not None:
            lib.sg_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sweep_replicas(lats: Sequence[Lattice], n: int, beta: float):
    arr = (_p * len(lats))(*[l.handle for l in lats])
    _check(lib.sg_sweep_replicas(arr, len(lats), int(n), float(beta)))


def autotune(lats: Sequence[Lattice], reps: int = 5):
    """Pick the fastest sweep kernel and tile for these lattices (1, or 2 replicas swept
    together); returns ((kind, tile_x, tile_y, z_chunk, band), ms per sweep or -1 if taken
    from the cache), kind being "twopass", "fused" or "fused2"."""
    arr = (_p * len(lats))(*[l.handle for l in lats])
    best = np.zeros(5, dtype=np.int32)
    ms = _d()
    _check(lib.sg_autotune(arr, len(lats), int(reps), _ptr(best), ctypes.byref(ms)))
    return (KERNEL_NAMES[int(best[0])],) + tuple(int(v) for v in best[1:]), float(ms.value)


def overlap(a: Lattice, b: Lattice):
    nd = np.zeros(a.nsamples, dtype=np.int64)
    q = np.zeros(a.nsamples, dtype=np.float64)
    _check(lib.sg_overlap(a.handle, b.handle, _ptr(nd), _ptr(q)))
    return nd, q


class Batch:
    """Lattices of mixed sizes advanced together (sg_batch_*): one persistent launch
    per run by default, or one launch per round.

    The lattices must be MINSTD single replicas created on ``stream``; use a
    non-default stream when rounds are replayed from graphs."""

    def __init__(self, max_lattices: int, max_items: int, stream, device=None):
        torch = _torch()
        n = _sz()
        _check(lib.sg_batch_footprint(int(max_lattices), int(max_items), ctypes.byref(n)))
        self.device = torch.device(device if device is not None else "cuda")
        with torch.cuda.stream(stream):  # see Lattice: the block stays with the batch's stream
            self.buf = torch.empty(int(n.value), dtype=torch.uint8, device=self.device)
        self.stream = stream
        h = _p()
        _check(lib.sg_batch_create(int(max_lattices), int(max_items), _p(self.buf.data_ptr()), int(n.value),
                                   _p(stream.cuda_stream), ctypes.byref(h)))
        self.handle = h
        self._members = {}  # handle value -> Lattice, keeps them alive while queued

    def set_group_bytes(self, nbytes: int):
        """Persistent runs launch lattices in groups of at most nbytes of spins and
        couplings (0: all in one launch)."""
        _check(lib.sg_batch_set_group_bytes(self.handle, int(nbytes)))

    def set_persistent(self, on: bool = True, spin_cap: int = 0):
        """One persistent launch per run (True, the default) or one launch per round."""
        _check(lib.sg_batch_set_persistent(self.handle, int(bool(on)), int(spin_cap)))

    def check(self):
        """Synchronise and raise if a persistent run gave up waiting."""
        _check(lib.sg_batch_check(self.handle))

    def add(self, lat: Lattice, nsweeps: int, beta: float):
        _check(lib.sg_batch_add(self.handle, lat.handle, int(nsweeps), float(beta)))
        self._members[lat.handle.value] = lat

    def run(self, max_rounds: int, rounds_per_graph: int = 0) -> int:
        done = _i64()
        _check(lib.sg_batch_run(self.handle, int(max_rounds), int(rounds_per_graph), ctypes.byref(done)))
        return int(done.value)

    def take_finished(self):
        out = []
        while True:
            arr = (_p * 64)()
            n = _i()
            _check(lib.sg_batch_take_finished(self.handle, arr, 64, ctypes.byref(n)))
            for k in range(n.value):
                out.append(self._members.pop(arr[k]))
            if n.value < 64:
                return out

    def rounds_left(self):
        """(rounds until the first active lattice finishes, rounds until the last does)."""
        lo, hi = _i64(), _i64()
        _check(lib.sg_batch_rounds_left(self.handle, ctypes.byref(lo), ctypes.byref(hi)))
        return int(lo.value), int(hi.value)

    def size(self):
        a, f, it = _i(), _i(), _i()
        _check(lib.sg_batch_size(self.handle, ctypes.byref(a), ctypes.byref(f), ctypes.byref(it)))
        return int(a.value), int(f.value), int(it.value)

    def close(self):
        if getattr(self, "handle", None) is not None:
            lib.sg_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
