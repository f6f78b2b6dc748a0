"""CPU oracle for the SNAP read-alignment path — TEST INFRASTRUCTURE ONLY.

Plain, slow, literal implementation of the paper's method (arXiv 1111.5572,
Section 3: hash index, seed order, bounded edit distance, Algorithm 1 with the
bucket merge and two-orientation lookup) in C (oracle.c), wrapped with ctypes.

Only tests/, the smoke check and the benchmark's CPU-baseline leg may import
this package. It shares no code with the GPU path; the two meet only through
inputs drawn from the `synth` module.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_HDR = os.path.join(_HERE, "oracle.h")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

INF = 0x3FFFFFFF


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc."""
    newest = max(os.path.getmtime(_SRC), os.path.getmtime(_HDR))
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < newest:
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread", "-Wall",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


class Params(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in
                ("seed_len", "n_min", "n_cap", "bp_per_seed", "conf_c", "max_hits", "d_max", "d_max_pct", "bucket")]


class Stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in
                ("seeds_looked_up", "seeds_over_limit", "seeds_with_n", "candidates", "ed_calls", "ed_over_limit",
                 "lv_extensions", "index_lookups", "select_visits")]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        lib.orc_index_build.argtypes = [P, i64, i32]
        lib.orc_index_build.restype = P
        lib.orc_index_build_threads.argtypes = [P, i64, i32, i32]
        lib.orc_index_build_threads.restype = P
        lib.orc_index_build_strided.argtypes = [P, i64, i32, i32, i32]
        lib.orc_index_build_strided.restype = P
        lib.orc_index_stride.argtypes = [P]
        lib.orc_index_stride.restype = i32
        lib.orc_index_entries.argtypes = [P, P, P, i64]
        lib.orc_index_entries.restype = i64
        lib.orc_dup_classes.argtypes = [P, i64, i64, P]
        lib.orc_dup_classes.restype = i32
        lib.orc_index_free.argtypes = [P]
        lib.orc_index_free.restype = None
        lib.orc_index_windows.argtypes = [P]
        lib.orc_index_windows.restype = i64
        lib.orc_index_occ.argtypes = [P, P, P, i64]
        lib.orc_index_occ.restype = i64
        lib.orc_seed_offsets.argtypes = [i32, i32, i32, P]
        lib.orc_seed_offsets.restype = i32
        lib.orc_seeds_for_length.argtypes = [ctypes.POINTER(Params), i32]
        lib.orc_seeds_for_length.restype = i32
        lib.orc_dmax_for_length.argtypes = [ctypes.POINTER(Params), i32]
        lib.orc_dmax_for_length.restype = i32
        lib.orc_edit_distance.argtypes = [P, i32, P, i32, i32]
        lib.orc_edit_distance.restype = i32
        lib.orc_align.argtypes = [P, P, P, P, i64, ctypes.POINTER(Params), P, P, P, P, P,
                                  ctypes.POINTER(Stats), i32]
        lib.orc_align.restype = i32
        lib.orc_align_log.argtypes = [P, P, i32, ctypes.POINTER(Params), P, P, P, P, i32]
        lib.orc_align_log.restype = i32
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _bytes(x) -> np.ndarray:
    if isinstance(x, (bytes, bytearray)):
        return np.frombuffer(bytes(x), dtype=np.uint8).copy()
    if isinstance(x, str):
        return np.frombuffer(x.encode(), dtype=np.uint8).copy()
    return np.ascontiguousarray(x, dtype=np.uint8)


def make_params(seed_len=20, n_min=10, n_cap=32, bp_per_seed=100, conf_c=2, max_hits=300, d_max=8,
                d_max_pct=0, bucket=32) -> Params:
    return Params(seed_len, n_min, n_cap, bp_per_seed, conf_c, max_hits, d_max, d_max_pct, bucket)


def params_from(p) -> Params:
    """From any object with the Table 3 fields (e.g. synth.workloads.Params)."""
    return make_params(p.seed_len, p.n_min, p.n_cap, p.bp_per_seed, p.conf_c, p.max_hits, p.d_max,
                       p.d_max_pct, p.bucket)


def edit_distance(read, text, lim: int) -> int:
    """Bounded edit distance (start anchored, end free); INF above lim."""
    r, t = _bytes(read), _bytes(text)
    return int(_load().orc_edit_distance(_p(r), len(r), _p(t), len(t), lim))


def dup_classes(genome, W: int) -> np.ndarray:
    """rep[p]: the smallest position whose W-base window equals p's (exact duplicates)."""
    g = _bytes(genome)
    rep = np.empty(max(len(g), 1), np.int64)
    if _load().orc_dup_classes(_p(g), len(g), W, _p(rep)) != 0:
        raise ValueError("invalid sizes")
    return rep[:len(g)]


def seed_offsets(L: int, s: int, n: int) -> list[int]:
    out = np.zeros(max(n, 1), dtype=np.int32)
    k = _load().orc_seed_offsets(L, s, n, _p(out))
    return [int(v) for v in out[:k]]


def seeds_for_length(params: Params, L: int) -> int:
    return int(_load().orc_seeds_for_length(ctypes.byref(params), L))


def dmax_for_length(params: Params, L: int) -> int:
    return int(_load().orc_dmax_for_length(ctypes.byref(params), L))


@dataclass
class Result:
    pos: np.ndarray
    strand: np.ndarray
    dist: np.ndarray
    second: np.ndarray
    call: np.ndarray
    stats: dict
    threads: int

    def fields(self):
        return (self.pos, self.strand, self.dist, self.second, self.call)


class Index:
    """Sorted (window, position) index of every N-free s-mer of a genome."""

    def __init__(self, genome, seed_len: int = 20, threads: int = 1, stride: int = 1):
        """threads > 1 builds the same sorted array with a parallel bucket sort; stride > 1
        indexes only the windows at multiples of the stride."""
        self.genome = _bytes(genome)
        self.seed_len = seed_len
        self.stride = stride
        if stride != 1:
            self._h = _load().orc_index_build_strided(_p(self.genome), len(self.genome), seed_len, stride, threads)
        elif threads > 1:
            self._h = _load().orc_index_build_threads(_p(self.genome), len(self.genome), seed_len, threads)
        else:
            self._h = _load().orc_index_build(_p(self.genome), len(self.genome), seed_len)
        if not self._h:
            raise ValueError("invalid index arguments")

    def close(self):
        if self._h:
            _load().orc_index_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def windows(self) -> int:
        return int(_load().orc_index_windows(self._h))

    def entries(self):
        """The sorted (window key, position) arrays of the index."""
        n = self.windows
        keys = np.empty(max(n, 1), np.uint64)
        qs = np.empty(max(n, 1), np.int64)
        _load().orc_index_entries(self._h, _p(keys), _p(qs), n)
        return keys[:n], qs[:n]

    def occ(self, seed) -> list[int] | None:
        s = _bytes(seed)
        assert len(s) == self.seed_len
        cap = 1 << 16
        out = np.zeros(cap, dtype=np.int64)
        k = int(_load().orc_index_occ(self._h, _p(s), _p(out), cap))
        if k < 0:
            return None
        if k > cap:
            out = np.zeros(k, dtype=np.int64)
            _load().orc_index_occ(self._h, _p(s), _p(out), k)
        return [int(v) for v in out[:k]]

    def align(self, bases, offsets, lengths, params: Params, threads: int = 0) -> Result:
        bases = _bytes(bases)
        offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        lengths = np.ascontiguousarray(lengths, dtype=np.int32)
        n = lengths.shape[0]
        pos = np.empty(n, np.int64)
        strand = np.empty(n, np.int8)
        dist = np.empty(n, np.int32)
        second = np.empty(n, np.int32)
        call = np.empty(n, np.int8)
        st = Stats()
        used = _load().orc_align(self._h, _p(bases), _p(offsets), _p(lengths), n, ctypes.byref(params),
                                 _p(pos), _p(strand), _p(dist), _p(second), _p(call), ctypes.byref(st),
                                 threads)
        return Result(pos, strand, dist, second, call, st.as_dict(), int(used))

    def align_reads(self, reads, params: Params, threads: int = 0) -> Result:
        """reads: synth.Reads."""
        return self.align(reads.bases, reads.offsets, reads.lengths, params, threads)

    def align_one(self, read, params: Params):
        """(pos, strand, dist, second, call) of one read given as str/bytes."""
        r = _bytes(read)
        res = self.align(r, np.array([0, len(r)], np.int64), np.array([len(r)], np.int32), params, 1)
        return (int(res.pos[0]), int(res.strand[0]), int(res.dist[0]), int(res.second[0]), int(res.call[0]))

    def score_log(self, read, params: Params, cap: int = 100000):
        """Locations scored for one read: list of (p, strand, d or INF, d_limit)."""
        r = _bytes(read)
        lp = np.zeros(cap, np.int64)
        ls = np.zeros(cap, np.int8)
        ld = np.zeros(cap, np.int32)
        ll = np.zeros(cap, np.int32)
        k = _load().orc_align_log(self._h, _p(r), len(r), ctypes.byref(params), _p(lp), _p(ls), _p(ld),
                                  _p(ll), cap)
        return [(int(lp[i]), int(ls[i]), int(ld[i]), int(ll[i])) for i in range(k)]
