"""Seeded synthetic genomes, reads and request arrivals.

Inputs only: nothing here computes any step of the alignment method. Both the
CPU oracle's tests and the GPU path's tests and benchmark draw their inputs from
this module, so the two sides see byte-identical data.

The C source (synth.c) is compiled with gcc into libsynth.so beside it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB = os.path.join(_HERE, "libsynth.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile libsynth.so (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Err(ctypes.Structure):
    _fields_ = [("p_sub", ctypes.c_double), ("p_indel", ctypes.c_double), ("indel_max", ctypes.c_int32),
                ("p_sub_long", ctypes.c_double), ("p_indel_long", ctypes.c_double),
                ("indel_max_long", ctypes.c_int32), ("long_thr", ctypes.c_int32)]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, u64, i32, dbl = ctypes.c_int64, ctypes.c_uint64, ctypes.c_int32, ctypes.c_double
        lib.synth_genome_uniform.argtypes = [P, i64, u64]
        lib.synth_genome_uniform.restype = i64
        lib.synth_genome_repeats.argtypes = [P, i64, u64, dbl, dbl, dbl, dbl, dbl, dbl, dbl, i64, i64]
        lib.synth_genome_repeats.restype = i64
        lib.synth_read_lengths.argtypes = [i64, u64, ctypes.c_int, i32, i32, P]
        lib.synth_read_lengths.restype = None
        lib.synth_reads_fill.argtypes = [P, i64, i64, u64, P, P, ctypes.POINTER(_Err), P, P, P, P]
        lib.synth_reads_fill.restype = i64
        lib.synth_arrivals.argtypes = [i64, u64, dbl, dbl, P, P]
        lib.synth_arrivals.restype = None
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


# ------------------------------------------------------------------ genomes

def genome_uniform(G: int, seed: int) -> np.ndarray:
    """i.i.d. uniform A/C/G/T genome of G bases (ASCII uint8)."""
    out = np.empty(G, dtype=np.uint8)
    _load().synth_genome_uniform(_p(out), G, seed)
    return out


def genome_family(G: int, seed: int, copies: int, elem_len: int = 300, div: float = 0.015) -> np.ndarray:
    """Uniform genome of G bases holding `copies` diverged copies (substitutions at rate
    div) of one elem_len-base element at random non-overlapping places: a high-copy
    repeat family, whose reads have as many candidate locations (ASCII uint8)."""
    if copies * elem_len > G:
        raise ValueError("the copies do not fit the genome")
    rng = np.random.default_rng(seed)
    acgt = np.frombuffer(b"ACGT", dtype=np.uint8)
    g = acgt[rng.integers(0, 4, G)]
    elem = rng.integers(0, 4, elem_len)
    for slot in np.sort(rng.choice(G // elem_len, copies, replace=False)):
        c = elem.copy()
        m = rng.random(elem_len) < div
        c[m] = (c[m] + rng.integers(1, 4, int(m.sum()))) % 4
        g[slot * elem_len:(slot + 1) * elem_len] = acgt[c]
    return g


def genome_repeats(G: int, seed: int, f_unique=0.5, f_segdup=0.4, f_tandem=0.1,
                   div_lo=0.01, div_hi=0.03, tandem_mut=0.01,
                   n_frac=0.0, n_run_lo=1000, n_run_hi=100000) -> np.ndarray:
    """Genome with unique blocks, segmental duplicates, tandem arrays and N-runs."""
    out = np.empty(G, dtype=np.uint8)
    _load().synth_genome_repeats(_p(out), G, seed, f_unique, f_segdup, f_tandem,
                                 div_lo, div_hi, tandem_mut, n_frac, n_run_lo, n_run_hi)
    return out


# -------------------------------------------------------------------- reads

@dataclass
class ReadModel:
    """Length and error model of a simulated read set."""
    len_mode: int = 0          # 0 fixed len_a; 1 len_a or len_b 50/50; 2 log-uniform [len_a, len_b)
    len_a: int = 100
    len_b: int = 100
    p_sub: float = 0.005
    p_indel: float = 0.0005
    indel_max: int = 5
    p_sub_long: float = 0.0
    p_indel_long: float = 0.0
    indel_max_long: int = 1
    long_thr: int = 2 ** 31 - 1


@dataclass
class Reads:
    bases: np.ndarray        # uint8, concatenated ASCII
    lengths: np.ndarray      # int32
    offsets: np.ndarray      # int64, n+1 entries (exclusive sum of lengths)
    truth_pos: np.ndarray    # int64 leftmost genome coordinate of the source span
    truth_strand: np.ndarray  # int8 0 forward, 1 reverse complement
    truth_edits: np.ndarray  # int32 events applied

    @property
    def n(self) -> int:
        return int(self.lengths.shape[0])

    def subset(self, idx) -> "Reads":
        idx = np.asarray(idx, dtype=np.int64)
        lens = self.lengths[idx]
        offs = np.zeros(len(idx) + 1, dtype=np.int64)
        np.cumsum(lens, out=offs[1:])
        bases = np.empty(int(offs[-1]), dtype=np.uint8)
        for k, i in enumerate(idx):
            bases[offs[k]:offs[k + 1]] = self.bases[self.offsets[i]:self.offsets[i + 1]]
        return Reads(bases, lens.copy(), offs, self.truth_pos[idx].copy(),
                     self.truth_strand[idx].copy(), self.truth_edits[idx].copy())


def read_lengths(n: int, seed: int, model: ReadModel) -> np.ndarray:
    out = np.empty(n, dtype=np.int32)
    _load().synth_read_lengths(n, seed, model.len_mode, model.len_a, model.len_b, _p(out))
    return out


def simulate_reads(genome: np.ndarray, n: int, seed: int, model: ReadModel) -> Reads:
    """Sample n reads from either strand of `genome` under `model`."""
    genome = np.ascontiguousarray(genome, dtype=np.uint8)
    lens = read_lengths(n, seed, model)
    offs = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lens, out=offs[1:])
    bases = np.empty(int(offs[-1]), dtype=np.uint8)
    tpos = np.empty(n, dtype=np.int64)
    tstr = np.empty(n, dtype=np.int8)
    ted = np.empty(n, dtype=np.int32)
    e = _Err(model.p_sub, model.p_indel, model.indel_max, model.p_sub_long, model.p_indel_long,
             model.indel_max_long, model.long_thr)
    _load().synth_reads_fill(_p(genome), genome.shape[0], n, seed, _p(lens), _p(offs), ctypes.byref(e),
                             _p(bases), _p(tpos), _p(tstr), _p(ted))
    return Reads(bases, lens, offs, tpos, tstr, ted)


def arrivals(n: int, seed: int, rate: float, decades: float = 4.0):
    """Poisson request arrivals (seconds) and request sizes floor(10^(decades*u))."""
    t = np.empty(n, dtype=np.float64)
    k = np.empty(n, dtype=np.int32)
    _load().synth_arrivals(n, seed, rate, decades, _p(t), _p(k))
    return t, k
