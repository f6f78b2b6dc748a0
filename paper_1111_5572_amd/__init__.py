"""snapgpu: SNAP's read-alignment path (arXiv 1111.5572, Section 3) on MI355X.

Thin ctypes binding over the C-ABI library libsnapgpu.so (declared in
include/snapgpu.h). Every step of the path runs in the library's HIP kernels;
this module only marshals arguments. PyTorch supplies device memory and
streams. There is no CPU fallback: if the library is missing, loading fails.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsnapgpu.so")
_lib = None

SNAP_OK, SNAP_EINVAL, SNAP_ENOMEM, SNAP_EDEVICE, SNAP_EBUSY, SNAP_EAGAIN, SNAP_EINTERNAL, SNAP_ETOOBIG = range(8)
NOT_FOUND, SINGLE, MULTIPLE = 0, 1, 2


class SnapError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {strerror(code)} ({code})")


class Params(ctypes.Structure):
    """Table 3 parameters (s is fixed by the index) and the length rules."""
    _fields_ = [(n, ctypes.c_int32) for n in
                ("n_min", "n_cap", "bp_per_seed", "conf_c", "max_hits", "d_max_pct", "bucket")]


class IndexSizes(ctypes.Structure):
    _fields_ = [("genome_len", ctypes.c_uint64), ("seed_len", ctypes.c_int32), ("stride", ctypes.c_int32),
                ("windows", ctypes.c_uint64), ("distinct_keys", ctypes.c_uint64),
                ("table_slots", ctypes.c_uint64), ("position_entries", ctypes.c_uint64),
                ("device_bytes", ctypes.c_uint64), ("device", ctypes.c_int32), ("dup_window", ctypes.c_int32)]


class KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double)]


class Tuning(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("pass1_seeds", "pass1_limit", "final_limit", "lane_max_len",
                                               "exact_rounds", "verify_seeds", "chunk_reads", "workers",
                                               "request_top", "pass1_max_len")]

    def astuple(self):
        return tuple(int(getattr(self, n)) for n, _ in self._fields_)


DEFAULT_EXACT_ROUNDS = 1


def make_tuning(t) -> "Tuning":
    """A Tuning from a Tuning or a tuple of its fields (the trailing exact_rounds,
    verify_seeds, chunk_reads, workers, request_top and pass1_max_len may be left out: 1, 0,
    0, 0, 0 and 0)."""
    if isinstance(t, Tuning):
        return t
    t = tuple(int(x) for x in t)
    if len(t) == 4:
        t = t + (DEFAULT_EXACT_ROUNDS,)
    t = t + (0,) * (10 - len(t))
    return Tuning(*t)


def set_tuning(pass1_seeds: int, pass1_limit: int, final_limit: int = 0, lane_max_len: int = 0,
               exact_rounds: int = DEFAULT_EXACT_ROUNDS, verify_seeds: int = 0, chunk_reads: int = 0,
               workers: int = 0, request_top: int = 0, pass1_max_len: int = 0):
    """Output-invariant pass schedule and verify tiling (see snap_set_tuning); 0 = no cap."""
    _check(lib().snap_set_tuning(ctypes.byref(Tuning(pass1_seeds, pass1_limit, final_limit, lane_max_len,
                                                     exact_rounds, verify_seeds, chunk_reads, workers,
                                                     request_top, pass1_max_len))),
           "snap_set_tuning")


def get_tuning() -> tuple[int, int, int, int, int, int, int, int, int, int]:
    t = Tuning()
    _check(lib().snap_get_tuning(ctypes.byref(t)), "snap_get_tuning")
    return t.astuple()


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_uint64), ("slots", ctypes.c_int32), ("max_waiting", ctypes.c_int32),
                ("batch_reads", ctypes.c_int64), ("batch_bases", ctypes.c_int64), ("max_len", ctypes.c_int32),
                ("d_max", ctypes.c_int32)]


class Result(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("status", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("pos", ctypes.POINTER(ctypes.c_int64)), ("strand", ctypes.POINTER(ctypes.c_int8)),
                ("dist", ctypes.POINTER(ctypes.c_int32)), ("second", ctypes.POINTER(ctypes.c_int32)),
                ("call", ctypes.POINTER(ctypes.c_int8)), ("t_submit", ctypes.c_double),
                ("t_start", ctypes.c_double), ("t_done", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in
                ("slots", "submitted", "completed", "failed", "batches", "waiting", "busy_slots")] + \
               [("slot_device_bytes", ctypes.c_uint64)]


class Counters(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in
                ("passes", "reads", "seed_slots", "hits", "locations", "lv_steps", "second_pass_reads", "requests",
                 "workers", "lv_steps_first", "dup_aliases")]


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run paper_1111_5572_amd.build_library() first")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, u64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_size_t
        L.snap_strerror.argtypes = [ctypes.c_int]
        L.snap_strerror.restype = ctypes.c_char_p
        L.snap_index_build.argtypes = [P, u64, i32, ctypes.POINTER(P)]
        L.snap_index_build.restype = ctypes.c_int
        L.snap_index_build_progress.argtypes = [P, u64, i32, PROGRESS_FN, P, ctypes.POINTER(P)]
        L.snap_index_build_progress.restype = ctypes.c_int
        L.snap_index_build_device.argtypes = [P, u64, i32, P, PROGRESS_FN, P, ctypes.POINTER(P)]
        L.snap_index_build_device.restype = ctypes.c_int
        L.snap_index_build_strided.argtypes = [P, u64, i32, i32, P, PROGRESS_FN, P, ctypes.POINTER(P)]
        L.snap_index_build_strided.restype = ctypes.c_int
        L.snap_index_dup_classes.argtypes = [P, i32, P]
        L.snap_index_dup_classes.restype = ctypes.c_int
        L.snap_debug_dup_download.argtypes = [P, P, u64]
        L.snap_debug_dup_download.restype = ctypes.c_int
        L.snap_debug_index_download.argtypes = [P, i32, P, u64]
        L.snap_debug_index_download.restype = ctypes.c_int
        L.snap_index_free.argtypes = [P]
        L.snap_index_free.restype = ctypes.c_int
        L.snap_index_info.argtypes = [P, ctypes.POINTER(IndexSizes)]
        L.snap_index_info.restype = ctypes.c_int
        L.snap_default_params.argtypes = []
        L.snap_default_params.restype = Params
        L.snap_align_workspace_bytes.argtypes = [P, i64, i64, i32, i32, ctypes.POINTER(Params)]
        L.snap_align_workspace_bytes.restype = sz
        L.snap_align.argtypes = [P, P, P, i64, i32, ctypes.POINTER(Params), P, P, P, P, P, P, sz, P]
        L.snap_align.restype = ctypes.c_int
        L.snap_align_noalloc.argtypes = [P, P, P, i64, i32, ctypes.POINTER(Params), P, P, P, P, P, P]
        L.snap_align_noalloc.restype = ctypes.c_int
        L.snap_align_noalloc_scratch_bytes.argtypes = []
        L.snap_align_noalloc_scratch_bytes.restype = sz
        L.snap_max_limit.argtypes = []
        L.snap_max_limit.restype = i32
        L.snap_debug_host_lookup.argtypes = [P, u64, i32, P, i64, P, P, P, ctypes.POINTER(u64)]
        L.snap_debug_host_lookup.restype = ctypes.c_int
        L.snap_debug_seed_offsets.argtypes = [i32, i32, i32, P]
        L.snap_debug_seed_offsets.restype = i32
        L.snap_profile_begin.argtypes = []
        L.snap_profile_begin.restype = ctypes.c_int
        L.snap_profile_end.argtypes = [ctypes.POINTER(KernelTime), i32, ctypes.POINTER(i32)]
        L.snap_profile_end.restype = ctypes.c_int
        L.snap_profile_counters.argtypes = [ctypes.POINTER(Counters)]
        L.snap_profile_counters.restype = ctypes.c_int
        L.snap_set_tuning.argtypes = [ctypes.POINTER(Tuning)]
        L.snap_set_tuning.restype = ctypes.c_int
        L.snap_get_tuning.argtypes = [ctypes.POINTER(Tuning)]
        L.snap_get_tuning.restype = ctypes.c_int
        L.snap_align_batched.argtypes = [P, P, P, i64, i32, ctypes.POINTER(Params), ctypes.POINTER(Tuning),
                                         P, P, P, P, P, P, sz, P]
        L.snap_align_batched.restype = ctypes.c_int
        L.snap_server_default_config.argtypes = []
        L.snap_server_default_config.restype = ServerConfig
        L.snap_server_create.argtypes = [P, ctypes.POINTER(Params), ctypes.POINTER(ServerConfig),
                                         ctypes.POINTER(Tuning), ctypes.POINTER(P)]
        L.snap_server_create.restype = ctypes.c_int
        L.snap_server_submit.argtypes = [P, P, P, i64, i32, ctypes.POINTER(u64)]
        L.snap_server_submit.restype = ctypes.c_int
        L.snap_server_poll.argtypes = [P, u64, ctypes.POINTER(Result)]
        L.snap_server_poll.restype = ctypes.c_int
        L.snap_server_release.argtypes = [P, u64]
        L.snap_server_release.restype = ctypes.c_int
        L.snap_server_stats.argtypes = [P, ctypes.POINTER(ServerStats)]
        L.snap_server_stats.restype = ctypes.c_int
        L.snap_server_destroy.argtypes = [P]
        L.snap_server_destroy.restype = ctypes.c_int
        L.snap_debug_gather_lines.argtypes = [P, u64, i32, i32, u64, u64, P, P]
        L.snap_debug_gather_lines.restype = ctypes.c_int
        L.snap_debug_copy.argtypes = [P, P, u64, P]
        L.snap_debug_copy.restype = ctypes.c_int
        _lib = L
    return _lib


def strerror(code: int) -> str:
    return lib().snap_strerror(code).decode()


def _check(code: int, what: str):
    if code != SNAP_OK:
        raise SnapError(code, what)


def default_params(**kw) -> Params:
    p = lib().snap_default_params()
    for k, v in kw.items():
        setattr(p, k, int(v))
    return p


def params_from(w) -> Params:
    """From an object with the Table 3 fields (e.g. synth.workloads.Params)."""
    return default_params(n_min=w.n_min, n_cap=w.n_cap, bp_per_seed=w.bp_per_seed, conf_c=w.conf_c,
                          max_hits=w.max_hits, d_max_pct=w.d_max_pct, bucket=w.bucket)


def max_limit() -> int:
    return int(lib().snap_max_limit())


def _np_u8(x) -> np.ndarray:
    if isinstance(x, (bytes, bytearray)):
        return np.frombuffer(bytes(x), dtype=np.uint8)
    if isinstance(x, str):
        return np.frombuffer(x.encode(), dtype=np.uint8)
    return np.ascontiguousarray(x, dtype=np.uint8)


PROGRESS_FN = ctypes.CFUNCTYPE(None, ctypes.c_char_p, ctypes.c_void_p)


class Index:
    """Device-resident seed index of a genome: built on the host (snap_index_build) or,
    with on_device=True, by device kernels on the current stream (snap_index_build_device).
    `progress`, if given, is called with the text of each finished build stage."""

    def __init__(self, genome, seed_len: int = 20, progress=None, on_device: bool = False, stride: int = 1):
        g = _np_u8(genome)
        h = ctypes.c_void_p()
        if stride != 1:
            import torch
            stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
            cb = PROGRESS_FN(lambda stage, ctx: progress(stage.decode())) if progress else PROGRESS_FN()
            _check(lib().snap_index_build_strided(g.ctypes.data, g.shape[0], seed_len, stride, stream, cb, None,
                                                  ctypes.byref(h)), "snap_index_build_strided")
        elif on_device:
            import torch
            stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
            cb = PROGRESS_FN(lambda stage, ctx: progress(stage.decode())) if progress else PROGRESS_FN()
            _check(lib().snap_index_build_device(g.ctypes.data, g.shape[0], seed_len, stream, cb, None,
                                                 ctypes.byref(h)), "snap_index_build_device")
        elif progress is None:
            _check(lib().snap_index_build(g.ctypes.data, g.shape[0], seed_len, ctypes.byref(h)), "snap_index_build")
        else:
            cb = PROGRESS_FN(lambda stage, ctx: progress(stage.decode()))
            _check(lib().snap_index_build_progress(g.ctypes.data, g.shape[0], seed_len, cb, None, ctypes.byref(h)),
                   "snap_index_build_progress")
        self._h = h
        self.seed_len = seed_len
        self.stride = stride
        self.genome_len = int(g.shape[0])

    @property
    def handle(self):
        return self._h

    def download(self, which: str) -> np.ndarray:
        """A copy of one device array: "gcode", "gmask", "table" (slots x 2 uint64) or
        "positions"."""
        sz = self.sizes()
        G = sz["genome_len"]
        shape, dt, idx = {
            "gcode": ((G + 15) // 16 + 4, np.uint32, 0),
            "gmask": ((G + 31) // 32 + 4, np.uint32, 1),
            "table": ((sz["table_slots"], 2), np.uint64, 2),
            "positions": (sz["position_entries"], np.uint32, 3),
        }[which]
        out = np.empty(shape, dtype=dt)
        _check(lib().snap_debug_index_download(self._h, idx, out.ctypes.data, out.nbytes), "snap_debug_index_download")
        return out

    def dup_classes(self, window: int, stream=None):
        """Attach exact-duplicate classes of `window`-base windows (snap_index_dup_classes)."""
        _check(lib().snap_index_dup_classes(self._h, int(window), _stream_ptr(stream)), "snap_index_dup_classes")

    def download_dup_classes(self) -> np.ndarray:
        """The class array (one uint32 per genome position)."""
        G = self.sizes()["genome_len"]
        out = np.empty(G, dtype=np.uint32)
        _check(lib().snap_debug_dup_download(self._h, out.ctypes.data, G), "snap_debug_dup_download")
        return out

    def sizes(self) -> dict:
        s = IndexSizes()
        _check(lib().snap_index_info(self._h, ctypes.byref(s)), "snap_index_info")
        return {n: int(getattr(s, n)) for n, _ in s._fields_ if not n.startswith("reserved")}

    def close(self):
        if self._h:
            lib().snap_index_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Alignment:
    pos: "torch.Tensor"      # int64
    strand: "torch.Tensor"   # int8
    dist: "torch.Tensor"     # int32
    second: "torch.Tensor"   # int32
    call: "torch.Tensor"     # int8

    def numpy(self):
        return tuple(t.cpu().numpy() for t in (self.pos, self.strand, self.dist, self.second, self.call))


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def workspace_bytes(index: Index, n_reads: int, total_bases: int, max_len: int, d_max: int, params: Params) -> int:
    return int(lib().snap_align_workspace_bytes(index.handle, n_reads, total_bases, max_len, d_max,
                                                ctypes.byref(params)))


def align(index: Index, reads, lengths, d_max: int, params: Params | None = None, out: Alignment | None = None,
          workspace=None, stream=None, max_len: int | None = None, batched: bool = False,
          tuning: "Tuning | tuple | None" = None) -> Alignment:
    """snap_align (or snap_align_batched when batched=True) on device tensors:
    reads (uint8, concatenated ASCII) and lengths (int32). Returns device tensors;
    they are valid once `stream` is synchronized."""
    import torch
    params = params or default_params()
    n = int(lengths.shape[0])
    dev = lengths.device
    if out is None:
        out = Alignment(torch.empty(n, dtype=torch.int64, device=dev), torch.empty(n, dtype=torch.int8, device=dev),
                        torch.empty(n, dtype=torch.int32, device=dev), torch.empty(n, dtype=torch.int32, device=dev),
                        torch.empty(n, dtype=torch.int8, device=dev))
    if workspace is None:
        ml = int(max_len) if max_len is not None else (int(lengths.max().item()) if n else 0)
        wb = workspace_bytes(index, n, int(reads.numel()), ml, d_max, params)
        if wb == 0 and n:
            raise SnapError(SNAP_EINVAL, "snap_align_workspace_bytes")
        workspace = torch.empty(max(wb, 256), dtype=torch.uint8, device=dev)
    if batched:
        if isinstance(tuning, tuple):
            tuning = make_tuning(tuning)
        tp = ctypes.byref(tuning) if tuning is not None else None
        code = lib().snap_align_batched(index.handle, reads.data_ptr(), lengths.data_ptr(), n, d_max,
                                        ctypes.byref(params), tp, out.pos.data_ptr(), out.strand.data_ptr(),
                                        out.dist.data_ptr(), out.second.data_ptr(), out.call.data_ptr(),
                                        workspace.data_ptr(), workspace.numel(), _stream_ptr(stream))
        _check(code, "snap_align_batched")
        return out
    code = lib().snap_align(index.handle, reads.data_ptr(), lengths.data_ptr(), n, d_max, ctypes.byref(params),
                            out.pos.data_ptr(), out.strand.data_ptr(), out.dist.data_ptr(), out.second.data_ptr(),
                            out.call.data_ptr(), workspace.data_ptr(), workspace.numel(), _stream_ptr(stream))
    _check(code, "snap_align")
    return out


def noalloc_scratch_bytes() -> int:
    return int(lib().snap_align_noalloc_scratch_bytes())


def align_noalloc(index: Index, reads, lengths, d_max: int, params: Params, out: Alignment, stream=None) -> Alignment:
    """snap_align_noalloc: snap_align on the library's fixed per-device scratch array (no
    workspace, no device allocation); the caller provides the output tensors."""
    n = int(lengths.shape[0])
    code = lib().snap_align_noalloc(index.handle, reads.data_ptr(), lengths.data_ptr(), n, d_max,
                                    ctypes.byref(params), out.pos.data_ptr(), out.strand.data_ptr(),
                                    out.dist.data_ptr(), out.second.data_ptr(), out.call.data_ptr(),
                                    _stream_ptr(stream))
    _check(code, "snap_align_noalloc")
    return out


# ---------------------------------------------------------------- host-only checks

def debug_host_lookup(genome, seed_len: int, queries: list[str]):
    """Build the table in host memory and look seeds up with the device's probe
    sequence: returns (windows, [(forward hits, reverse hits, first forward hit)])."""
    g = _np_u8(genome)
    q = _np_u8("".join(queries))
    nq = len(queries)
    fwd = np.zeros(max(nq, 1), np.int64)
    rev = np.zeros(max(nq, 1), np.int64)
    first = np.zeros(max(nq, 1), np.int64)
    win = ctypes.c_uint64()
    _check(lib().snap_debug_host_lookup(g.ctypes.data, g.shape[0], seed_len, q.ctypes.data, nq, fwd.ctypes.data,
                                        rev.ctypes.data, first.ctypes.data, ctypes.byref(win)),
           "snap_debug_host_lookup")
    return int(win.value), [(int(fwd[i]), int(rev[i]), int(first[i])) for i in range(nq)]


def debug_seed_offsets(L: int, s: int, n: int) -> list[int]:
    out = np.zeros(64, np.int32)
    k = lib().snap_debug_seed_offsets(L, s, n, out.ctypes.data)
    return [int(v) for v in out[:k]]


def server_config(**kw) -> ServerConfig:
    c = lib().snap_server_default_config()
    for k, v in kw.items():
        setattr(c, k, int(v))
    return c


class Server:
    """snap_server: continuous-batching request server (host arrays in and out)."""

    def __init__(self, index: Index, d_max: int, params: Params | None = None, tuning=None, **cfg):
        self.index = index
        self.params = params or default_params()
        self.cfg = server_config(d_max=d_max, **cfg)
        tp = None
        if tuning is not None:
            tp = ctypes.byref(make_tuning(tuning))
        h = ctypes.c_void_p()
        _check(lib().snap_server_create(index.handle, ctypes.byref(self.params), ctypes.byref(self.cfg), tp,
                                        ctypes.byref(h)), "snap_server_create")
        self._h = h

    def submit(self, bases: np.ndarray, lengths: np.ndarray) -> int:
        """Queue a request; returns its ticket (raises SnapError, e.g. SNAP_EBUSY)."""
        bases = np.ascontiguousarray(bases, dtype=np.uint8)
        lengths = np.ascontiguousarray(lengths, dtype=np.int32)
        t = ctypes.c_uint64()
        _check(lib().snap_server_submit(self._h, bases.ctypes.data, lengths.ctypes.data, lengths.shape[0],
                                        self.cfg.d_max, ctypes.byref(t)), "snap_server_submit")
        return int(t.value)

    def poll(self, ticket: int, release: bool = True):
        """None while pending; else (pos, strand, dist, second, call, (t_submit, t_start, t_done))."""
        r = Result()
        code = lib().snap_server_poll(self._h, ticket, ctypes.byref(r))
        if code == SNAP_EAGAIN:
            return None
        _check(code, "snap_server_poll")
        _check(r.status, "server request")
        n = int(r.n)
        arrs = tuple(np.ctypeslib.as_array(p, shape=(n,)).copy() if n else np.zeros(0, dt)
                     for p, dt in ((r.pos, np.int64), (r.strand, np.int8), (r.dist, np.int32),
                                   (r.second, np.int32), (r.call, np.int8)))
        times = (float(r.t_submit), float(r.t_start), float(r.t_done))
        if release:
            _check(lib().snap_server_release(self._h, ticket), "snap_server_release")
        return arrs + (times,)

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().snap_server_stats(self._h, ctypes.byref(st)), "snap_server_stats")
        return {n: int(getattr(st, n)) for n, _ in st._fields_}

    def close(self):
        if self._h:
            lib().snap_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def profile_begin():
    _check(lib().snap_profile_begin(), "snap_profile_begin")


def profile_end() -> dict:
    """{kernel name: (launches, total device ms)} since profile_begin."""
    arr = (KernelTime * 64)()
    n = ctypes.c_int32()
    _check(lib().snap_profile_end(arr, 64, ctypes.byref(n)), "snap_profile_end")
    return {arr[i].name.decode(): (int(arr[i].launches), float(arr[i].total_ms)) for i in range(n.value)}


def profile_counters() -> dict:
    c = Counters()
    _check(lib().snap_profile_counters(ctypes.byref(c)), "snap_profile_counters")
    return {n: int(getattr(c, n)) for n, _ in c._fields_}


def debug_gather_lines(buf, nbytes: int, line_bytes: int, rounds: int, threads: int, seed: int, sink, stream=None):
    _check(lib().snap_debug_gather_lines(buf.data_ptr(), nbytes, line_bytes, rounds, threads, seed, sink.data_ptr(),
                                         _stream_ptr(stream)), "snap_debug_gather_lines")


def debug_copy(src, dst, nbytes: int, stream=None):
    _check(lib().snap_debug_copy(src.data_ptr(), dst.data_ptr(), nbytes, _stream_ptr(stream)), "snap_debug_copy")


def build_library(force: bool = True) -> str:
    """Compile libsnapgpu.so for gfx950 (see build.py)."""
    from .build import build as _b
    return _b(force=force)
