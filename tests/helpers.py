"""Shared helpers for the GPU parity tests."""
import sys

import numpy as np

FIELDS = ("pos", "strand", "dist", "second", "call")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_align(snapgpu, index, reads, d_max, params, workspace_bytes=None, stream=None):
    """Align synth.Reads on cuda:0; returns numpy outputs."""
    import torch
    dev = torch.device("cuda:0")
    rb = torch.from_numpy(np.ascontiguousarray(reads.bases)).to(dev)
    ln = torch.from_numpy(np.ascontiguousarray(reads.lengths)).to(dev)
    ws = None
    if workspace_bytes is not None:
        ws = torch.empty(workspace_bytes, dtype=torch.uint8, device=dev)
    out = snapgpu.align(index, rb, ln, d_max, params, workspace=ws, stream=stream,
                        max_len=int(reads.lengths.max()) if reads.n else 0)
    torch.cuda.synchronize()
    return out.numpy()


def oracle_threads():
    """Worker threads for the oracle: the host cores, at most 16 (one GPU's share of a box)."""
    import os
    return max(1, min(16, os.cpu_count() or 1))


def oracle_align(oracle_mod, oix, reads, wparams, threads=None):
    res = oix.align_reads(reads, oracle_mod.params_from(wparams), threads=threads or oracle_threads())
    return res.fields()


def compare(gpu, orc, reads=None, label="", limit=8):
    """Element-wise comparison of the five outputs; returns a mismatch report."""
    n = len(orc[0])
    bad = np.zeros(n, dtype=bool)
    for g, o in zip(gpu, orc):
        bad |= (np.asarray(g).astype(np.int64) != np.asarray(o).astype(np.int64))
    idx = np.nonzero(bad)[0]
    lines = [f"{label}: {len(idx)} of {n} reads differ"]
    for i in idx[:limit]:
        gi = tuple(int(np.asarray(x)[i]) for x in gpu)
        oi = tuple(int(np.asarray(x)[i]) for x in orc)
        extra = ""
        if reads is not None:
            extra = f" len={int(reads.lengths[i])} truth=({int(reads.truth_pos[i])},{int(reads.truth_strand[i])})"
        lines.append(f"  read {i}: gpu={gi} oracle={oi}{extra}")
    return len(idx), "\n".join(lines)
