"""Autotuner for the output-invariant knobs of snap_align / snap_align_batched.

The knobs (snap_tuning): the seeds and verify limit of the first pass, the first
verify limit of the final pass, the verify tile bound (reads up to that length
get one lane per location, longer ones a wave per location) and the number of
replay rounds that ask for single locations, the seed slots whose locations
the first verification covers, and, for reads of mixed lengths, the length above
which reads take every seed slot in one complete pass. Outputs do
not depend on them; only the time does. The tuner aligns a sample of the batch
with each candidate, keeps the fastest, and records it in a JSON table keyed by
the batch's read-length class.
"""
from __future__ import annotations

import json
import os
import time

import numpy as np

from . import align, default_params, make_tuning

TABLE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_table.json")

# (pass1_seeds, pass1_limit, final_limit, lane_max_len, exact_rounds, verify_seeds); 0 = no cap / default
CANDIDATES = [
    (0, 0, 0, 0, 2, 0),
    (6, 0, 0, 0, 2, 0),
    (4, 5, 5, 0, 1, 0),
    (5, 5, 5, 0, 1, 0),
    (5, 6, 6, 0, 1, 0),
    (5, 6, 6, 0, 1, 3),
    (5, 6, 6, 0, 1, 4),
    (5, 5, 5, 0, 1, 3),
    (6, 6, 6, 0, 1, 3),
    (6, 6, 6, 0, 1, 4),
    (5, 8, 8, 0, 1, 3),
    (6, 5, 5, 0, 1, 0),
    (5, 5, 5, 256, 1, 0),
    # larger limits and more exact rounds, for longer reads and larger d_max
    (5, 6, 6, 0, 2, 0),
    (5, 6, 6, 0, 3, 0),
    (5, 8, 8, 0, 1, 0),
    (5, 8, 8, 0, 2, 0),
    (5, 10, 10, 0, 2, 0),
    (4, 6, 6, 0, 2, 0),
    (6, 8, 8, 0, 2, 0),
    (5, 4, 4, 0, 2, 0),
    (5, 6, 6, 0, 5, 0),
    (5, 6, 6, 0, 8, 0),
    (5, 4, 4, 0, 5, 0),
    (5, 8, 8, 0, 5, 0),
]


def candidates_for(lengths: np.ndarray, batched: bool, base=None) -> list:
    """The candidates for a batch: `base` (CANDIDATES), and for plain calls on reads of mixed
    lengths two of them again with pass1_max_len at each quartile of the lengths below the
    longest (the reads above it then take every seed slot in one complete pass)."""
    cands = list(base or CANDIDATES)
    if batched or len(lengths) == 0:
        return cands
    top = int(np.max(lengths))
    cuts = sorted({int(np.percentile(lengths, q)) for q in (25, 50, 75)} - {top})
    for b in ((5, 6, 6, 0, 1, 0), (5, 7, 7, 0, 5, 0)):
        cands += [b + (0, 0, 0, cut) for cut in cuts if 0 < cut < top]
    return cands


def length_class(lengths: np.ndarray) -> str:
    """Key of the tuning table: read-length span of the batch in powers of two."""
    if len(lengths) == 0:
        return "empty"
    lo = int(np.percentile(lengths, 5))
    hi = int(np.percentile(lengths, 95))
    b = lambda x: 1 << max(0, int(x).bit_length() - 1)
    return f"{b(max(lo, 1))}-{b(max(hi, 1))}"


def load_table(path: str = TABLE_PATH) -> dict:
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def lookup_entry(lengths: np.ndarray, batched: bool, path: str = TABLE_PATH):
    """The recorded entry (tuning, timings, sample) for this length class, or None."""
    e = load_table(path).get(("batched:" if batched else "plain:") + length_class(lengths))
    if e and 4 <= len(e.get("tuning", ())) <= 10:
        return e
    return None


def lookup(lengths: np.ndarray, batched: bool, path: str = TABLE_PATH):
    """The recorded tuning for this length class, or None."""
    e = lookup_entry(lengths, batched, path)
    return tuple(e["tuning"]) if e else None


def tune(index, reads_dev, lengths_dev, d_max: int, params=None, batched: bool = True, sample_reads: int = 200_000,
         candidates=None, repeats: int = 2, table_path: str | None = TABLE_PATH, log=None) -> dict:
    """Time each candidate on the first `sample_reads` reads (already on the device)
    and return {"tuning": best, "ms": {candidate: ms}}; record it in the table."""
    import torch
    params = params or default_params()
    lengths_host = lengths_dev.cpu().numpy()
    n = min(int(lengths_dev.shape[0]), sample_reads)
    nb = int(lengths_host[:n].astype(np.int64).sum())
    rb, ln = reads_dev[:nb], lengths_dev[:n]
    max_len = int(lengths_host[:n].max()) if n else 0
    candidates = candidates or candidates_for(lengths_host[:n], batched)
    out = None
    timings = {}
    stream = torch.cuda.current_stream()
    for cand in candidates:
        tp = make_tuning(cand)
        out = align(index, rb, ln, d_max, params, out=out, max_len=max_len, batched=True, tuning=tp) \
            if batched else _plain(index, rb, ln, d_max, params, out, max_len, cand)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(repeats):
            out = align(index, rb, ln, d_max, params, out=out, max_len=max_len, batched=True, tuning=tp) \
                if batched else _plain(index, rb, ln, d_max, params, out, max_len, cand)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / repeats
        timings[",".join(map(str, cand))] = round(ms, 3)
        if log:
            log(f"autotune {'batched' if batched else 'plain'} {cand}: {ms:.2f} ms on {n} reads")
    best = min(timings, key=timings.get)
    result = {"tuning": [int(x) for x in best.split(",")], "ms": timings, "sample_reads": n,
              "class": length_class(lengths_host), "when": time.strftime("%Y-%m-%d %H:%M:%S")}
    if table_path:
        tab = load_table(table_path)
        tab[("batched:" if batched else "plain:") + result["class"]] = result
        tmp = table_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(tab, f, indent=1, sort_keys=True)
        os.replace(tmp, table_path)
    return result


def _plain(index, rb, ln, d_max, params, out, max_len, cand):
    from . import get_tuning, set_tuning
    old = get_tuning()
    try:
        set_tuning(*cand)
        return align(index, rb, ln, d_max, params, out=out, max_len=max_len)
    finally:
        set_tuning(*old)
