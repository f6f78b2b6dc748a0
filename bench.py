#!/usr/bin/env python3
"""Benchmark of the read-alignment path on one MI355X.

One step = snap_align over the whole read batch of the workload (all reads
resident in HBM, index resident): seed probe, candidate gathering and dedupe,
bounded edit-distance verification and the best / second-best call.

Prints ONE JSON line: reads/s (whole job), Gbases/s, the roofline of the
dominant kernel measured with HIP events on its launch stream during the timed
steps, and the CPU oracle timed on a bounded sample of the same reads on the
host cores. The GPU outputs of that sample are checked bit-exact against the
oracle before the line is printed.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# 256 CUs x 64 lanes x 2.4 GHz, one 32-bit integer op per lane per cycle
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12

# Algorithmic bytes / ops per unit, per kernel: what each unit must move or compute.
PROBE_BYTES_PER_SLOT = 128 + 32       # one 128-byte bucket line read, one 32-byte probe record written
GATHER_BYTES_PER_SLOT = 32            # probe record read
GATHER_BYTES_PER_HIT = 4 + 8          # position read, hit record written
DEDUPE_BYTES_PER_HIT = 8              # hit record read
DEDUPE_BYTES_PER_LOC = 12             # location key + seed mask written
VERIFY_OPS_PER_STEP = 30              # integer ops per diagonal extension (neighbour max, bounds, one 16-base compare)
SELECT_OPS_PER_VISIT = 4              # integer ops per location looked at by a selection (and + popcount, compare + select)


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


INDEX_ON_HOST = False   # --host-index
INDEX_STRIDE = 1        # --stride


def build_index(g, seed_len):
    """Device index of the genome, built by the library's device kernels (or, with
    --host-index, on the host, logging each finished stage: minutes for a large genome;
    with --stride, the strided index of Section 3.1's footnote)."""
    import paper_1111_5572_amd as snapgpu
    t0 = time.time()
    report = lambda stage: log(f"  index: {stage} ({time.time() - t0:.3f}s)")
    return snapgpu.Index(g, seed_len, progress=report, on_device=not INDEX_ON_HOST, stride=INDEX_STRIDE)


HMAX_SWEEP = (10, 25, 50, 100, 200, 300, 500, 1000, 2000)


def accuracy_of(out, reads, tol=32):
    """The paper's Section 2 metrics for simulated reads: aligned = share of reads given a
    single (confident) location; errors = share of those whose strand differs from the
    read's source or whose position is more than `tol` bases from it."""
    pos, strand, _, _, call = out
    single = call == 1
    wrong = single & ((strand != reads.truth_strand) | (np.abs(pos - reads.truth_pos) > tol))
    n_single = int(single.sum())
    return {"aligned_pct": round(100.0 * n_single / max(reads.n, 1), 3),
            "error_pct": round(100.0 * int(wrong.sum()) / max(n_single, 1), 4)}


def bench_accuracy(args, w, dev):
    """The h_max trade-off (Section 4's figure on h_max: more candidate locations per seed
    align more reads with fewer errors, at lower throughput): 125 bp reads with a 2% error
    rate (1.8% substitutions, 0.2% indels of 1-5 bases) on the workload's genome, d_max 8,
    aligned and error rates against the reads' source and reads/s for each h_max."""
    import torch
    import synth
    import paper_1111_5572_amd as snapgpu
    from dataclasses import replace
    g = w.make_genome()
    model = synth.ReadModel(len_mode=0, len_a=125, len_b=125, p_sub=0.018, p_indel=0.002, indel_max=5)
    n = args.reads or 1_000_000
    t = time.time()
    reads = synth.simulate_reads(g, n, 105, model)
    log(f"genome {w.name}: {len(g)} bases; {n} reads of 125 bp in {time.time() - t:.1f}s")
    gix = build_index(g, w.params.seed_len)
    rb = torch.from_numpy(reads.bases).to(dev)
    ln = torch.from_numpy(reads.lengths).to(dev)
    from paper_1111_5572_amd import autotune
    tuning = autotune.lookup(reads.lengths, batched=False)
    if tuning:
        snapgpu.set_tuning(*tuning)
    log(f"schedule {tuning or 'library default'}")
    stream = torch.cuda.current_stream()
    import oracle
    t = time.time()
    oix = oracle.Index(g, w.params.seed_len, threads=oracle_threads())
    log(f"oracle index in {time.time() - t:.1f}s")
    rng = np.random.default_rng(9)
    rows = []
    out = None
    for h in HMAX_SWEEP:
        p = snapgpu.params_from(replace(w.params, max_hits=h, d_max=8))
        out = snapgpu.align(gix, rb, ln, 8, p, out=out, max_len=125)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(max(1, args.steps)):
            out = snapgpu.align(gix, rb, ln, 8, p, out=out, max_len=125)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / max(1, args.steps)
        got = out.numpy()
        idx = np.unique(rng.integers(0, n, min(n, 3000)))
        res = oix.align_reads(reads.subset(idx), oracle.params_from(replace(w.params, max_hits=h, d_max=8)),
                              threads=oracle_threads())
        mism = sum(int(np.count_nonzero(np.asarray(a)[idx].astype(np.int64) != np.asarray(b).astype(np.int64)))
                   for a, b in zip(got, res.fields()))
        if mism:
            print(json.dumps({"error": f"h_max {h}: GPU differs from the oracle on {mism} fields"}), flush=True)
            sys.exit(1)
        row = {"h_max": h, **accuracy_of(got, reads), "reads_per_s": round(n / (ms / 1e3), 1),
               "ms_per_step": round(ms, 3), "oracle_sample": int(len(idx))}
        log(f"h_max {h}: {row}")
        rows.append(row)
    gix.close()
    oix.close()
    print(json.dumps({"metric": "h_max trade-off", "unit": "aligned %, error %, reads/s", "n_gpus": 1,
                      "steps": max(1, args.steps), "data": "synthetic (seeded genome and simulated reads)",
                      "config": {"workload": w.name, "genome_bases": len(g), "reads": n, "read_len": 125,
                                 "errors": "1.8% substitutions, 0.2% indels (1-5)", "d_max": 8,
                                 "conf_c": w.params.conf_c, "seed_len": w.params.seed_len,
                                 "correct": "same strand, |pos - source| <= 32",
                                 "schedule": list(tuning) if tuning else None},
                      "rows": rows}), flush=True)


# Section 2's tables: (table, read length, error rate, reads, share of erroneous bases in indels)
ACCURACY_GRID = [
    ("Table 1", 100, 0.02, 200_000, 0.1), ("Table 1", 100, 0.05, 200_000, 0.1), ("Table 1", 100, 0.10, 200_000, 0.1),
    ("Table 1", 200, 0.02, 200_000, 0.1), ("Table 1", 200, 0.05, 200_000, 0.1), ("Table 1", 200, 0.10, 200_000, 0.1),
    ("Table 2", 1000, 0.02, 20_000, 0.2), ("Table 2", 1000, 0.05, 20_000, 0.2), ("Table 2", 1000, 0.10, 20_000, 0.2),
    ("Table 2", 10000, 0.02, 2_000, 0.2), ("Table 2", 10000, 0.05, 2_000, 0.2), ("Table 2", 10000, 0.10, 1_000, 0.2),
]
INDEL_MEAN_LEN = 57 / 31   # mean of the truncated geometric(1/2) indel length on 1..5


def grid_dmax(L, err):
    """d_max of a grid cell: 1.5 times the expected edits, at least 8, within the largest
    limit the verify kernels take (d_max + c - 1 <= 1023)."""
    return int(min(1022, max(8, -(-15 * err * L // 10))))


def bench_accuracy_grid(args, w, dev):
    """The metrics of Section 2's Tables 1 and 2 on the stand-in genome: for 100 / 200 bp
    reads (Table 1) and 1 kb / 10 kb reads (Table 2, 20% of the erroneous bases in indels)
    at 2 / 5 / 10% errors, the share of reads aligned confidently (a single call), the
    share of those more than 32 bases from their source or on the other strand, and
    reads/s; each cell's GPU outputs are checked bit-exact on a seeded sample against the
    oracle."""
    import torch
    import synth
    import oracle
    import paper_1111_5572_amd as snapgpu
    from dataclasses import replace
    g = w.make_genome()
    gix = build_index(g, w.params.seed_len)
    t = time.time()
    oix = oracle.Index(g, w.params.seed_len, threads=oracle_threads())
    log(f"oracle index in {time.time() - t:.1f}s")
    rng = np.random.default_rng(8)
    rows = []
    for k, (table, L, err, n, indel_share) in enumerate(ACCURACY_GRID):
        n = max(1, n // max(1, args.grid_scale))
        p_indel = err * indel_share / INDEL_MEAN_LEN
        model = synth.ReadModel(len_mode=0, len_a=L, len_b=L, p_sub=err * (1 - indel_share), p_indel=p_indel,
                                indel_max=5)
        reads = synth.simulate_reads(g, n, 200 + k, model)
        d_max = grid_dmax(L, err)
        wp = replace(w.params, d_max=d_max, d_max_pct=0)
        p = snapgpu.params_from(wp)
        rb = torch.from_numpy(reads.bases).to(dev)
        ln = torch.from_numpy(reads.lengths).to(dev)
        out = snapgpu.align(gix, rb, ln, d_max, p, max_len=L)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(max(1, args.steps)):
            out = snapgpu.align(gix, rb, ln, d_max, p, out=out, max_len=L)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / max(1, args.steps)
        got = out.numpy()
        # oracle sample: bit-exact on all five outputs
        ns = int(min(n, 2000 if L <= 200 else (200 if L <= 1000 else 16)))
        idx = np.unique(rng.integers(0, n, ns))
        res = oix.align_reads(reads.subset(idx), oracle.params_from(wp), threads=oracle_threads())
        mism = sum(int(np.count_nonzero(np.asarray(a)[idx].astype(np.int64) != np.asarray(b).astype(np.int64)))
                   for a, b in zip(got, res.fields()))
        if mism:
            print(json.dumps({"error": f"{table} L={L} err={err}: GPU differs from the oracle on {mism} fields"}),
                  flush=True)
            sys.exit(1)
        row = {"table": table, "read_len": L, "error_rate": err, "reads": n, "d_max": d_max,
               **accuracy_of(got, reads), "reads_per_s": round(n / sec, 1), "oracle_sample": int(len(idx))}
        log(f"{row}")
        rows.append(row)
        del rb, ln, out
    gix.close()
    oix.close()
    print(json.dumps({"metric": "aligned and error rates (Section 2's tables)", "unit": "%, reads/s", "n_gpus": 1,
                      "steps": max(1, args.steps), "data": "synthetic (seeded genome and simulated reads)",
                      "config": {"workload": w.name, "genome_bases": len(g), "seed_len": w.params.seed_len,
                                 "conf_c": w.params.conf_c, "max_hits": w.params.max_hits,
                                 "errors": "Table 1: 90% of erroneous bases substituted, 10% in indels of 1-5; "
                                           "Table 2: 80% / 20%",
                                 "d_max": "min(1022, max(8, ceil(1.5 * error rate * L)))",
                                 "correct": "same strand, |pos - source| <= 32"},
                      "rows": rows}), flush=True)


def bench_gather(args, dev):
    """The random-line gather ceiling: 32 / 64 / 128-byte lines read at pseudo-random
    places of a `--gather-gb` GB device buffer (the probe's bucket lines, the position
    reads), GB/s of lines delivered, beside the 8 TB/s HBM peak."""
    import torch
    import paper_1111_5572_amd as snapgpu
    nbytes = int(args.gather_gb * (1 << 30)) // 128 * 128
    buf = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    threads = 1 << 22
    sink = torch.empty(threads, dtype=torch.int32, device=dev)
    rows = []
    for line in (32, 64, 128):
        rounds = 64
        snapgpu.debug_gather_lines(buf, nbytes, line, rounds, threads, 1, sink)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 5
        e0.record()
        for r in range(reps):
            snapgpu.debug_gather_lines(buf, nbytes, line, rounds, threads, 2 + r, sink)
        e1.record()
        torch.cuda.synchronize()
        sec = e0.elapsed_time(e1) / 1e3 / reps
        moved = threads * rounds * 16
        row = {"line_bytes": line, "bytes_per_launch": moved, "ms": round(sec * 1e3, 3),
               "gb_per_s": round(moved / sec / 1e9, 1), "frac_of_hbm_peak": round(moved / sec / 1e9 / HBM_PEAK_GBS, 4)}
        log(f"gather {row}")
        rows.append(row)
    print(json.dumps({"metric": "random-line gather ceiling", "unit": "GB/s", "n_gpus": 1,
                      "config": {"buffer_bytes": nbytes, "threads": threads, "rounds": 64}, "rows": rows}), flush=True)


def bench_index(args, w):
    """The index build alone: the workload's genome indexed --steps times (after one
    untimed build); one JSON line with the mean build time (host-to-device copy of the
    genome included)."""
    import torch
    g = w.make_genome()
    log(f"genome {w.name}: {len(g)} bases")
    times = []
    for i in range(1 + max(1, args.steps)):
        torch.cuda.synchronize()
        t = time.time()
        ix = build_index(g, w.params.seed_len)
        torch.cuda.synchronize()
        dt = time.time() - t
        sizes = ix.sizes()
        ix.close()
        if i:
            times.append(dt)
        log(f"build {i}{' (untimed)' if i == 0 else ''}: {dt:.3f}s")
    mean = sum(times) / len(times)
    print(json.dumps({"metric": "index build", "value": round(mean, 4), "unit": "s", "higher_is_better": False,
                      "n_gpus": 1, "steps": len(times), "index_build": "host" if INDEX_ON_HOST else "device",
                      "config": {"workload": w.name, "genome_bases": len(g), "seed_len": w.params.seed_len},
                      "sizes": sizes, "windows_per_s": round(sizes["windows"] / mean)}), flush=True)


def roofline_of(kern, ctr, prefer=None, method=None):
    """Roofline entry of the dominant kernel (or `prefer` if given).

    For a verify kernel the work is Algorithm 1's own diagonal extensions when `method`
    (the oracle's count per read on a sample of the batch, each call at its own limit)
    is given: the batch's total, reads x extensions per read, shared among the verify
    kernels in proportion to the extensions each ran. The extensions the kernel ran
    (speculative ones included) give `achieved_executed` beside it."""
    if prefer is not None and prefer not in kern:
        return None
    dom = prefer if prefer in kern else max(kern.items(), key=lambda kv: kv[1][1])[0]
    launches, total_ms = kern[dom]
    avg_s = total_ms / 1000.0 / launches
    per_launch = 1.0 / launches
    extra = {}
    if dom == "probe":
        bound, unit, peak = "hbm", "GB/s", HBM_PEAK_GBS
        work = ctr["seed_slots"] * PROBE_BYTES_PER_SLOT * per_launch / 1e9
    elif dom == "gather":
        bound, unit, peak = "hbm", "GB/s", HBM_PEAK_GBS
        work = (ctr["seed_slots"] * GATHER_BYTES_PER_SLOT + ctr["hits"] * GATHER_BYTES_PER_HIT) * per_launch / 1e9
    elif dom.startswith("dedupe"):
        bound, unit, peak = "hbm", "GB/s", HBM_PEAK_GBS
        work = (ctr["hits"] * DEDUPE_BYTES_PER_HIT + ctr["locations"] * DEDUPE_BYTES_PER_LOC) * per_launch / 1e9
    elif dom.startswith("verify"):
        # the first verification's diagonal extensions are counted on their own; the
        # kernels that verify requested locations share the rest, split by their time
        bound, unit, peak = "alu", "TOP/s", VALU_PEAK_TOPS
        first = ctr.get("lv_steps_first", 0)
        if dom in ("verify", "verify_steal"):
            ran = first
        else:
            req = [k for k in kern if k.startswith("verify") and k not in ("verify", "verify_steal")]
            vt = sum(kern[k][1] for k in req)
            ran = (ctr["lv_steps"] - first) * (total_ms / vt if vt > 0 else 1.0)
        executed = ran * VERIFY_OPS_PER_STEP * per_launch / 1e12
        extra = {"ops_per_extension": VERIFY_OPS_PER_STEP,
                 "achieved_executed": round(executed / avg_s, 3),
                 "frac_executed": round(executed / avg_s / peak, 5),
                 "extensions_per_read_executed": round(ctr["lv_steps"] / max(ctr["reads"], 1), 2)}
        if method:
            own = method["lv_extensions_per_read"] * ctr["reads"] * (ran / max(ctr["lv_steps"], 1))
            work = own * VERIFY_OPS_PER_STEP * per_launch / 1e12
            extra["work"] = "Algorithm 1's own diagonal extensions (oracle sample, each call at its own limit)"
            extra["extensions_per_read_method"] = method["lv_extensions_per_read"]
        else:
            work = executed
            extra["work"] = "diagonal extensions the kernel ran (no oracle sample in this run)"
    elif dom.startswith("replay"):
        # Algorithm 1's control: each selection of "the unscored location with the most seeds
        # hitting" looks at every candidate location (the oracle's count on the sample),
        # shared among the replay kernels in proportion to their time
        bound, unit, peak = "alu", "TOP/s", VALU_PEAK_TOPS
        rep = [k for k in kern if k.startswith("replay")]
        rt = sum(kern[k][1] for k in rep)
        if method and "select_visits_per_read" in method:
            work = (method["select_visits_per_read"] * ctr["reads"] * (total_ms / rt if rt > 0 else 1.0)
                    * SELECT_OPS_PER_VISIT * per_launch / 1e12)
            extra = {"work": "Algorithm 1's own selection scans (oracle sample) x 4 ops per location looked at",
                     "ops_per_visit": SELECT_OPS_PER_VISIT,
                     "select_visits_per_read_method": method["select_visits_per_read"]}
        else:
            work = None
            extra = {"work": "no oracle sample in this run"}
    else:
        bound, unit, peak = "hbm", "GB/s", HBM_PEAK_GBS
        work = None
    if work is None:
        return {"bound": bound, "kernel": dom, "achieved": None, "peak": peak, "unit": unit, "frac": None,
                "avg_launch_ms": round(total_ms / launches, 4), "launches": launches, **extra}
    achieved = work / avg_s
    return {"bound": bound, "kernel": dom, "achieved": round(achieved, 3), "peak": peak, "unit": unit,
            "frac": round(achieved / peak, 5), "avg_launch_ms": round(total_ms / launches, 4), "launches": launches,
            **extra}


def phases_of(kern, ctr, method=None):
    """Roofline entries of the gather phase (HBM), of the longest verify kernel (VALU), and
    of every verify kernel together against Algorithm 1's own extensions."""
    ver = [k for k in kern if k.startswith("verify")]
    vdom = max(ver, key=lambda k: kern[k][1]) if ver else None
    out = {"gather": roofline_of(kern, ctr, "gather"),
           "verify": roofline_of(kern, ctr, vdom, method) if vdom else None}
    if ver and method:
        vms = sum(kern[k][1] for k in ver)
        ops = method["lv_extensions_per_read"] * ctr["reads"] * VERIFY_OPS_PER_STEP / 1e12
        out["verify_all"] = {"bound": "alu", "kernels": ver, "ms": round(vms, 3),
                             "achieved": round(ops / (vms / 1e3), 3), "peak": VALU_PEAK_TOPS, "unit": "TOP/s",
                             "frac": round(ops / (vms / 1e3) / VALU_PEAK_TOPS, 5)}
    return out


def kernel_source_sha1():
    """SHA-1 of the kernel source file, which a counter summary records: counters taken
    before the kernels last changed do not describe them."""
    import hashlib
    src = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1111_5572_amd", "csrc", "align.hip")
    with open(src, "rb") as f:
        return hashlib.sha1(f.read()).hexdigest()


def read_traffic(path, kernel, workload, schedule):
    """HBM bytes per launch from a counter summary ('key: value' lines, '#' comments),
    when it covers this kernel, workload and pass schedule and was taken on the kernel
    source as it is now; else None."""
    try:
        kv = {}
        for line in open(path):
            line = line.strip()
            if line and not line.startswith("#") and ":" in line:
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        from paper_1111_5572_amd import make_tuning
        sched = tuple(int(x) for x in kv.get("schedule", "").split(",") if x.strip())
        # the chunk-worker count changes which launches overlap, not what one launch reads
        # and writes (the counters are taken with every dispatch alone)
        strip = lambda t: make_tuning(t).astuple()[:7] + make_tuning(t).astuple()[8:]
        same = strip(sched) == strip(tuple(schedule))
        fresh = kv.get("source_sha1") == kernel_source_sha1()
        if kv.get("kernel") == kernel and kv.get("workload") == workload and same and fresh:
            return int(kv["bytes_per_launch"])
    except (OSError, ValueError, KeyError):
        pass
    return None


def oracle_threads():
    """Host threads for the oracle: the host cores, at most 16 (one GPU's share of a box)."""
    return max(1, min(16, os.cpu_count() or 1))


def oracle_check(g, reads, w, got, seconds, single_seconds=4.0, probe=4000, probe1=500):
    """The oracle on a seeded sample of the batch sized to about `seconds` on the host
    cores: the GPU outputs of the sample must equal it on all five fields (else the run
    stops with an error). Returns (cpu_baseline entry, Algorithm 1's own work per read on
    the sample: scored locations and diagonal extensions at each call's own limit)."""
    import oracle
    threads = oracle_threads()
    t = time.time()
    oix = oracle.Index(g, w.params.seed_len, threads=threads, stride=INDEX_STRIDE)
    log(f"oracle index in {time.time() - t:.1f}s ({threads} threads)")
    op = oracle.params_from(w.params)
    rng = np.random.default_rng(7)

    def sample(k):
        return np.unique(rng.integers(0, reads.n, size=min(k, reads.n)))

    def run(idx, nthreads):
        sub = reads.subset(idx)
        t0 = time.perf_counter()
        res = oix.align_reads(sub, op, threads=nthreads)
        return res, time.perf_counter() - t0

    # one thread on a small sample (the paper quotes one core's rate)
    idx1 = sample(probe1)
    res1, dt1 = run(idx1, 1)
    n1 = int(min(reads.n, max(len(idx1), len(idx1) / max(dt1, 1e-9) * single_seconds)))
    if n1 > len(idx1):
        idx1 = sample(n1)
        res1, dt1 = run(idx1, 1)
    single = round(len(idx1) / dt1, 1)
    # all threads, sized from a probe
    idx = sample(probe)
    res, dt = run(idx, threads)
    n_s = int(min(reads.n, max(len(idx), len(idx) / max(dt, 1e-9) * seconds)))
    if n_s > len(idx):
        idx = sample(n_s)
        res, dt = run(idx, threads)
    oix.close()
    checked = [(idx, res), (idx1, res1)]
    mism = 0
    for ix_, r_ in checked:
        mism += sum(int(np.count_nonzero(np.asarray(a)[ix_].astype(np.int64) != np.asarray(b).astype(np.int64)))
                    for a, b in zip(got, r_.fields()))
    if mism:
        print(json.dumps({"error": f"GPU output differs from the oracle on {mism} fields of the sample"}), flush=True)
        sys.exit(1)
    st = res.stats
    method = {"reads": len(idx), "ed_calls_per_read": round(st["ed_calls"] / len(idx), 3),
              "lv_extensions_per_read": round(st["lv_extensions"] / len(idx), 2),
              "seeds_looked_up_per_read": round(st["seeds_looked_up"] / len(idx), 3),
              "select_visits_per_read": round(st["select_visits"] / len(idx), 2),
              "candidates_per_read": round(st["candidates"] / len(idx), 2)}
    # the oracle hands out ranges of at least 4096 reads (Section 2.3's rule), so a small
    # sample keeps fewer threads busy than it was given
    busy = int(min(res.threads, max(1, -(-len(idx) // 4096))))
    cpu = {"value": round(len(idx) / dt, 1), "unit": "reads/s", "cores": busy, "kind": "oracle",
           "single_thread_value": single,
           "sample": f"{len(idx)} seeded-random reads of the {w.name} workload on {busy} busy threads "
                     f"({dt:.1f}s) and {len(idx1)} on one thread ({dt1:.1f}s), each bit-exact vs GPU on all "
                     f"five outputs; the oracle is plain, not a tuned CPU aligner"}
    log(f"cpu baseline: {cpu}")
    log(f"Algorithm 1's own work on the sample: {method}")
    return cpu, method


LENGTH_BUCKETS = [(0, 300), (301, 1000), (1001, 3000), (3001, 1 << 30)]


def bench_batched(args, w, dev):
    """Reads of mixed length (100 bp - 10 kb): per-length-bucket snap_align calls
    (the plain form) vs one snap_align_batched call with the autotuned schedule."""
    import torch
    import paper_1111_5572_amd as snapgpu
    from paper_1111_5572_amd import autotune

    t = time.time()
    g = w.make_genome()
    log(f"genome {w.name}: {len(g)} bases in {time.time() - t:.1f}s")
    t = time.time()
    reads = w.make_reads(g)
    log(f"reads: {reads.n} ({int(reads.bases.shape[0])} bases) in {time.time() - t:.1f}s")
    t = time.time()
    gix = build_index(g, w.params.seed_len)
    index_s = time.time() - t
    sizes = gix.sizes()
    log(f"index built and resident in {index_s:.1f}s: {sizes}")
    params = snapgpu.params_from(w.params)
    d_max = w.params.d_max

    # plain form, one call per length bucket (each bucket resident on the device)
    parts = []
    for lo, hi in LENGTH_BUCKETS:
        idx = np.nonzero((reads.lengths >= lo) & (reads.lengths <= hi))[0]
        if len(idx) == 0:
            continue
        sub = reads.subset(idx)
        rb = torch.from_numpy(sub.bases).to(dev)
        ln = torch.from_numpy(sub.lengths).to(dev)
        ml = int(sub.lengths.max())
        wb = snapgpu.workspace_bytes(gix, sub.n, int(sub.bases.shape[0]), ml, d_max, params)
        ws = torch.empty(wb, dtype=torch.uint8, device=dev)
        parts.append((idx, rb, ln, ml, ws, None))
        del sub
    log("buckets: " + ", ".join(f"{len(p[0])}" for p in parts))

    def run_plain(outs):
        for k, (idx, rb, ln, ml, ws, _) in enumerate(parts):
            outs[k] = snapgpu.align(gix, rb, ln, d_max, params, out=outs[k], workspace=ws, max_len=ml)
        return outs

    outs = run_plain([None] * len(parts))
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        run_plain(outs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        run_plain(outs)
    torch.cuda.synchronize()
    plain_s = (time.perf_counter() - t0) / args.steps
    plain_out = [np.zeros(reads.n, dt) for dt in (np.int64, np.int8, np.int32, np.int32, np.int8)]
    for (idx, *_), o in zip(parts, outs):
        for f, x in zip(plain_out, o.numpy()):
            f[idx] = x
    log(f"plain per-bucket: {plain_s * 1000:.1f} ms/step, {reads.n / plain_s:,.0f} reads/s")
    del parts, outs
    torch.cuda.empty_cache()

    # batched form over the whole batch
    rb = torch.from_numpy(reads.bases).to(dev)
    ln = torch.from_numpy(reads.lengths).to(dev)
    ml = int(reads.lengths.max())
    tuning = None
    tune_info = None
    if args.tuning:
        tuning = tuple(int(x) for x in args.tuning.split(","))
    elif not args.no_autotune:
        rec = None if args.retune else autotune.lookup_entry(reads.lengths, batched=True)
        if rec:
            tune_info = dict(rec, source="tuning table")
        else:
            tune_info = autotune.tune(gix, rb, ln, d_max, params, batched=True, sample_reads=min(reads.n, 100_000),
                                      table_path=None, log=log)
        tuning = tuple(tune_info["tuning"])
        log(f"schedule {tuning} ({tune_info.get('source', 'autotuned')})")
    wb = snapgpu.workspace_bytes(gix, reads.n, int(reads.bases.shape[0]), ml, d_max, params) * 2
    ws = torch.empty(wb, dtype=torch.uint8, device=dev)
    out = snapgpu.align(gix, rb, ln, d_max, params, workspace=ws, max_len=ml, batched=True, tuning=tuning)
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        snapgpu.align(gix, rb, ln, d_max, params, out=out, workspace=ws, max_len=ml, batched=True, tuning=tuning)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        snapgpu.align(gix, rb, ln, d_max, params, out=out, workspace=ws, max_len=ml, batched=True, tuning=tuning)
    torch.cuda.synchronize()
    batched_s = (time.perf_counter() - t0) / args.steps
    # one profiled step of its own (one chunk worker): per-kernel times and counters
    from paper_1111_5572_amd import make_tuning
    t1 = make_tuning(tuning if tuning is not None else snapgpu.get_tuning()).astuple()
    t1 = t1[:7] + (1,) + t1[8:]
    kern, ctr, _ = profiled_steps(
        lambda: snapgpu.align(gix, rb, ln, d_max, params, out=out, workspace=ws, max_len=ml, batched=True,
                              tuning=t1), 1, dev)
    got = out.numpy()
    same = all(np.array_equal(np.asarray(a).astype(np.int64), np.asarray(b).astype(np.int64))
               for a, b in zip(got, plain_out))
    log(f"batched: {batched_s * 1000:.1f} ms/step, {reads.n / batched_s:,.0f} reads/s, identical to plain: {same}")
    log("kernels: " + ", ".join(f"{k} {v[1] / max(v[0], 1):.3f} ms x{v[0]}" for k, v in kern.items()))
    if not same:
        print(json.dumps({"error": "batched and per-bucket plain outputs differ"}), flush=True)
        sys.exit(1)
    cpu, method = (None, None) if args.no_cpu_baseline else oracle_check(g, reads, w, got, args.cpu_seconds,
                                                                             probe=64, probe1=8)
    roofline = roofline_of(kern, ctr, method=method)
    roofline["traffic"] = None
    calls = np.bincount(got[4].astype(np.int64), minlength=3)
    line = {
        "metric": "reads aligned/s", "value": round(reads.n / batched_s, 1), "unit": "reads/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(batched_s * 1000, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic (seeded genome and simulated reads; no real data)",
        "config": {"workload": "batched", "genome_bases": len(g), "reads": reads.n,
                   "read_len": f"{int(reads.lengths.min())}-{int(reads.lengths.max())} log-uniform",
                   "seed_len": w.params.seed_len, "d_max": "max(8, ceil(0.08 L))", "conf_c": w.params.conf_c,
                   "max_hits": w.params.max_hits, "form": "batched (one work-stealing verify launch per pass)"},
        "gbases_per_s": round(float(reads.bases.shape[0]) / batched_s / 1e9, 4),
        "plain_per_bucket": {"reads_per_s": round(reads.n / plain_s, 1), "ms_per_step": round(plain_s * 1000, 3),
                             "buckets": [list(b) for b in LENGTH_BUCKETS]},
        "speedup_vs_per_bucket": round(plain_s / batched_s, 3),
        "autotune": tune_info,
        "index_build_s": round(index_s, 2), "index_build": "host" if INDEX_ON_HOST else "device",
        "index_device_bytes": sizes["device_bytes"],
        "calls": {"not_found": int(calls[0]), "single": int(calls[1]), "multiple": int(calls[2])},
        "kernel_ms_per_step": {k: round(v[1], 4) for k, v in kern.items()},
        "counters_per_step": ctr,
        "roofline": roofline,
        # the two phases the method hinges on: gather (HBM-bound) and verify (VALU-bound)
        "phases": phases_of(kern, ctr, method),
        "cpu_baseline": cpu,
        "method_work": method,
    }
    print(json.dumps(line), flush=True)
    gix.close()


def bench_served(args, w, dev):
    """Request server: saturated throughput, then Poisson arrivals at 25/50/90% of
    it; per level the request latency (completion - submission) p50 / p99."""
    import threading
    import paper_1111_5572_amd as snapgpu
    import synth

    t = time.time()
    g = w.make_genome()
    pool = w.make_reads(g)
    log(f"genome {len(g)} bases, read pool {pool.n} reads in {time.time() - t:.1f}s")
    t = time.time()
    gix = build_index(g, w.params.seed_len)
    log(f"index resident in {time.time() - t:.1f}s")
    params = snapgpu.params_from(w.params)
    # the batched form's schedule for this length mix, when the tuning table has it
    from paper_1111_5572_amd import autotune
    if args.tuning:
        tuning = tuple(int(x) for x in args.tuning.split(","))
    else:
        tuning = None if args.no_autotune else autotune.lookup(pool.lengths, batched=True)
    log(f"server schedule: {tuning or 'library default'}")
    srv = snapgpu.Server(gix, w.params.d_max, params, tuning=tuning, slots=4, batch_reads=1 << 16,
                         batch_bases=160 << 20, hbm_budget=48 << 30, max_waiting=1 << 14)
    log(f"server: {srv.stats()}")

    offs = pool.offsets
    cursor = [0]

    def next_request(k):
        i = cursor[0]
        if i + k > pool.n:
            i = 0
        cursor[0] = i + k
        return pool.bases[offs[i]:offs[i + k]], pool.lengths[i:i + k]

    kept = []   # (bases, lengths, outputs) of sampled requests, for the oracle check

    def run(n_req, arrivals=None, sizes=None, keep_every=0):
        """Submit n_req requests (open loop at `arrivals` seconds, or back to back),
        poll them all; returns (elapsed, reads, latencies). With keep_every, the outputs
        of every keep_every-th request of at most 300 reads are kept."""
        done = {}
        tickets = []
        inputs = {}
        lock = threading.Lock()
        stop = [False]

        def poller():
            while True:
                with lock:
                    pend = [x for x in tickets if x[0] not in done]
                    finished = stop[0] and not pend
                for tk, _ in pend:
                    r = srv.poll(tk)
                    if r is not None:
                        done[tk] = r[5]
                        if tk in inputs:
                            kept.append((*inputs[tk], r[:5]))
                if finished:
                    return
                time.sleep(0.0002)

        th = threading.Thread(target=poller)
        th.start()
        t0 = time.perf_counter()
        nreads = 0
        for q in range(n_req):
            if arrivals is not None:
                dt = arrivals[q] - (time.perf_counter() - t0)
                if dt > 0:
                    time.sleep(dt)
            b, l = next_request(int(sizes[q]))
            while True:
                try:
                    tk = srv.submit(b, l)
                    break
                except snapgpu.SnapError as e:
                    if e.code != snapgpu.SNAP_EBUSY:
                        raise
                    time.sleep(0.0005)
            nreads += len(l)
            with lock:
                if keep_every and q % keep_every == 0 and len(l) <= 300:
                    inputs[tk] = (np.array(b), np.array(l))
                tickets.append((tk, len(l)))
        with lock:
            stop[0] = True
        th.join()
        elapsed = time.perf_counter() - t0
        lat = np.array([done[tk][2] - done[tk][0] for tk, _ in tickets])
        return elapsed, nreads, lat

    rng_sizes = lambda n, seed: synth.arrivals(n, seed, 1.0)[1]
    nq = max(args.requests, 1)
    run(max(20, nq // 10), sizes=rng_sizes(max(20, nq // 10), 104))   # warm-up
    el, nr, lat = run(nq, sizes=rng_sizes(nq, 105), keep_every=20)
    sat = nr / el
    log(f"saturated: {nq} requests, {nr} reads in {el:.2f}s = {sat:,.0f} reads/s; p50 {np.median(lat)*1e3:.1f} ms")
    levels = {}
    for load in (0.25, 0.5, 0.9):
        sizes = rng_sizes(nq, 106)
        rate = load * sat / float(np.mean(sizes))
        arr, _ = synth.arrivals(nq, 107, rate)
        el, nr, lat = run(nq, arrivals=arr, sizes=sizes)
        offered = nr / float(arr[-1]) if len(arr) and arr[-1] > 0 else load * sat
        levels[f"{int(load * 100)}%"] = {"offered_reads_per_s": round(offered, 1),
                                         "achieved_reads_per_s": round(nr / el, 1),
                                         "kept_up": bool(nr / el >= 0.95 * offered),
                                         "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 2),
                                         "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 2),
                                         "requests": nq}
        log(f"load {load:.0%}: {levels[f'{int(load * 100)}%']}")
    st = srv.stats()
    srv.close()
    gix.close()
    # the outputs of sampled requests against the oracle, bit for bit
    checked = None
    if not args.no_cpu_baseline and kept:
        import oracle
        import synth as sy
        t = time.time()
        oix = oracle.Index(g, w.params.seed_len, threads=oracle_threads())
        op = oracle.params_from(w.params)
        nreq = nrd = 0
        for bases, lens, outs in kept[:8]:
            offs_ = np.zeros(len(lens) + 1, np.int64)
            np.cumsum(lens, out=offs_[1:])
            res = oix.align(bases, offs_, lens, op, threads=oracle_threads())
            mism = sum(int(np.count_nonzero(np.asarray(a).astype(np.int64) != np.asarray(b).astype(np.int64)))
                       for a, b in zip(outs, res.fields()))
            if mism:
                print(json.dumps({"error": f"a served request differs from the oracle on {mism} fields"}), flush=True)
                sys.exit(1)
            nreq += 1
            nrd += len(lens)
        oix.close()
        checked = {"requests": nreq, "reads": nrd, "bit_exact": True, "seconds": round(time.time() - t, 1)}
        log(f"oracle check of served requests: {checked}")
    line = {
        "metric": "reads aligned/s", "value": round(sat, 1), "unit": "reads/s", "n_gpus": 1,
        "steps": args.steps, "warmup": 1, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic (seeded genome and simulated reads; no real data)",
        "config": {"workload": "served", "genome_bases": len(g), "read_pool": pool.n,
                   "request_reads": "floor(10^(4u))", "read_len": "100 bp-10 kb log-uniform",
                   "slots": st["slots"], "slot_device_bytes": st["slot_device_bytes"]},
        "latency": levels, "server": st, "roofline": None, "cpu_baseline": None, "oracle_check": checked,
    }
    print(json.dumps(line), flush=True)


def profiled_steps(step, n, dev):
    """Run `step` n times with profiling on and one chunk worker (the process-wide
    schedule's worker field set to 1; a step that passes its own schedule sets it there),
    between two marker launches of the library's copy kernel; returns (per-kernel times,
    counters, ms per step)."""
    import torch
    import paper_1111_5572_amd as snapgpu
    old = snapgpu.get_tuning()
    one = old[:7] + (1,) + old[8:]
    snapgpu.set_tuning(*one)
    mark = torch.zeros(64, dtype=torch.int32, device=dev)
    mark2 = torch.empty_like(mark)
    try:
        torch.cuda.synchronize()
        snapgpu.debug_copy(mark, mark2, 256)
        torch.cuda.synchronize()
        snapgpu.profile_begin()
        tp = time.perf_counter()
        for _ in range(n):
            step()
        torch.cuda.synchronize()
        ms = 1000.0 * (time.perf_counter() - tp) / n
        kern = snapgpu.profile_end()
        ctr = snapgpu.profile_counters()
        snapgpu.debug_copy(mark, mark2, 256)
        torch.cuda.synchronize()
    finally:
        snapgpu.set_tuning(*old)
    return kern, ctr, ms


def streamed_steps(gix, reads, w, params, got, chunks, steps, dev):
    """The batch aligned from pinned host memory: the reads go to the device in `chunks`
    parts (one stream copies part k+1 in while part k is aligned on another; two device
    buffers alternate) and each part's outputs come back on a third stream as soon as it
    is aligned. Timed from the first host-to-device copy to the last device-to-host copy
    (index resident). Outputs must equal the resident run's."""
    import torch
    import paper_1111_5572_amd as snapgpu
    n = reads.n
    offs = reads.offsets
    rb = np.linspace(0, n, chunks + 1).astype(np.int64)
    t = time.time()
    hb = torch.empty(int(reads.bases.shape[0]), dtype=torch.uint8, pin_memory=True)
    hb.numpy()[:] = reads.bases
    hl = torch.empty(n, dtype=torch.int32, pin_memory=True)
    hl.numpy()[:] = reads.lengths
    host_out = [torch.empty(n, dtype=dt, pin_memory=True)
                for dt in (torch.int64, torch.int8, torch.int32, torch.int32, torch.int8)]
    log(f"streamed: {hb.numel() / 1e9:.1f} GB of reads in pinned host memory ({time.time() - t:.1f}s)")
    max_b = int(max(offs[rb[k + 1]] - offs[rb[k]] for k in range(chunks)))
    max_r = int(max(rb[k + 1] - rb[k] for k in range(chunks)))
    ml = int(reads.lengths.max())
    dbuf = [torch.empty(max_b, dtype=torch.uint8, device=dev) for _ in range(2)]
    dlen = [torch.empty(max_r, dtype=torch.int32, device=dev) for _ in range(2)]
    out = snapgpu.Alignment(*(torch.empty(n, dtype=t_.dtype, device=dev) for t_ in host_out))
    wb = 4 * snapgpu.workspace_bytes(gix, max_r, max_b, ml, w.params.d_max, params)
    ws = torch.empty(wb, dtype=torch.uint8, device=dev)
    s_in, s_out = torch.cuda.Stream(), torch.cuda.Stream()
    s_c = torch.cuda.current_stream()

    def h2d(k, ev_done):
        b = k % 2
        r0, r1 = int(rb[k]), int(rb[k + 1])
        o0, o1 = int(offs[r0]), int(offs[r1])
        with torch.cuda.stream(s_in):
            if k >= 2:
                s_in.wait_event(ev_done[k - 2])   # the buffer's previous part is aligned
            dbuf[b][:o1 - o0].copy_(hb[o0:o1], non_blocking=True)
            dlen[b][:r1 - r0].copy_(hl[r0:r1], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(s_in)
        return ev

    def one_step():
        ev_in = [None] * chunks
        ev_done = [None] * chunks
        ev_in[0] = h2d(0, ev_done)
        for k in range(chunks):
            if k + 1 < chunks:
                ev_in[k + 1] = h2d(k + 1, ev_done)
            b = k % 2
            r0, r1 = int(rb[k]), int(rb[k + 1])
            o0, o1 = int(offs[r0]), int(offs[r1])
            s_c.wait_event(ev_in[k])
            part = snapgpu.Alignment(*(t_[r0:r1] for t_ in (out.pos, out.strand, out.dist, out.second, out.call)))
            snapgpu.align(gix, dbuf[b][:o1 - o0], dlen[b][:r1 - r0], w.params.d_max, params, out=part,
                          workspace=ws, stream=s_c, max_len=ml)
            ev_done[k] = torch.cuda.Event()
            ev_done[k].record(s_c)
            with torch.cuda.stream(s_out):
                s_out.wait_event(ev_done[k])
                for h, d in zip(host_out, (part.pos, part.strand, part.dist, part.second, part.call)):
                    h[r0:r1].copy_(d, non_blocking=True)
        torch.cuda.synchronize()

    one_step()   # untimed
    times = []
    for _ in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        one_step()
        times.append(time.perf_counter() - t0)
    same = all(np.array_equal(h.numpy().astype(np.int64), np.asarray(g_).astype(np.int64))
               for h, g_ in zip(host_out, got))
    if not same:
        print(json.dumps({"error": "outputs aligned from host memory differ from the resident run's"}), flush=True)
        sys.exit(1)
    sec = sum(times) / len(times)
    res = {"reads_per_s": round(n / sec, 1), "ms_per_step": round(sec * 1000, 3), "steps": steps,
           "chunks": chunks, "host_bytes_in": int(hb.numel() + 4 * n), "host_bytes_out": int(18 * n),
           "outputs_equal_resident": True}
    log(f"streamed from host memory: {res}")
    del hb, hl, host_out, dbuf, dlen, out, ws
    torch.cuda.empty_cache()
    return res


def bench_plain(args, w, dev):
    """One step = snap_align over the whole batch (reads and index resident in HBM)."""
    import torch
    import paper_1111_5572_amd as snapgpu

    t = time.time()
    g = w.make_genome()
    log(f"genome {w.name}: {len(g)} bases in {time.time() - t:.1f}s")
    t = time.time()
    reads = w.make_reads(g)
    log(f"reads: {reads.n} ({int(reads.bases.shape[0])} bases) in {time.time() - t:.1f}s")
    t = time.time()
    gix = build_index(g, w.params.seed_len)
    index_s = time.time() - t
    sizes = gix.sizes()
    log(f"index built and resident in {index_s:.1f}s: {sizes}")
    dup = None
    if args.dup_window:
        torch.cuda.synchronize()
        t = time.time()
        gix.dup_classes(args.dup_window)
        torch.cuda.synchronize()
        dup = {"window": args.dup_window, "build_s": round(time.time() - t, 3),
               "device_bytes": gix.sizes()["device_bytes"] - sizes["device_bytes"]}
        log(f"exact-duplicate classes of {args.dup_window}-base windows in {dup['build_s']}s")

    rb = torch.from_numpy(reads.bases).to(dev)
    ln = torch.from_numpy(reads.lengths).to(dev)
    params = snapgpu.params_from(w.params)
    max_len = int(reads.lengths.max())
    # a generous workspace: more reads per internal pass, fewer waits (outputs do not change)
    wb = 4 * snapgpu.workspace_bytes(gix, reads.n, int(reads.bases.shape[0]), max_len, w.params.d_max, params)
    ws = torch.empty(wb, dtype=torch.uint8, device=dev)
    tune_info = None
    if args.tuning:
        snapgpu.set_tuning(*[int(x) for x in args.tuning.split(",")])
        log(f"fixed schedule {snapgpu.get_tuning()}")
    elif not args.no_autotune:
        from paper_1111_5572_amd import autotune
        rec = None if args.retune else autotune.lookup_entry(reads.lengths, batched=False)
        if rec:
            tune_info = dict(rec, source="tuning table")
        else:
            tune_info = autotune.tune(gix, rb, ln, w.params.d_max, params, batched=False,
                                      sample_reads=min(reads.n, 1_000_000), table_path=args.tuning_out or None,
                                      log=log)
            tune_info["workload"] = f"{w.name} ({w.notes}), MI355X"
        snapgpu.set_tuning(*tune_info["tuning"])
        log(f"schedule {tuple(tune_info['tuning'])} ({tune_info.get('source', 'autotuned')})")
    out = snapgpu.align(gix, rb, ln, w.params.d_max, params, workspace=ws, max_len=max_len)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        snapgpu.align(gix, rb, ln, w.params.d_max, params, out=out, workspace=ws, max_len=max_len)
    torch.cuda.synchronize()
    log(f"warmup done ({args.warmup} steps)")

    # timed steps, nothing else on: reads resident in HBM when the clock starts
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        snapgpu.align(gix, rb, ln, w.params.d_max, params, out=out, workspace=ws, stream=stream, max_len=max_len)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1000.0 * elapsed / args.steps
    reads_per_s = reads.n * args.steps / elapsed
    gbases_per_s = float(reads.bases.shape[0]) * args.steps / elapsed / 1e9
    log(f"timed {args.steps} steps: {ms_per_step:.2f} ms/step, {reads_per_s:,.0f} reads/s")

    # profiled steps of their own: per-kernel times (an event pair on each launch's
    # stream) and device counters, with one chunk worker so that each kernel runs alone
    # and its events time the kernel itself; a marker launch before and after (the
    # library's copy kernel on 256 bytes) brackets these steps in a profiler's trace
    prof_steps = max(1, min(args.steps, 2))
    kern, ctr, prof_ms = profiled_steps(
        lambda: snapgpu.align(gix, rb, ln, w.params.d_max, params, out=out, workspace=ws, stream=stream,
                              max_len=max_len), prof_steps, dev)
    log(f"profiled {prof_steps} steps: {prof_ms:.2f} ms/step")
    log("kernels: " + ", ".join(f"{k} {v[1] / max(v[0], 1):.3f} ms x{v[0]}" for k, v in kern.items()))
    log(f"counters: {ctr}")

    got = out.numpy()
    calls = np.bincount(got[4].astype(np.int64), minlength=3)
    del ws
    torch.cuda.empty_cache()
    streamed = None
    if args.stream_chunks > 0:
        del rb
        torch.cuda.empty_cache()
        streamed = streamed_steps(gix, reads, w, params, got, args.stream_chunks, max(1, min(args.steps, 2)), dev)

    # CPU oracle on a bounded sample: bit-exact check, baseline rate, Algorithm 1's own work
    cpu, method = (None, None) if args.no_cpu_baseline else oracle_check(g, reads, w, got, args.cpu_seconds)

    # roofline of the dominant kernel, with HBM traffic from the committed counter summary
    roofline = roofline_of(kern, ctr, method=method)
    line_phases = phases_of(kern, ctr, method)
    roofline["traffic"] = read_traffic(args.traffic.format(kernel=roofline["kernel"], workload=w.name),
                                       roofline["kernel"], w.name, snapgpu.get_tuning())
    for ph in line_phases.values():
        if ph and "kernel" in ph:
            ph["traffic"] = read_traffic(args.traffic.format(kernel=ph["kernel"], workload=w.name), ph["kernel"],
                                         w.name, snapgpu.get_tuning())

    line = {
        "metric": "reads aligned/s", "value": round(reads_per_s, 1), "unit": "reads/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic (seeded genome and simulated reads; no real data)",
        "config": {"workload": w.name, "genome_bases": len(g), "reads": reads.n,
                   "read_len": (int(reads.lengths.max()) if reads.lengths.min() == reads.lengths.max()
                                else sorted({int(x) for x in np.unique(reads.lengths)[:4]})),
                   "seed_len": w.params.seed_len,
                   "seeds_per_read": w.params.n_min, "d_max": w.params.d_max, "conf_c": w.params.conf_c,
                   "max_hits": w.params.max_hits, "index_stride": INDEX_STRIDE},
        "gbases_per_s": round(gbases_per_s, 4),
        "timed_region": "reads and index resident in HBM; no profiling in the timed steps",
        "with_host_copies": streamed,
        "index_build_s": round(index_s, 2), "index_build": "host" if INDEX_ON_HOST else "device",
        "index_device_bytes": sizes["device_bytes"],
        "dup_classes": dup,
        "calls": {"not_found": int(calls[0]), "single": int(calls[1]), "multiple": int(calls[2])},
        "profiled_ms_per_step": round(prof_ms, 3),
        "profiled_workers": 1,
        "kernel_ms_per_step": {k: round(v[1] / prof_steps, 4) for k, v in kern.items()},
        "counters_per_step": {k: v // prof_steps for k, v in ctr.items()},
        "schedule": tune_info,
        "roofline": roofline,
        # the two phases the method hinges on: gather (HBM-bound) and verify (VALU-bound)
        "phases": line_phases,
        "cpu_baseline": cpu,
        "method_work": method,
    }
    print(json.dumps(line), flush=True)
    gix.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="human")
    ap.add_argument("--reads", type=int, default=0, help="override the read count (profiling runs)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--requests", type=int, default=2000, help="served workload: requests per load level")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "{kernel}_traffic_{workload}.txt"),
                    help="counter summary giving a kernel's HBM bytes per launch ({kernel}, {workload} filled in)")
    ap.add_argument("--genome-len", type=int, default=0, help="override the genome length (batched/served runs)")
    ap.add_argument("--no-autotune", action="store_true", help="library default schedule")
    ap.add_argument("--host-index", action="store_true", help="build the index on the host (snap_index_build)")
    ap.add_argument("--dup-window", type=int, default=0,
                    help="attach exact-duplicate classes of windows of this many bases (0: none)")
    ap.add_argument("--stride", type=int, default=1,
                    help="index only the windows at multiples of this stride (1, 2 or 4; device build)")
    ap.add_argument("--accuracy", action="store_true",
                    help="h_max sweep: aligned / error rates and reads/s for 125 bp reads at 2%% errors")
    ap.add_argument("--accuracy-grid", action="store_true",
                    help="Section 2's tables: aligned / error rates and reads/s over read lengths and error rates")
    ap.add_argument("--grid-scale", type=int, default=1, help="divide the grid's read counts by this")
    ap.add_argument("--gather-gb", type=float, default=0.0,
                    help="only run the random-line gather microbenchmark over a buffer of this many GB")
    ap.add_argument("--index-only", action="store_true",
                    help="time the index build of the workload's genome (--steps builds) and stop")
    ap.add_argument("--retune", action="store_true",
                    help="run the autotuner even when the package's tuning table has this length class")
    ap.add_argument("--tuning-out", default="", help="record an autotuned schedule in this JSON table")
    ap.add_argument("--stream-chunks", type=int, default=8,
                    help="also time the batch aligned from pinned host memory in this many parts (0: skip)")
    ap.add_argument("--tuning", default="", help="fixed schedule a,b,c,d (snap_tuning fields); skips the autotuner")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run the library's plain copy kernel over this many bytes, 3 times "
                         "(the known-size reference for HBM byte counters)")
    args = ap.parse_args()
    global INDEX_ON_HOST, INDEX_STRIDE
    INDEX_ON_HOST = args.host_index
    INDEX_STRIDE = args.stride
    if INDEX_STRIDE != 1 and INDEX_ON_HOST:
        print(json.dumps({"error": "a strided index is built on the device only"}), flush=True)
        sys.exit(2)

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "runs on one GPU only: the read batch is not sharded across GPUs",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import torch
    import paper_1111_5572_amd as snapgpu
    from synth.workloads import WORKLOADS

    w = WORKLOADS[args.workload]
    if args.reads or args.genome_len:
        w = w.scaled(genome_len=args.genome_len or None, n_reads=args.reads or None)
    dev = torch.device("cuda:0")
    snapgpu.lib()
    if args.copy_bytes:
        src = torch.ones(args.copy_bytes // 4, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            snapgpu.debug_copy(src, dst, args.copy_bytes)
        torch.cuda.synchronize()
        log(f"copied {args.copy_bytes} bytes 3 times, equal: {bool(torch.equal(src, dst))}")
        return
    if args.gather_gb:
        return bench_gather(args, dev)
    if args.index_only:
        return bench_index(args, w)
    if args.accuracy:
        return bench_accuracy(args, w, dev)
    if args.accuracy_grid:
        return bench_accuracy_grid(args, w, dev)
    if args.workload == "batched":
        return bench_batched(args, w, dev)
    if args.workload == "served":
        return bench_served(args, w, dev)

    return bench_plain(args, w, dev)


if __name__ == "__main__":
    main()
