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


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


INDEX_ON_HOST = False   # --host-index


def build_index(g, seed_len):
    """Device index of the genome, built by the library's device kernels (or, with
    --host-index, on the host, logging each finished stage: minutes for a large genome)."""
    import paper_1111_5572_amd as snapgpu
    t0 = time.time()
    report = lambda stage: log(f"  index: {stage} ({time.time() - t0:.3f}s)")
    return snapgpu.Index(g, seed_len, progress=report, on_device=not INDEX_ON_HOST)


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
        row = {"h_max": h, **accuracy_of(out.numpy(), reads), "reads_per_s": round(n / (ms / 1e3), 1),
               "ms_per_step": round(ms, 3)}
        log(f"h_max {h}: {row}")
        rows.append(row)
    gix.close()
    print(json.dumps({"metric": "h_max trade-off", "unit": "aligned %, error %, reads/s", "n_gpus": 1,
                      "steps": max(1, args.steps), "data": "synthetic (seeded genome and simulated reads)",
                      "config": {"workload": w.name, "genome_bases": len(g), "reads": n, "read_len": 125,
                                 "errors": "1.8% substitutions, 0.2% indels (1-5)", "d_max": 8,
                                 "conf_c": w.params.conf_c, "seed_len": w.params.seed_len,
                                 "correct": "same strand, |pos - source| <= 32",
                                 "schedule": list(tuning) if tuning else None},
                      "rows": rows}), flush=True)


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


def roofline_of(kern, ctr, prefer=None):
    """Roofline entry of the dominant kernel (or `prefer` if given)."""
    if prefer is not None and prefer not in kern:
        return None
    dom = prefer if prefer in kern else max(kern.items(), key=lambda kv: kv[1][1])[0]
    launches, total_ms = kern[dom]
    avg_s = total_ms / 1000.0 / launches
    per_launch = 1.0 / launches
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
            steps = first
        else:
            req = [k for k in kern if k.startswith("verify") and k not in ("verify", "verify_steal")]
            vt = sum(kern[k][1] for k in req)
            steps = (ctr["lv_steps"] - first) * (total_ms / vt if vt > 0 else 1.0)
        work = steps * VERIFY_OPS_PER_STEP * per_launch / 1e12
    else:
        bound, unit, peak = "hbm", "GB/s", HBM_PEAK_GBS
        work = float("nan")
    achieved = work / avg_s
    return {"bound": bound, "kernel": dom, "achieved": round(achieved, 3), "peak": peak, "unit": unit,
            "frac": round(achieved / peak, 5), "avg_launch_ms": round(total_ms / launches, 4), "launches": launches}


def phases_of(kern, ctr):
    """Roofline entries of the gather phase (HBM) and of the longest verify kernel (VALU)."""
    ver = [k for k in kern if k.startswith("verify")]
    vdom = max(ver, key=lambda k: kern[k][1]) if ver else None
    return {"gather": roofline_of(kern, ctr, "gather"), "verify": roofline_of(kern, ctr, vdom) if vdom else None}


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
        strip = lambda t: make_tuning(t).astuple()[:7]
        same = strip(sched) == strip(tuple(schedule))
        fresh = kv.get("source_sha1") == kernel_source_sha1()
        if kv.get("kernel") == kernel and kv.get("workload") == workload and same and fresh:
            return int(kv["bytes_per_launch"])
    except (OSError, ValueError, KeyError):
        pass
    return None


def cpu_baseline(g, reads, w, got, seconds, log_fn=None):
    """The oracle on a seeded sample sized to about `seconds` of CPU time; checks
    the GPU outputs of the sample bit-exact first."""
    import oracle
    threads = max(1, min(16, os.cpu_count() or 1))
    t = time.time()
    oix = oracle.Index(g, w.params.seed_len)
    log(f"oracle index in {time.time() - t:.1f}s")
    op = oracle.params_from(w.params)
    rng = np.random.default_rng(7)
    probe_n = min(reads.n, 2000)
    idx = np.sort(rng.choice(reads.n, probe_n, replace=False))
    sub = reads.subset(idx)
    t = time.perf_counter()
    res = oix.align_reads(sub, op, threads=threads)
    dt = time.perf_counter() - t
    rate = probe_n / max(dt, 1e-9)
    n_s = int(min(reads.n, max(probe_n, rate * seconds)))
    if n_s > probe_n:
        idx = np.sort(rng.choice(reads.n, n_s, replace=False))
        sub = reads.subset(idx)
        t = time.perf_counter()
        res = oix.align_reads(sub, op, threads=threads)
        dt = time.perf_counter() - t
    oix.close()
    mism = sum(int(np.count_nonzero(np.asarray(a)[idx].astype(np.int64) != np.asarray(b).astype(np.int64)))
               for a, b in zip(got, res.fields()))
    if mism:
        print(json.dumps({"error": f"GPU output differs from the oracle on {mism} fields of the sample"}), flush=True)
        sys.exit(1)
    return {"value": round(len(idx) / dt, 1), "unit": "reads/s", "cores": res.threads, "kind": "oracle",
            "sample": f"{len(idx)} seeded-random reads of the {w.name} workload, {dt:.1f}s, "
                      f"bit-exact vs GPU on all five outputs"}


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
    snapgpu.profile_begin()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        snapgpu.align(gix, rb, ln, d_max, params, out=out, workspace=ws, max_len=ml, batched=True, tuning=tuning)
    torch.cuda.synchronize()
    batched_s = (time.perf_counter() - t0) / args.steps
    kern = snapgpu.profile_end()
    ctr = snapgpu.profile_counters()
    got = out.numpy()
    same = all(np.array_equal(np.asarray(a).astype(np.int64), np.asarray(b).astype(np.int64))
               for a, b in zip(got, plain_out))
    log(f"batched: {batched_s * 1000:.1f} ms/step, {reads.n / batched_s:,.0f} reads/s, identical to plain: {same}")
    log("kernels: " + ", ".join(f"{k} {v[1] / max(v[0], 1):.3f} ms x{v[0]}" for k, v in kern.items()))
    if not same:
        print(json.dumps({"error": "batched and per-bucket plain outputs differ"}), flush=True)
        sys.exit(1)
    roofline = roofline_of(kern, ctr)
    roofline["traffic"] = None
    cpu = None if args.no_cpu_baseline else cpu_baseline(g, reads, w, got, args.cpu_seconds)
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
        "kernel_ms_per_step": {k: round(v[1] / args.steps, 4) for k, v in kern.items()},
        "counters_per_step": {k: v // max(args.steps, 1) for k, v in ctr.items()},
        "roofline": roofline,
        # the two phases the method hinges on: gather (HBM-bound) and verify (VALU-bound)
        "phases": phases_of(kern, ctr),
        "cpu_baseline": cpu,
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

    def run(n_req, arrivals=None, sizes=None):
        """Submit n_req requests (open loop at `arrivals` seconds, or back to back),
        poll them all; returns (elapsed, reads, latencies)."""
        done = {}
        tickets = []
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
                tickets.append((tk, len(l)))
        with lock:
            stop[0] = True
        th.join()
        elapsed = time.perf_counter() - t0
        lat = np.array([done[tk][2] - done[tk][0] for tk, _ in tickets])
        return elapsed, nreads, lat

    rng_sizes = lambda n, seed: synth.arrivals(n, seed, 1.0)[1]
    nq = args.steps * 100
    run(max(20, nq // 10), sizes=rng_sizes(max(20, nq // 10), 104))   # warm-up
    el, nr, lat = run(nq, sizes=rng_sizes(nq, 105))
    sat = nr / el
    log(f"saturated: {nq} requests, {nr} reads in {el:.2f}s = {sat:,.0f} reads/s; p50 {np.median(lat)*1e3:.1f} ms")
    levels = {}
    for load in (0.25, 0.5, 0.9):
        sizes = rng_sizes(nq, 106)
        rate = load * sat / float(np.mean(sizes))
        arr, _ = synth.arrivals(nq, 107, rate)
        el, nr, lat = run(nq, arrivals=arr, sizes=sizes)
        levels[f"{int(load * 100)}%"] = {"offered_reads_per_s": round(load * sat, 1),
                                         "achieved_reads_per_s": round(nr / el, 1),
                                         "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 2),
                                         "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 2),
                                         "requests": nq}
        log(f"load {load:.0%}: {levels[f'{int(load * 100)}%']}")
    st = srv.stats()
    srv.close()
    gix.close()
    line = {
        "metric": "reads aligned/s", "value": round(sat, 1), "unit": "reads/s", "n_gpus": 1,
        "steps": args.steps, "warmup": 1, "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic (seeded genome and simulated reads; no real data)",
        "config": {"workload": "served", "genome_bases": len(g), "read_pool": pool.n,
                   "request_reads": "floor(10^(4u))", "read_len": "100 bp-10 kb log-uniform",
                   "slots": st["slots"], "slot_device_bytes": st["slot_device_bytes"]},
        "latency": levels, "server": st, "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="mid")
    ap.add_argument("--reads", type=int, default=0, help="override the read count (profiling runs)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "verify_traffic_mid.txt"),
                    help="counter summary giving the dominant kernel's HBM bytes per launch")
    ap.add_argument("--genome-len", type=int, default=0, help="override the genome length (batched/served runs)")
    ap.add_argument("--no-autotune", action="store_true", help="library default schedule")
    ap.add_argument("--host-index", action="store_true", help="build the index on the host (snap_index_build)")
    ap.add_argument("--accuracy", action="store_true",
                    help="h_max sweep: aligned / error rates and reads/s for 125 bp reads at 2%% errors")
    ap.add_argument("--index-only", action="store_true",
                    help="time the index build of the workload's genome (--steps builds) and stop")
    ap.add_argument("--retune", action="store_true",
                    help="run the autotuner even when the package's tuning table has this length class")
    ap.add_argument("--tuning", default="", help="fixed schedule a,b,c,d (snap_tuning fields); skips the autotuner")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run the library's plain copy kernel over this many bytes, 3 times "
                         "(the known-size reference for HBM byte counters)")
    args = ap.parse_args()
    global INDEX_ON_HOST
    INDEX_ON_HOST = args.host_index

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
    if args.index_only:
        return bench_index(args, w)
    if args.accuracy:
        return bench_accuracy(args, w, dev)
    if args.workload == "batched":
        return bench_batched(args, w, dev)
    if args.workload == "served":
        return bench_served(args, w, dev)

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
                                      sample_reads=min(reads.n, 1_000_000), table_path=None, log=log)
        snapgpu.set_tuning(*tune_info["tuning"])
        log(f"schedule {tuple(tune_info['tuning'])} ({tune_info.get('source', 'autotuned')})")
    out = snapgpu.align(gix, rb, ln, w.params.d_max, params, workspace=ws, max_len=max_len)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        snapgpu.align(gix, rb, ln, w.params.d_max, params, out=out, workspace=ws, max_len=max_len)
    torch.cuda.synchronize()
    log(f"warmup done ({args.warmup} steps)")

    snapgpu.profile_begin()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        snapgpu.align(gix, rb, ln, w.params.d_max, params, out=out, workspace=ws, stream=stream, max_len=max_len)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern = snapgpu.profile_end()
    ctr = snapgpu.profile_counters()
    elapsed = t1 - t0
    ms_per_step = 1000.0 * elapsed / args.steps
    reads_per_s = reads.n * args.steps / elapsed
    gbases_per_s = float(reads.bases.shape[0]) * args.steps / elapsed / 1e9
    log(f"timed {args.steps} steps: {ms_per_step:.2f} ms/step, {reads_per_s:,.0f} reads/s")
    log("kernels: " + ", ".join(f"{k} {v[1] / max(v[0], 1):.3f} ms x{v[0]}" for k, v in kern.items()))
    log(f"counters: {ctr}")

    got = out.numpy()
    calls = np.bincount(got[4].astype(np.int64), minlength=3)

    # roofline of the dominant kernel, with HBM traffic from the committed counter summary
    roofline = roofline_of(kern, ctr)
    roofline["traffic"] = read_traffic(args.traffic, roofline["kernel"], w.name, snapgpu.get_tuning())

    # CPU oracle on a bounded sample, and a bit-exact check of that sample
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        threads = max(1, min(16, os.cpu_count() or 1))
        t = time.time()
        oix = oracle.Index(g, w.params.seed_len)
        log(f"oracle index in {time.time() - t:.1f}s")
        op = oracle.params_from(w.params)
        rng = np.random.default_rng(7)
        probe_n = min(reads.n, 4000)
        idx = np.sort(rng.choice(reads.n, probe_n, replace=False))
        sub = reads.subset(idx)
        t = time.perf_counter()
        res = oix.align_reads(sub, op, threads=threads)
        dt = time.perf_counter() - t
        rate = probe_n / max(dt, 1e-9)
        n_s = int(min(reads.n, max(probe_n, rate * args.cpu_seconds)))
        if n_s > probe_n:
            idx = np.sort(rng.choice(reads.n, n_s, replace=False))
            sub = reads.subset(idx)
            t = time.perf_counter()
            res = oix.align_reads(sub, op, threads=threads)
            dt = time.perf_counter() - t
        oix.close()
        mism = sum(int(np.count_nonzero(np.asarray(a)[idx].astype(np.int64) != np.asarray(b).astype(np.int64)))
                   for a, b in zip(got, res.fields()))
        if mism:
            print(json.dumps({"error": f"GPU output differs from the oracle on {mism} fields of the sample"}), flush=True)
            sys.exit(1)
        cpu = {"value": round(len(idx) / dt, 1), "unit": "reads/s", "cores": res.threads, "kind": "oracle",
               "sample": f"{len(idx)} seeded-random reads of the {w.name} workload, {dt:.1f}s, "
                         f"bit-exact vs GPU on all five outputs"}
        log(f"cpu baseline: {cpu}")

    line = {
        "metric": "reads aligned/s", "value": round(reads_per_s, 1), "unit": "reads/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic (seeded genome and simulated reads; no real data)",
        "config": {"workload": w.name, "genome_bases": len(g), "reads": reads.n,
                   "read_len": (int(reads.lengths.max()) if reads.lengths.min() == reads.lengths.max()
                                else f"{int(reads.lengths.min())}-{int(reads.lengths.max())}"),
                   "seed_len": w.params.seed_len,
                   "seeds_per_read": w.params.n_min, "d_max": w.params.d_max, "conf_c": w.params.conf_c,
                   "max_hits": w.params.max_hits},
        "gbases_per_s": round(gbases_per_s, 4),
        "index_build_s": round(index_s, 2), "index_build": "host" if INDEX_ON_HOST else "device",
        "index_device_bytes": sizes["device_bytes"],
        "calls": {"not_found": int(calls[0]), "single": int(calls[1]), "multiple": int(calls[2])},
        "kernel_ms_per_step": {k: round(v[1] / args.steps, 4) for k, v in kern.items()},
        "counters_per_step": {k: v // max(args.steps, 1) for k, v in ctr.items()},
        "schedule": tune_info,
        "roofline": roofline,
        # the two phases the method hinges on: gather (HBM-bound) and verify (VALU-bound)
        "phases": phases_of(kern, ctr),
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    gix.close()


if __name__ == "__main__":
    main()
