"""HIP path vs the CPU oracle: bit-exact on all five outputs (pos, strand, dist,
second, call) for every read, on seeded synthetic workloads with the shapes of
the paper's (Section 2: uniform and repeat-rich genomes, 100 / 250 bp and longer
reads, substitutions and indels), plus edge cases and invariance checks.
All of this is integer work, so the tolerance is zero.
"""
import os

import numpy as np
import pytest

from helpers import compare, gpu_align, oracle_align, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def snapgpu(torch_cuda):
    import paper_1111_5572_amd as m
    m.lib()   # fails loudly if the HIP library is missing
    return m


def _world(synth_mod, workload, G, n):
    w = workload.scaled(genome_len=G, n_reads=n)
    g = w.make_genome()
    return w, g, w.make_reads(g)


def _check(snapgpu, oracle_mod, w, g, reads, label, params=None, d_max=None, ws=None, gix=None, oix=None):
    params = params or w.params
    d_max = params.d_max if d_max is None else d_max
    say(f"[{label}] G={len(g)} reads={reads.n} d_max={d_max} c={params.conf_c} hmax={params.max_hits}")
    own_g = gix is None
    gix = gix or snapgpu.Index(g, params.seed_len)
    gp = snapgpu.params_from(params)
    gout = gpu_align(snapgpu, gix, reads, d_max, gp, workspace_bytes=ws)
    own_o = oix is None
    oix = oix or oracle_mod.Index(g, params.seed_len)
    oout = oracle_align(oracle_mod, oix, reads, params)
    nbad, rep = compare(gout, oout, reads, label)
    if own_g:
        gix.close()
    if own_o:
        oix.close()
    assert nbad == 0, rep
    return gout


def test_tiny_full_config(snapgpu, oracle_mod, synth_mod):
    from synth.workloads import TINY
    g = TINY.make_genome()
    reads = TINY.make_reads(g)
    out = _check(snapgpu, oracle_mod, TINY, g, reads, "tiny")
    assert (out[4] == 1).mean() > 0.99


def test_mid_recipe_scaled(snapgpu, oracle_mod, synth_mod):
    from synth.workloads import MID
    w, g, reads = _world(synth_mod, MID, 3_000_000, 30_000)
    out = _check(snapgpu, oracle_mod, w, g, reads, "mid-scaled")
    calls = np.bincount(out[4], minlength=3)
    say(f"  calls not/single/multi = {calls.tolist()}")
    assert calls[2] > 0   # repeats produce ambiguous reads


def test_human_recipe_scaled_with_n(snapgpu, oracle_mod, synth_mod):
    from synth.workloads import HUMAN
    w, g, reads = _world(synth_mod, HUMAN, 3_000_000, 20_000)
    assert (g == ord("N")).mean() > 0.005
    _check(snapgpu, oracle_mod, w, g, reads, "human-scaled")


@pytest.mark.parametrize("c,hmax,dmax", [(1, 300, 10), (3, 300, 10), (2, 8, 10), (2, 60, 4), (2, 300, 0),
                                         (2, 2000, 8)])
def test_parameter_sweep(snapgpu, oracle_mod, synth_mod, c, hmax, dmax):
    from dataclasses import replace
    from synth.workloads import MID
    w, g, reads = _world(synth_mod, MID, 1_500_000, 8_000)
    p = replace(w.params, conf_c=c, max_hits=hmax, d_max=dmax)
    _check(snapgpu, oracle_mod, w, g, reads, f"sweep c={c} h={hmax} d={dmax}", params=p)


@pytest.mark.parametrize("copies", [1400, 5000])
def test_high_copy_family(snapgpu, oracle_mod, synth_mod, copies):
    """Reads from a high-copy repeat family: over 1024 and over 4096 candidate
    locations per read, more than a heavy-replay wave stages in LDS (its reads
    work in global memory), with hundreds of hits per seed."""
    from dataclasses import replace
    from synth.workloads import MID
    G = 2_000_000 if copies < 3000 else 3_000_000
    g = synth_mod.genome_family(G, 11, copies)
    reads = synth_mod.simulate_reads(g, 1000, 12, MID.reads)
    p = replace(MID.params, max_hits=2 * copies)
    # the family's seeds hit most copies
    oix = oracle_mod.Index(g, p.seed_len)
    first = [oix.occ(bytes(reads.bases[reads.offsets[i]:reads.offsets[i] + 20])) or [] for i in range(reads.n)]
    assert sum(len(o) > 0.5 * copies for o in first) > 50
    _check(snapgpu, oracle_mod, MID, g, reads, f"family x{copies}", params=p, oix=oix)
    oix.close()


def test_long_reads_percent_dmax(snapgpu, oracle_mod, synth_mod):
    """Reads 100-700 bp with d_max = ceil(0.08 L) and the long-read error model."""
    from dataclasses import replace
    from synth.workloads import BATCHED
    w = BATCHED.scaled(genome_len=2_000_000, n_reads=1500)
    w = replace(w, reads=replace(w.reads, len_b=700))
    g = w.make_genome()
    reads = w.make_reads(g)
    _check(snapgpu, oracle_mod, w, g, reads, "long-pct")


@pytest.mark.parametrize("len_a,len_b,n", [(300, 3000, 250), (3000, 10000, 16)])
def test_long_reads_wave_verify(snapgpu, oracle_mod, synth_mod, len_a, len_b, n):
    """Reads of 300 bp - 10 kb (5% error, half indels, d_max = ceil(0.08 L), limits
    up to 801): locations go to the wave-per-location verify."""
    from dataclasses import replace
    from synth.workloads import BATCHED
    w = BATCHED.scaled(genome_len=3_000_000, n_reads=n)
    w = replace(w, reads=replace(w.reads, len_a=len_a, len_b=len_b))
    g = w.make_genome()
    reads = w.make_reads(g)
    out = _check(snapgpu, oracle_mod, w, g, reads, f"long {len_a}-{len_b}")
    assert (out[4] > 0).mean() > 0.5


def test_mixed_lengths_batched_recipe(snapgpu, oracle_mod, synth_mod):
    """The batched recipe (log-uniform 100 bp - 10 kb) at reduced size: both verify
    tiles in one call."""
    from synth.workloads import BATCHED
    w = BATCHED.scaled(genome_len=3_000_000, n_reads=300)
    g = w.make_genome()
    reads = w.make_reads(g)
    _check(snapgpu, oracle_mod, w, g, reads, "batched-recipe")


def test_small_workspace_many_passes(snapgpu, oracle_mod, synth_mod):
    """The minimum workspace forces many internal passes; outputs are unchanged."""
    from synth.workloads import MID
    w, g, reads = _world(synth_mod, MID, 1_000_000, 6_000)
    gix = snapgpu.Index(g, 20)
    gp = snapgpu.params_from(w.params)
    full = gpu_align(snapgpu, gix, reads, w.params.d_max, gp)
    wmin = snapgpu.workspace_bytes(gix, reads.n, int(reads.bases.shape[0]), int(reads.lengths.max()),
                                   w.params.d_max, gp)
    # smaller than the recommended size but above the one-read minimum
    small = gpu_align(snapgpu, gix, reads, w.params.d_max, gp, workspace_bytes=max(wmin // 40, 1 << 20))
    nbad, rep = compare(small, full, reads, "small workspace vs default")
    gix.close()
    assert nbad == 0, rep


@pytest.mark.parametrize("seeds,limit,limit2,rounds,vseeds,chunk", [
    (0, 0, 0, 2, 0, 0), (1, 1, 0, 2, 0, 0), (2, 0, 0, 2, 1, 0), (3, 2, 5, 0, 0, 0), (4, 4, 0, 1, 2, 0),
    (4, 3, 7, 3, 0, 0), (6, 8, 9, 2, 3, 0), (32, 63, 0, 2, 0, 0), (1, 0, 3, 5, 0, 0), (6, 4, 4, 2, 0, 0),
    (6, 1, 1, 0, 5, 0), (0, 2, 2, 1, 3, 0), (8, 3, 3, 9, 1, 0), (6, 4, 4, 0, 0, 0), (5, 6, 6, 1, 3, 0),
    (0, 0, 0, 1, 2, 0), (5, 6, 6, 1, 0, 1000), (5, 6, 6, 1, 0, 2500), (0, 0, 0, 2, 0, 1500),
    (6, 4, 4, 0, 3, 700), (5, 6, 6, 1, 0, 7)])
def test_pass_schedule_invariance(snapgpu, oracle_mod, synth_mod, seeds, limit, limit2, rounds, vseeds, chunk):
    """The pass schedule (stage seeds, first verify limits, exact-request rounds, seeds covered by
    the first verification, reads per chunk and so one or two workers) never changes outputs."""
    from synth.workloads import MID
    w, g, reads = _world(synth_mod, MID, 1_000_000, 6_000)
    old = snapgpu.get_tuning()
    try:
        snapgpu.set_tuning(seeds, limit, limit2, 0, rounds, vseeds, chunk)
        _check(snapgpu, oracle_mod, w, g, reads, f"schedule {seeds}/{limit}/{limit2}/{rounds}/{vseeds}/{chunk}")
    finally:
        snapgpu.set_tuning(*old)


@pytest.mark.parametrize("top", [1, 2, 8, 16])
def test_request_top_invariance(snapgpu, oracle_mod, synth_mod, top):
    """How many best-voted undecided locations a single-location request takes changes the
    verification rounds, never the outputs: 100 and 250 bp reads at d_max 15 (reads with
    more than 64 locations in the repeats), exact requests for up to 5 rounds."""
    from synth.workloads import HUMAN
    w, g, reads = _world(synth_mod, HUMAN, 2_000_000, 8_000)
    old = snapgpu.get_tuning()
    try:
        snapgpu.set_tuning(5, 6, 6, 0, 5, 0, 0, 0, top)
        _check(snapgpu, oracle_mod, w, g, reads, f"request_top {top}")
    finally:
        snapgpu.set_tuning(*old)


@pytest.mark.parametrize("max_len,seeds,chunk", [(99, 5, 0), (100, 5, 0), (128, 5, 0), (249, 5, 0), (250, 5, 0),
                                                   (128, 3, 1500), (128, 0, 0), (128, 6, 0)])
def test_long_read_first_pass_invariance(snapgpu, oracle_mod, synth_mod, max_len, seeds, chunk):
    """Reads longer than pass1_max_len take every seed slot in one complete pass over their own
    list, the others the first and the final pass: outputs never change. 100 and 250 bp reads
    at d_max 15, bounds on either side of both lengths and at them (a read of exactly that
    length stays in the two passes), small chunks (several chunks a pass and two workers), and
    no first stage at all (pass1_seeds 0: nothing to split)."""
    from synth.workloads import HUMAN
    w, g, reads = _world(synth_mod, HUMAN, 2_000_000, 8_000)
    old = snapgpu.get_tuning()
    try:
        snapgpu.set_tuning(seeds, 7, 7, 0, 5, 0, chunk, 2, 4, max_len)
        _check(snapgpu, oracle_mod, w, g, reads, f"pass1_max_len {max_len} seeds {seeds} chunk {chunk}")
    finally:
        snapgpu.set_tuning(*old)


def test_long_read_first_pass_counters(snapgpu, oracle_mod, synth_mod):
    """With the long reads' complete pass, the profiling counters still count every read of
    the batch once as the batch's and only the short reads a first pass left as later-pass
    reads (both first-stage passes run over read lists)."""
    from synth.workloads import HUMAN
    w, g, reads = _world(synth_mod, HUMAN, 2_000_000, 8_000)
    n_long = int((reads.lengths > 128).sum())
    old = snapgpu.get_tuning()
    try:
        snapgpu.set_tuning(5, 7, 7, 0, 5, 0, 1500, 2, 4, 128)
        snapgpu.profile_begin()
        _check(snapgpu, oracle_mod, w, g, reads, "pass1_max_len 128, counters")
        ctr = snapgpu.profile_counters()
        snapgpu.profile_end()
        say(f"counters {ctr}; long reads {n_long}")
        assert 0 < n_long < reads.n
        assert ctr["reads"] == reads.n, ctr
        assert 0 <= ctr["second_pass_reads"] <= reads.n - n_long, ctr
    finally:
        snapgpu.set_tuning(*old)


def test_long_read_first_pass_mixed_wave_tile(snapgpu, oracle_mod, synth_mod):
    """The same on the batched recipe at reduced size (log-uniform 100 bp - 10 kb, d_max 8% of
    the length): the long reads' complete pass runs the wave tile."""
    from synth.workloads import BATCHED
    w = BATCHED.scaled(genome_len=3_000_000, n_reads=300)
    g = w.make_genome()
    reads = w.make_reads(g)
    old = snapgpu.get_tuning()
    try:
        snapgpu.set_tuning(5, 6, 6, 0, 1, 0, 0, 0, 0, 300)
        _check(snapgpu, oracle_mod, w, g, reads, "pass1_max_len 300, batched recipe")
    finally:
        snapgpu.set_tuning(*old)


def test_batch_composition_invariance(snapgpu, synth_mod):
    """A read's output does not depend on the other reads in the batch or their order."""
    from synth.workloads import MID
    w, g, reads = _world(synth_mod, MID, 1_000_000, 5_000)
    gix = snapgpu.Index(g, 20)
    gp = snapgpu.params_from(w.params)
    full = gpu_align(snapgpu, gix, reads, w.params.d_max, gp)
    rng = np.random.default_rng(3)
    perm = rng.permutation(reads.n)
    sub = reads.subset(perm)
    shuf = gpu_align(snapgpu, gix, sub, w.params.d_max, gp)
    back = tuple(np.empty_like(x) for x in shuf)
    for b, s in zip(back, shuf):
        b[perm] = s
    nbad, rep = compare(back, full, reads, "shuffled vs original")
    assert nbad == 0, rep
    few = perm[:37]
    part = gpu_align(snapgpu, gix, reads.subset(few), w.params.d_max, gp)
    nbad, rep = compare(part, tuple(x[few] for x in full), None, "subset vs full")
    gix.close()
    assert nbad == 0, rep


def test_edge_cases(snapgpu, oracle_mod, synth_mod):
    """Empty batch; reads shorter than s, of length exactly s; N-rich reads; reads at
    the genome ends; identical reads in one batch."""
    import torch
    import synth
    g = synth_mod.genome_uniform(200_000, 9)
    gs = g.tobytes().decode()
    seqs = ["", "ACGT", gs[10:29], gs[10:30], gs[0:100], gs[-100:], "N" * 100,
            gs[500:550] + "N" + gs[551:600], gs[700:800].lower(), gs[900:1000], gs[900:1000],
            gs[5000:5250], "ACGTX" * 20]
    lens = np.array([len(x) for x in seqs], np.int32)
    offs = np.zeros(len(seqs) + 1, np.int64)
    np.cumsum(lens, out=offs[1:])
    bases = np.frombuffer("".join(seqs).encode(), np.uint8).copy()
    n = len(seqs)
    reads = synth.Reads(bases, lens, offs, np.zeros(n, np.int64), np.zeros(n, np.int8), np.zeros(n, np.int32))
    from synth.workloads import TINY
    gix = snapgpu.Index(g, 20)
    oix = oracle_mod.Index(g, 20)
    gp = snapgpu.params_from(TINY.params)
    gout = gpu_align(snapgpu, gix, reads, 8, gp)
    oout = oracle_align(oracle_mod, oix, reads, TINY.params)
    nbad, rep = compare(gout, oout, reads, "edges")
    assert nbad == 0, rep
    # empty batch
    dev = torch.device("cuda:0")
    empty = snapgpu.align(gix, torch.empty(0, dtype=torch.uint8, device=dev),
                          torch.empty(0, dtype=torch.int32, device=dev), 8, gp, max_len=0)
    assert empty.pos.numel() == 0
    gix.close()
    oix.close()


@pytest.mark.parametrize("misaligned", [False, True])
def test_read_bytes_any_case_and_codes(snapgpu, oracle_mod, synth_mod, misaligned):
    """Reads with lowercase bases and bytes that are not bases (IUPAC codes, punctuation,
    0x00, bytes with the high bit set): A, C, G, T in either case are bases, every
    other byte is N. The batch is passed 16-byte aligned (word-wise decode) and one byte
    off (byte-wise decode)."""
    import torch
    from synth.workloads import TINY
    w = TINY.scaled(genome_len=300_000, n_reads=3_000)
    g = w.make_genome()
    reads = w.make_reads(g)
    rng = np.random.default_rng(21)
    b = reads.bases.copy()
    low = rng.random(b.size) < 0.15
    b[low] = b[low] + 32
    odd = rng.random(b.size) < 0.004
    junk = np.frombuffer(b"RYKMSWBDHVNX-.@`{0\x00\xff\xc1\xe1\xd4", dtype=np.uint8)
    b[odd] = junk[rng.integers(0, junk.size, int(odd.sum()))]
    reads.bases = b
    gix = snapgpu.Index(g, 20)
    oix = oracle_mod.Index(g, 20)
    gp = snapgpu.params_from(w.params)
    dev = torch.device("cuda:0")
    if misaligned:
        whole = torch.from_numpy(np.concatenate([np.zeros(1, np.uint8), b])).to(dev)
        rb = whole[1:]
        assert rb.data_ptr() % 16 != 0
    else:
        rb = torch.from_numpy(b).to(dev)
    ln = torch.from_numpy(reads.lengths).to(dev)
    out = snapgpu.align(gix, rb, ln, w.params.d_max, gp, max_len=int(reads.lengths.max()))
    torch.cuda.synchronize()
    gout = out.numpy()
    oout = oracle_align(oracle_mod, oix, reads, w.params)
    nbad, rep = compare(gout, oout, reads, f"read bytes misaligned={misaligned}")
    gix.close()
    oix.close()
    assert nbad == 0, rep


def test_invalid_arguments(snapgpu, synth_mod):
    import torch
    g = synth_mod.genome_uniform(10_000, 1)
    gix = snapgpu.Index(g, 20)
    dev = torch.device("cuda:0")
    rb = torch.zeros(100, dtype=torch.uint8, device=dev)
    ln = torch.full((1,), 100, dtype=torch.int32, device=dev)
    with pytest.raises(snapgpu.SnapError):
        snapgpu.align(gix, rb, ln, -1)
    with pytest.raises(snapgpu.SnapError):
        snapgpu.align(gix, rb, ln, 8, snapgpu.default_params(conf_c=0))
    with pytest.raises(snapgpu.SnapError):
        snapgpu.align(gix, rb, ln, 8, snapgpu.default_params(n_cap=33))
    with pytest.raises(snapgpu.SnapError):
        snapgpu.align(gix, rb, ln, snapgpu.max_limit() + 5)
    with pytest.raises(snapgpu.SnapError):
        snapgpu.Index(b"ACGT", 20)
    gix.close()


def test_mid_full_size_sampled(snapgpu, oracle_mod, synth_mod):
    """The mid workload at full size (100 Mbase, 10M reads) in the launch
    configuration the benchmark times; the oracle re-computes a seeded sample."""
    if os.environ.get("SNAP_SKIP_FULL"):
        pytest.skip("SNAP_SKIP_FULL set")
    from synth.workloads import MID
    g = MID.make_genome()
    say("[mid-full] genome ready")
    reads = MID.make_reads(g)
    say("[mid-full] reads ready")
    gix = snapgpu.Index(g, 20)
    say("[mid-full] GPU index ready")
    gp = snapgpu.params_from(MID.params)
    gout = gpu_align(snapgpu, gix, reads, MID.params.d_max, gp)
    say("[mid-full] GPU aligned")
    gix.close()
    rng = np.random.default_rng(2024)
    idx = np.sort(rng.choice(reads.n, 3000, replace=False))
    sub = reads.subset(idx)
    oix = oracle_mod.Index(g, 20)
    say("[mid-full] oracle index ready")
    oout = oracle_align(oracle_mod, oix, sub, MID.params)
    oix.close()
    nbad, rep = compare(tuple(x[idx] for x in gout), oout, sub, "mid-full sample")
    assert nbad == 0, rep
    calls = np.bincount(gout[4], minlength=3)
    say(f"  calls not/single/multi = {calls.tolist()}")


@pytest.mark.gpu
@pytest.mark.parametrize("workers", [2, 3, 4])
def test_chunk_workers(snapgpu, oracle_mod, synth_mod, workers):
    """A batch of several chunks with a workspace for several chunk parts is worked by
    that many host threads with a stream each; outputs equal the oracle's."""
    from synth.workloads import MID
    w, g, reads = _world(synth_mod, MID, 1_000_000, 8_000)
    old = snapgpu.get_tuning()
    try:
        snapgpu.set_tuning(5, 6, 6, 0, 1, 0, 1500, workers)
        snapgpu.profile_begin()
        _check(snapgpu, oracle_mod, w, g, reads, f"{workers} workers, chunks of 1500 reads",
               ws=1 << 30)
        ctr = snapgpu.profile_counters()
        snapgpu.profile_end()
        say(f"counters {ctr}")
        assert ctr["workers"] == workers, ctr
        assert ctr["passes"] >= 6, ctr
    finally:
        snapgpu.set_tuning(*old)
