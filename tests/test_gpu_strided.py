"""The strided index (Section 3.1, the footnote to overlapping seeds: windows slid
`stride` bases at a time) on the GPU against the oracle's strided index, bit-exact on
all five outputs, plus the index's size and contents against a brute-force scan.

Reading (shared with the oracle, which states it in full): only windows at multiples
of the stride are indexed; each seed slot at read offset o looks up the seeds at
o .. o + stride - 1 that fit the read, is skipped for an N in any of them, is over h_max
on the sum of their entries, votes once per location, and counts in t only as a round-0
slot whose stride seeds all fit.
"""
import numpy as np
import pytest

from helpers import compare, gpu_align, oracle_threads, say

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


def _check(snapgpu, oracle_mod, g, reads, wparams, stride, label, d_max=None):
    d_max = wparams.d_max if d_max is None else d_max
    say(f"[{label}] stride={stride} G={len(g)} reads={reads.n} d_max={d_max} hmax={wparams.max_hits}")
    gix = snapgpu.Index(g, wparams.seed_len, stride=stride)
    sz = gix.sizes()
    gout = gpu_align(snapgpu, gix, reads, d_max, snapgpu.params_from(wparams))
    gix.close()
    oix = oracle_mod.Index(g, wparams.seed_len, threads=oracle_threads(), stride=stride)
    op = oracle_mod.params_from(wparams)
    op.d_max = d_max
    res = oix.align_reads(reads, op, threads=oracle_threads())
    oix.close()
    nbad, rep = compare(gout, res.fields(), reads, label)
    assert nbad == 0, rep
    return gout, sz, res.stats


@pytest.mark.parametrize("stride", [2, 4])
def test_strided_index_contents(snapgpu, oracle_mod, synth_mod, stride):
    """The strided index holds exactly the N-free windows at multiples of the stride:
    the positions array (a position per window and orientation, palindromes twice)
    against a scan of the genome."""
    from synth.workloads import HUMAN
    w = HUMAN.scaled(genome_len=300_000)
    g = w.make_genome()
    s = w.params.seed_len
    gix = snapgpu.Index(g, s, stride=stride)
    sz = gix.sizes()
    pos = gix.download("positions")
    gix.close()
    isn = ~np.isin(g, np.frombuffer(b"ACGTacgt", np.uint8))
    nwin = len(g) - s + 1
    bad = np.convolve(isn.astype(np.int32), np.ones(s, np.int32), "valid")[:nwin] > 0
    q = np.arange(nwin)
    want = q[(~bad) & (q % stride == 0)]
    say(f"[contents] stride={stride} windows={sz['windows']} want={len(want)} entries={sz['position_entries']}")
    assert sz["stride"] == stride and sz["windows"] == len(want)
    assert np.all(pos % stride == 0)
    assert np.array_equal(np.unique(pos), want)


def test_strided_mid_recipe(snapgpu, oracle_mod, synth_mod):
    from synth.workloads import MID
    w = MID.scaled(genome_len=3_000_000, n_reads=20_000)
    g = w.make_genome()
    reads = w.make_reads(g)
    out, sz, st = _check(snapgpu, oracle_mod, g, reads, w.params, 2, "mid-scaled stride 2")
    calls = np.bincount(out[4], minlength=3)
    say(f"  calls not/single/multi = {calls.tolist()}; index windows {sz['windows']}; oracle {st}")
    assert calls[1] > 0.5 * reads.n


def test_strided_human_recipe_mixed_lengths_with_n(snapgpu, oracle_mod, synth_mod):
    """100 and 250 bp reads, N runs in the genome, d_max 15, stride 2."""
    from synth.workloads import HUMAN
    w = HUMAN.scaled(genome_len=3_000_000, n_reads=12_000)
    g = w.make_genome()
    reads = w.make_reads(g)
    _check(snapgpu, oracle_mod, g, reads, w.params, 2, "human-scaled stride 2")


def test_strided_stride4_and_parameter_sweep(snapgpu, oracle_mod, synth_mod):
    """Stride 4 (16 seed slots at most: 64 probe records a read), c 1 and 3, h_max 8
    and 60 (the per-slot sum decides), short reads whose last round-0 slot is not
    complete (t counts fewer slots)."""
    from dataclasses import replace
    from synth.workloads import MID
    import synth
    w = MID.scaled(genome_len=2_000_000, n_reads=8_000)
    g = w.make_genome()
    reads = w.make_reads(g)
    for stride, c, hmax in ((4, 2, 300), (2, 1, 60), (2, 3, 8), (4, 1, 60)):
        p = replace(w.params, conf_c=c, max_hits=hmax, n_cap=16)
        _check(snapgpu, oracle_mod, g, reads, p, stride, f"sweep stride {stride} c {c} hmax {hmax}")
    # lengths around s + stride - 1 and multiples of s (which round-0 slots are complete)
    model = synth.ReadModel(len_mode=2, len_a=19, len_b=84, p_sub=0.01, p_indel=0.001, indel_max=3)
    short = synth.simulate_reads(g, 6_000, 77, model)
    for stride in (2, 4):
        _check(snapgpu, oracle_mod, g, short, replace(w.params, n_cap=16), stride, f"short reads stride {stride}")


def test_strided_refuses_too_many_records_per_read(snapgpu, torch_cuda, synth_mod):
    """Stride 4 with 32 seed slots would need 128 probe records a read: SNAP_EINVAL."""
    from dataclasses import replace
    from synth.workloads import MID
    import synth
    w = MID.scaled(genome_len=200_000, n_reads=100)
    g = w.make_genome()
    model = synth.ReadModel(len_mode=0, len_a=3200, len_b=3200, p_sub=0.01, p_indel=0.0, indel_max=1)
    reads = synth.simulate_reads(g, 10, 5, model)
    gix = snapgpu.Index(g, 20, stride=4)
    with pytest.raises(snapgpu.SnapError) as e:
        gpu_align(snapgpu, gix, reads, 8, snapgpu.params_from(replace(w.params, n_cap=32)))
    assert e.value.code == snapgpu.SNAP_EINVAL
    gix.close()
