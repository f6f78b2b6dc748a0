"""Limits at the edges of the verify tiles, reads at the length limit and long reads
holding N, against the oracle (bit-exact on all five outputs).

The lane tile (a lane per location) takes reads whose full limit d_max(L) + c - 1 is at
most 63; above it a read's locations go to the wave tile, also when a pass verifies with
a smaller capped limit first (the library's default schedule caps the first limit at 6).
"""
import numpy as np
import pytest

from helpers import compare, gpu_align, oracle_align, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def snapgpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1111_5572_amd as m
    m.lib()
    return m


@pytest.fixture(scope="module")
def world(synth_mod):
    from synth.workloads import MID
    w = MID.scaled(genome_len=1_000_000, n_reads=1500)
    g = w.make_genome()
    return w, g, w.make_reads(g)


@pytest.mark.parametrize("d_max", [61, 62, 63, 64, 120])
@pytest.mark.parametrize("tuning", ["default", "uncapped"])
def test_limits_around_the_lane_tile_bound(snapgpu, oracle_mod, world, d_max, tuning):
    """100 bp reads at d_max 61..64 (full limits 62..65 with c = 2) and 120: the reads
    straddle the lane tile's bound of 63, under the capped default schedule and with
    no cap. Each call must end (the request loop is bounded) and equal the oracle."""
    from dataclasses import replace
    w, g, reads = world
    p = replace(w.params, d_max=d_max)
    old = snapgpu.get_tuning()
    try:
        if tuning == "default":
            snapgpu.set_tuning(5, 6, 6, 0, 1, 0, 0, 0)
        else:
            snapgpu.set_tuning(0, 0, 0, 0, 1, 0, 0, 0)
        say(f"[limits] d_max={d_max} tuning={tuning} reads={reads.n}")
        gix = snapgpu.Index(g, 20)
        gout = gpu_align(snapgpu, gix, reads, d_max, snapgpu.params_from(p))
        gix.close()
    finally:
        snapgpu.set_tuning(*old)
    oix = oracle_mod.Index(g, 20)
    oout = oracle_align(oracle_mod, oix, reads, p)
    oix.close()
    nbad, rep = compare(gout, oout, reads, f"d_max {d_max} {tuning}")
    assert nbad == 0, rep


def test_read_over_the_length_limit_is_refused(snapgpu, synth_mod):
    """A read of 16,385 bases (one over the limit) makes snap_align return SNAP_EINVAL
    before any device work; 16,384 is accepted."""
    import torch
    g = synth_mod.genome_uniform(100_000, 3)
    gix = snapgpu.Index(g, 20)
    dev = torch.device("cuda:0")
    p = snapgpu.default_params(d_max_pct=0)
    # a workspace sized for the longest accepted read, so that the over-long read reaches
    # snap_align's own check rather than the workspace query's
    wb = snapgpu.workspace_bytes(gix, 1, 16_385, 16_384, 8, p)
    assert wb > 0
    ws = torch.empty(2 * wb, dtype=torch.uint8, device=dev)
    assert snapgpu.workspace_bytes(gix, 1, 16_385, 16_385, 8, p) == 0
    for L, ok in ((16_384, True), (16_385, False)):
        rb = torch.from_numpy(np.resize(g, L).copy()).to(dev)
        ln = torch.full((1,), L, dtype=torch.int32, device=dev)
        say(f"[length limit] L={L}")
        if ok:
            out = snapgpu.align(gix, rb, ln, 8, p, workspace=ws, max_len=L)
            torch.cuda.synchronize()
            assert int(out.call[0]) in (0, 1, 2)
        else:
            with pytest.raises(snapgpu.SnapError) as ei:
                snapgpu.align(gix, rb, ln, 8, p, workspace=ws, max_len=L)
            assert ei.value.code == snapgpu.SNAP_EINVAL
    gix.close()


def test_long_reads_with_n(snapgpu, oracle_mod, synth_mod):
    """Reads of 600 bp - 3 kb (wave tile) with runs and single bases of N planted in the
    read: N matches nothing, a seed holding one is not looked up."""
    import synth
    from dataclasses import replace
    from synth.workloads import BATCHED
    w = BATCHED.scaled(genome_len=2_000_000, n_reads=120)
    w = replace(w, reads=replace(w.reads, len_a=600, len_b=3000))
    g = w.make_genome()
    reads = w.make_reads(g)
    rng = np.random.default_rng(31)
    b = reads.bases.copy()
    for i in range(reads.n):
        o, L = int(reads.offsets[i]), int(reads.lengths[i])
        if i % 3 == 0:   # a run of 1-40 N
            a = int(rng.integers(0, L - 40))
            b[o + a:o + a + int(rng.integers(1, 41))] = ord("N")
        if i % 3 != 2:   # scattered single N
            k = rng.choice(L, size=max(1, L // 400), replace=False)
            b[o + k] = ord("N")
    reads = synth.Reads(b, reads.lengths, reads.offsets, reads.truth_pos, reads.truth_strand, reads.truth_edits)
    say(f"[long N] reads={reads.n} N bases={int((b == ord('N')).sum())}")
    gix = snapgpu.Index(g, 20)
    gout = gpu_align(snapgpu, gix, reads, w.params.d_max, snapgpu.params_from(w.params))
    gix.close()
    oix = oracle_mod.Index(g, 20)
    oout = oracle_align(oracle_mod, oix, reads, w.params)
    oix.close()
    nbad, rep = compare(gout, oout, reads, "long reads with N")
    assert nbad == 0, rep
    assert (gout[4] > 0).mean() > 0.5
