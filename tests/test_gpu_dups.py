"""Exact-duplicate classes (Section 4.2, "Approach") on the GPU: the class array built on
the device equals the oracle's (the smallest position with an identical W-base window,
N equal to N, windows past the end their own class), bit for bit; and alignments with
the classes attached (one verification per class and strand within a read) equal those
without them and the oracle's on all five outputs, while the classes answer a share of
the locations."""
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


def _tandem_genome(synth_mod):
    """Repeat recipe with N runs, plus exact tandem arrays and an exact 3-copy block."""
    g = synth_mod.genome_repeats(400_000, 5, n_frac=0.02).copy()
    rng = np.random.default_rng(11)
    unit = rng.integers(0, 4, 7)
    g[50_000:52_000] = np.frombuffer(b"ACGT", np.uint8)[np.tile(unit, 2_000 // 7 + 1)[:2_000]]
    block = g[100_000:100_600].copy()
    g[200_000:200_600] = block
    g[300_000:300_600] = block
    g[10_000:10_005] = ord("n")
    return g


@pytest.mark.parametrize("W", [1, 20, 111, 266])
def test_classes_equal_oracle(snapgpu, oracle_mod, synth_mod, W):
    g = _tandem_genome(synth_mod)
    ix = snapgpu.Index(g, 20, on_device=True)
    ix.dup_classes(W)
    got = ix.download_dup_classes()
    sz = ix.sizes()
    ix.close()
    want = oracle_mod.dup_classes(g, W)
    bad = np.nonzero(got.astype(np.int64) != want)[0]
    say(f"[classes W={W}] G={len(g)} non-trivial={int((want != np.arange(len(g))).sum())} window={sz['dup_window']}")
    assert sz["dup_window"] == W
    assert bad.size == 0, f"{bad.size} positions differ, first {bad[:10].tolist()}"


def test_classes_window_longer_than_genome(snapgpu, oracle_mod, synth_mod):
    g = synth_mod.genome_uniform(5_000, 3)
    ix = snapgpu.Index(g, 20, on_device=True)
    ix.dup_classes(6_000)
    got = ix.download_dup_classes()
    ix.close()
    assert np.array_equal(got.astype(np.int64), oracle_mod.dup_classes(g, 6_000))
    assert np.array_equal(got, np.arange(5_000, dtype=np.uint32))


def _align_both(snapgpu, torch, g, reads, params, W, label, batched=False):
    """GPU outputs without and with classes of W-base windows, and the alias count."""
    import paper_1111_5572_amd as m
    ix = snapgpu.Index(g, params.seed_len, on_device=True)
    gp = snapgpu.params_from(params)
    dev = torch.device("cuda:0")
    rb = torch.from_numpy(np.ascontiguousarray(reads.bases)).to(dev)
    ln = torch.from_numpy(np.ascontiguousarray(reads.lengths)).to(dev)
    ml = int(reads.lengths.max())
    plain = snapgpu.align(ix, rb, ln, params.d_max, gp, max_len=ml, batched=batched).numpy()
    ix.dup_classes(W)
    m.profile_begin()
    with_dups = snapgpu.align(ix, rb, ln, params.d_max, gp, max_len=ml, batched=batched).numpy()
    torch.cuda.synchronize()
    m.profile_end()
    ctr = m.profile_counters()
    ix.close()
    say(f"[{label}] W={W} reads={reads.n} locations={ctr['locations']} aliases={ctr['dup_aliases']}")
    for name, a, b in zip(("pos", "strand", "dist", "second", "call"), with_dups, plain):
        assert np.array_equal(np.asarray(a, np.int64), np.asarray(b, np.int64)), f"{label}: {name} changed"
    return with_dups, ctr


def test_alignment_with_classes_mid_recipe(snapgpu, torch_cuda, oracle_mod, synth_mod):
    """100 bp reads, d_max 10: windows of L + d_max + c - 1 = 111 bases."""
    from synth.workloads import MID
    w = MID.scaled(genome_len=3_000_000, n_reads=20_000)
    g = w.make_genome()
    reads = w.make_reads(g)
    out, ctr = _align_both(snapgpu, torch_cuda, g, reads, w.params, 111, "mid-scaled")
    assert ctr["dup_aliases"] > 0
    oix = oracle_mod.Index(g, w.params.seed_len)
    nbad, rep = compare(out, oracle_align(oracle_mod, oix, reads, w.params), reads, "mid with classes")
    oix.close()
    assert nbad == 0, rep


def test_alignment_with_classes_mixed_lengths(snapgpu, torch_cuda, oracle_mod, synth_mod):
    """100 and 250 bp reads at d_max 15 with classes of 116-base windows: only the 100 bp
    reads can use them (250 + 16 > 116); then 266-base windows, which both use."""
    from synth.workloads import HUMAN
    w = HUMAN.scaled(genome_len=3_000_000, n_reads=12_000)
    g = w.make_genome()
    reads = w.make_reads(g)
    oix = oracle_mod.Index(g, w.params.seed_len)
    want = oracle_align(oracle_mod, oix, reads, w.params)
    oix.close()
    for W in (116, 266):
        out, ctr = _align_both(snapgpu, torch_cuda, g, reads, w.params, W, f"human-scaled W {W}")
        nbad, rep = compare(out, want, reads, f"human with classes W {W}")
        assert nbad == 0, rep


def test_alignment_with_classes_tandem_genome_and_batched(snapgpu, torch_cuda, oracle_mod, synth_mod):
    """Exact tandem arrays and copies: reads from them have many aliased locations (in the
    heavy replay too); the plain and the batched form, both strands."""
    import synth
    from dataclasses import replace
    from synth.workloads import MID
    g = _tandem_genome(synth_mod)
    model = synth.ReadModel(len_mode=2, len_a=60, len_b=400, p_sub=0.01, p_indel=0.001, indel_max=3)
    reads = synth.simulate_reads(g, 6_000, 31, model)
    params = replace(MID.params, d_max=8, max_hits=2000)
    oix = oracle_mod.Index(g, params.seed_len)
    want = oracle_align(oracle_mod, oix, reads, params)
    oix.close()
    for batched in (False, True):
        out, ctr = _align_both(snapgpu, torch_cuda, g, reads, params, 420, f"tandem batched={batched}", batched)
        assert ctr["dup_aliases"] > 0
        nbad, rep = compare(out, want, reads, f"tandem with classes batched={batched}")
        assert nbad == 0, rep
