"""Batched form (snap_align_batched: one persistent work-stealing verify launch
per pass over reads of mixed length) vs the oracle and vs the plain form:
identical outputs on every field, whatever the schedule and tile bound."""
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


def batched_align(snapgpu, index, reads, d_max, params, tuning=None):
    import torch
    dev = torch.device("cuda:0")
    rb = torch.from_numpy(reads.bases).to(dev)
    ln = torch.from_numpy(reads.lengths).to(dev)
    out = snapgpu.align(index, rb, ln, d_max, params, batched=True, tuning=tuning,
                        max_len=int(reads.lengths.max()))
    torch.cuda.synchronize()
    return out.numpy()


@pytest.fixture(scope="module")
def mixed(synth_mod):
    from synth.workloads import BATCHED
    w = BATCHED.scaled(genome_len=3_000_000, n_reads=300)
    g = w.make_genome()
    return w, g, w.make_reads(g)


def test_batched_vs_oracle(snapgpu, oracle_mod, mixed):
    w, g, reads = mixed
    say(f"[batched] reads={reads.n} max_len={int(reads.lengths.max())}")
    gix = snapgpu.Index(g, 20)
    gp = snapgpu.params_from(w.params)
    got = batched_align(snapgpu, gix, reads, w.params.d_max, gp)
    gix.close()
    oix = oracle_mod.Index(g, 20)
    want = oracle_align(oracle_mod, oix, reads, w.params)
    oix.close()
    nbad, rep = compare(got, want, reads, "batched vs oracle")
    assert nbad == 0, rep


@pytest.mark.parametrize("tuning", [(0, 0, 0, 0), (4, 4, 0, 0), (2, 3, 8, 128), (6, 10, 40, 512), (1, 1, 0, 64),
                                    (3, 0, 0, 300), (6, 3, 3, 0, 0), (6, 2, 2, 256, 1)])
def test_batched_schedule_and_tile_invariance(snapgpu, mixed, tuning):
    w, g, reads = mixed
    gix = snapgpu.Index(g, 20)
    gp = snapgpu.params_from(w.params)
    ref = gpu_align(snapgpu, gix, reads, w.params.d_max, gp)
    got = batched_align(snapgpu, gix, reads, w.params.d_max, gp, tuning)
    gix.close()
    nbad, rep = compare(got, ref, reads, f"batched {tuning} vs plain")
    assert nbad == 0, rep


def test_batched_equals_plain_on_short_reads(snapgpu, synth_mod):
    from synth.workloads import MID
    w = MID.scaled(genome_len=2_000_000, n_reads=20_000)
    g = w.make_genome()
    reads = w.make_reads(g)
    gix = snapgpu.Index(g, 20)
    gp = snapgpu.params_from(w.params)
    ref = gpu_align(snapgpu, gix, reads, w.params.d_max, gp)
    got = batched_align(snapgpu, gix, reads, w.params.d_max, gp, (4, 4, 0, 0))
    gix.close()
    nbad, rep = compare(got, ref, reads, "batched vs plain (100 bp)")
    assert nbad == 0, rep
