"""snap_align_noalloc (the entry point that allocates nothing: its scratch is a fixed
array per device) against snap_align with a caller workspace: all five outputs equal
on every read, on two calls in a row (the second with a smaller batch, so the scratch
holds the first call's contents), and against the oracle; a batch larger than the
scratch is refused with SNAP_ETOOBIG before any output is written."""
import numpy as np
import pytest

from helpers import FIELDS, compare, oracle_align, say

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


def _outputs(torch, n, dev, fill):
    import paper_1111_5572_amd as m
    return m.Alignment(torch.full((n,), fill, dtype=torch.int64, device=dev),
                       torch.full((n,), fill, dtype=torch.int8, device=dev),
                       torch.full((n,), fill, dtype=torch.int32, device=dev),
                       torch.full((n,), fill, dtype=torch.int32, device=dev),
                       torch.full((n,), fill, dtype=torch.int8, device=dev))


def _both(torch, snapgpu, gix, reads, d_max, params, label):
    """snap_align (caller workspace) and snap_align_noalloc on the same batch; numpy outputs."""
    dev = torch.device("cuda:0")
    rb = torch.from_numpy(np.ascontiguousarray(reads.bases)).to(dev)
    ln = torch.from_numpy(np.ascontiguousarray(reads.lengths)).to(dev)
    ml = int(reads.lengths.max())
    need = snapgpu.workspace_bytes(gix, reads.n, int(reads.bases.shape[0]), ml, d_max, params)
    say(f"[{label}] reads={reads.n} bases={int(reads.bases.shape[0])} workspace_bytes={need} "
        f"scratch={snapgpu.noalloc_scratch_bytes()}")
    assert need <= snapgpu.noalloc_scratch_bytes()
    ref = snapgpu.align(gix, rb, ln, d_max, params, max_len=ml)
    torch.cuda.synchronize()
    out = _outputs(torch, reads.n, dev, 7)
    free0 = torch.cuda.mem_get_info()[0]
    snapgpu.align_noalloc(gix, rb, ln, d_max, params, out)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    say(f"[{label}] device free bytes before / after the call: {free0} / {free1}")
    assert free1 >= free0, "snap_align_noalloc took device memory"
    return ref.numpy(), out.numpy()


def test_noalloc_equals_workspace_form_twice(snapgpu, torch_cuda, oracle_mod, synth_mod):
    torch = torch_cuda
    from synth.workloads import MID
    w = MID.scaled(genome_len=2_000_000, n_reads=20_000)
    g = w.make_genome()
    reads = w.make_reads(g)
    gix = snapgpu.Index(g, w.params.seed_len, on_device=True)
    oix = oracle_mod.Index(g, w.params.seed_len)
    params = snapgpu.params_from(w.params)
    # first call: 20,000 reads; second: a smaller batch of other reads (the scratch still
    # holds the first call's contents)
    second = reads.subset(np.arange(5_000, 12_000))
    for label, batch in (("first, 20000 reads", reads), ("second, 7000 reads", second)):
        ref, got = _both(torch, snapgpu, gix, batch, w.params.d_max, params, label)
        for name, a, b in zip(FIELDS, got, ref):
            bad = np.nonzero(np.asarray(a, np.int64) != np.asarray(b, np.int64))[0]
            assert bad.size == 0, f"{label}: {name} differs from snap_align at reads {bad[:10].tolist()}"
        nbad, rep = compare(got, oracle_align(oracle_mod, oix, batch, w.params), batch, label)
        assert nbad == 0, rep
    gix.close()
    oix.close()


def test_noalloc_refuses_a_batch_beyond_the_scratch(snapgpu, torch_cuda, synth_mod):
    torch = torch_cuda
    from synth.workloads import TINY
    w = TINY.scaled(genome_len=200_000, n_reads=400_000)
    g = w.make_genome()
    reads = w.make_reads(g)
    gix = snapgpu.Index(g, w.params.seed_len, on_device=True)
    params = snapgpu.params_from(w.params)
    need = snapgpu.workspace_bytes(gix, reads.n, int(reads.bases.shape[0]), 100, w.params.d_max, params)
    say(f"[too big] reads={reads.n} workspace_bytes={need} scratch={snapgpu.noalloc_scratch_bytes()}")
    assert need > snapgpu.noalloc_scratch_bytes()
    dev = torch.device("cuda:0")
    rb = torch.from_numpy(reads.bases).to(dev)
    ln = torch.from_numpy(reads.lengths).to(dev)
    out = _outputs(torch, reads.n, dev, 7)
    with pytest.raises(snapgpu.SnapError) as e:
        snapgpu.align_noalloc(gix, rb, ln, w.params.d_max, params, out)
    assert e.value.code == snapgpu.SNAP_ETOOBIG
    torch.cuda.synchronize()
    assert all(bool((t == 7).all()) for t in (out.pos, out.strand, out.dist, out.second, out.call))
    # the next call that fits still works after the refusal
    small = reads.subset(np.arange(0, 3_000))
    ref, got = _both(torch, snapgpu, gix, small, w.params.d_max, params, "after refusal, 3000 reads")
    for name, a, b in zip(FIELDS, got, ref):
        assert np.array_equal(np.asarray(a, np.int64), np.asarray(b, np.int64)), name
    gix.close()
