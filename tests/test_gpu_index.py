"""The index built by device kernels (snap_index_build_device) against the host build
(snap_index_build): the same packed genome, N mask and positions array, the same set of
table entries (an entry's slot depends on the order of the concurrent insertions, so
entries are compared sorted by key), and identical alignments through either index,
which are also the oracle's. Integer work: tolerance zero."""
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


def _entries(tab):
    t = tab[tab[:, 0] != np.uint64(0xFFFFFFFFFFFFFFFF)]
    return t[np.argsort(t[:, 0], kind="stable")]


def _same_index(snapgpu, g, s, label):
    say(f"[{label}] G={len(g)} s={s}")
    h = snapgpu.Index(g, s)
    d = snapgpu.Index(g, s, on_device=True)
    try:
        sh, sd = h.sizes(), d.sizes()
        assert sh == sd, (sh, sd)
        for w in ("gcode", "gmask", "positions"):
            assert np.array_equal(h.download(w), d.download(w)), w
        eh, ed = _entries(h.download("table")), _entries(d.download("table"))
        assert eh.shape[0] == sh["distinct_keys"]
        assert np.array_equal(eh, ed)
    finally:
        h.close()
        d.close()


def _mixed_case(synth_mod, G, seed):
    """Uniform genome with lowercase bases and IUPAC codes (read as N) mixed in."""
    g = synth_mod.genome_uniform(G, seed).copy()
    rng = np.random.default_rng(seed)
    low = rng.random(G) < 0.1
    g[low] = g[low] + 32
    g[rng.random(G) < 0.002] = ord("R")
    return g


@pytest.mark.parametrize("kind,G,s", [
    ("uniform", 200_000, 20),
    ("repeats", 1_500_000, 20),
    ("repeats", 300_000, 11),
    ("repeats", 300_000, 31),
    ("repeats_n", 1_000_000, 20),
    ("family", 600_000, 8),
    ("mixed_case", 300_000, 16),
])
def test_device_index_equals_host(snapgpu, synth_mod, kind, G, s):
    if kind == "uniform":
        g = synth_mod.genome_uniform(G, 3)
    elif kind == "repeats":
        g = synth_mod.genome_repeats(G, 4)
    elif kind == "repeats_n":
        g = synth_mod.genome_repeats(G, 5, n_frac=0.02, n_run_lo=30, n_run_hi=3000)
    elif kind == "family":
        g = synth_mod.genome_family(G, 6, 1500)   # s = 8: many palindromic windows
    else:
        g = _mixed_case(synth_mod, G, 7)
    _same_index(snapgpu, g, s, f"{kind} s={s}")


def test_device_index_edge_genomes(snapgpu):
    # one window; a few windows; an N-only genome (no entries); a homopolymer whose one
    # key has more windows than the counts hold (saturated in both builds)
    for g, s in ((b"ACGTACGTACGTACGTACGT", 20), (b"ACGTTGCAACGTTGCAACGTAAC", 20), (b"N" * 500, 20),
                 (b"A" * 40_000 + b"C" * 30, 20), (b"ACGT" * 5000, 2), (b"GATTACA" * 3, 1)):
        _same_index(snapgpu, np.frombuffer(g, dtype=np.uint8), s, f"edge G={len(g)} s={s}")


def test_device_index_rejects(snapgpu):
    g = b"ACGT" * 100
    for s in (0, 32, 33):
        with pytest.raises(snapgpu.SnapError):
            snapgpu.Index(g, s, on_device=True)
    with pytest.raises(snapgpu.SnapError):
        snapgpu.Index(b"ACGT", 20, on_device=True)


def test_alignments_through_device_index(snapgpu, oracle_mod, synth_mod):
    from synth.workloads import HUMAN
    w = HUMAN.scaled(genome_len=3_000_000, n_reads=6_000)
    g = w.make_genome()
    reads = w.make_reads(g)
    gp = snapgpu.params_from(w.params)
    d = snapgpu.Index(g, w.params.seed_len, on_device=True)
    h = snapgpu.Index(g, w.params.seed_len)
    try:
        out_d = gpu_align(snapgpu, d, reads, w.params.d_max, gp)
        out_h = gpu_align(snapgpu, h, reads, w.params.d_max, gp)
    finally:
        d.close()
        h.close()
    for name, a, b in zip(("pos", "strand", "dist", "second", "call"), out_d, out_h):
        assert np.array_equal(a, b), name
    oix = oracle_mod.Index(g, w.params.seed_len)
    nbad, rep = compare(out_d, oracle_align(oracle_mod, oix, reads, w.params), reads, "device index")
    oix.close()
    assert nbad == 0, rep


def _table_digest(tab):
    """Order-free digest of a table's entries (their slots do not matter)."""
    acc = np.uint64(0)
    step = 1 << 24
    with np.errstate(over="ignore"):
        for i in range(0, tab.shape[0], step):
            t = tab[i:i + step]
            t = t[t[:, 0] != np.uint64(0xFFFFFFFFFFFFFFFF)]
            acc += np.bitwise_xor(t[:, 0] * np.uint64(0x9E3779B97F4A7C15), t[:, 1]).sum(dtype=np.uint64)
    return int(acc)


def test_device_index_over_2e30_records(snapgpu, oracle_mod, synth_mod):
    """More records than 2^30 (1.1 Gbase uniform genome, one record per window): every
    window position appears in the positions array (once, twice for a palindrome), and
    reads aligned through this index equal the oracle's on all five outputs (the oracle's
    index is built from the same genome; the host build is not needed)."""
    from synth.workloads import TINY
    g = synth_mod.genome_uniform(1_100_000_000, 9)
    say(f"[over 2^30 records] G={len(g)}")
    d = snapgpu.Index(g, 20, on_device=True)
    try:
        sz = d.sizes()
        nwin = len(g) - 20 + 1
        assert sz["position_entries"] > (1 << 30) and sz["windows"] == nwin, sz
        pos = d.download("positions")
        pos.sort()
        first = np.ones(pos.shape[0], dtype=bool)
        first[1:] = pos[1:] != pos[:-1]
        uniq = pos[first]
        del pos
        assert uniq.shape[0] == nwin and int(uniq[0]) == 0 and int(uniq[-1]) == nwin - 1
        assert sz["position_entries"] - nwin < 10_000   # palindromic 20-mers: about G / 4^10
        del uniq, first
        w = TINY.scaled(n_reads=4_000)
        reads = w.make_reads(g)
        out = gpu_align(snapgpu, d, reads, w.params.d_max, snapgpu.params_from(w.params))
    finally:
        d.close()
    oix = oracle_mod.Index(g, 20, threads=16)
    nbad, rep = compare(out, oracle_align(oracle_mod, oix, reads, w.params), reads, "over 2^30 records")
    oix.close()
    assert nbad == 0, rep


def test_alignments_beyond_2e31(snapgpu, oracle_mod, synth_mod):
    """Locations at genome positions past 2^31: the genome is an N run of 2^31 + 4,321
    bases followed by 3 Mbase of the repeat recipe (segmental duplicates, tandem arrays);
    reads from the tail (both strands, substitutions and indels, 100 and 250 bp) align
    bit-exact with the oracle on all five outputs."""
    from synth.workloads import HUMAN
    pad = (1 << 31) + 4_321
    w = HUMAN.scaled(genome_len=3_000_000, n_reads=8_000)
    tail = w.make_genome()
    reads = w.make_reads(tail)
    g = np.empty(pad + tail.shape[0], dtype=np.uint8)
    g[:pad] = ord("N")
    g[pad:] = tail
    del tail
    say(f"[beyond 2^31] G={len(g)} reads={reads.n}")
    d = snapgpu.Index(g, 20, on_device=True)
    try:
        out = gpu_align(snapgpu, d, reads, w.params.d_max, snapgpu.params_from(w.params))
    finally:
        d.close()
    hit = out[0] >= 0
    assert hit.mean() > 0.9 and int(out[0][hit].min()) >= pad
    oix = oracle_mod.Index(g, 20, threads=16)
    nbad, rep = compare(out, oracle_align(oracle_mod, oix, reads, w.params), reads, "beyond 2^31")
    oix.close()
    assert nbad == 0, rep
