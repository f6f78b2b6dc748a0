"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: values the
paper prints (seed order, seed probabilities), brute-force search on tiny
inputs (edit distance over all alignments, occurrence scans), closed forms, and
toy genomes whose Algorithm 1 outcome is derived by hand in the docstring.
"""
import random

import numpy as np
import pytest

from conftest import read_golden

COMP = {ord("A"): "T", ord("C"): "G", ord("G"): "C", ord("T"): "A", ord("N"): "N"}


def rc(s: str) -> str:
    return s.translate(COMP)[::-1]


# ------------------------------------------------------------- seed order

def test_seed_order_matches_paper_examples(oracle_mod):
    """Section 3.1 (five non-overlapping seeds of a 100 bp read) and Section 3.2
    omitted aspect 3 (0, s, 2s, ... then shifted by s/2, then s/4, 3s/4)."""
    for row in read_golden("seed_order.txt"):
        L, n = int(row[0]), int(row[1])
        want = [int(v) for v in row[2:]]
        assert oracle_mod.seed_offsets(L, 20, n) == want


def test_seed_shift_order(oracle_mod):
    """All 20 shifts appear once, in the order of the golden list (first four from the paper)."""
    shifts = [int(v) for v in read_golden("seed_shifts.txt")[0]]
    # a read of length 39 holds exactly one seed per shift (offset = shift)
    assert oracle_mod.seed_offsets(39, 20, 32) == shifts
    assert sorted(shifts) == list(range(20))


def test_seed_order_edges(oracle_mod):
    assert oracle_mod.seed_offsets(19, 20, 10) == []          # read shorter than a seed
    assert oracle_mod.seed_offsets(20, 20, 10) == [0]
    assert oracle_mod.seed_offsets(40, 20, 3) == [0, 20, 10]
    # non-overlapping seeds come first: all multiples of s that fit
    for L in (60, 99, 100, 101, 250, 1000):
        offs = oracle_mod.seed_offsets(L, 20, 64)
        k = L // 20
        assert offs[:k] == [20 * i for i in range(k)]
        assert all(o + 20 <= L for o in offs)
        assert len(set(offs)) == len(offs)


def test_seeds_and_dmax_for_length(oracle_mod):
    p = oracle_mod.make_params(n_min=10, n_cap=32, bp_per_seed=100, d_max=8, d_max_pct=8)
    assert oracle_mod.seeds_for_length(p, 100) == 10
    assert oracle_mod.seeds_for_length(p, 250) == 10
    assert oracle_mod.seeds_for_length(p, 1001) == 11
    assert oracle_mod.seeds_for_length(p, 10000) == 32
    # ceil(0.08 L) in integers
    assert oracle_mod.dmax_for_length(p, 100) == 8
    assert oracle_mod.dmax_for_length(p, 101) == 9
    assert oracle_mod.dmax_for_length(p, 1000) == 80
    assert oracle_mod.dmax_for_length(p, 9999) == 800


# ---------------------------------------------------------- edit distance

def brute_alignment_distance(read: str, text: str) -> int:
    """Minimum cost over every alignment of the whole read against any prefix of
    the text (exhaustive search with branch-and-bound, no table): each step
    either pairs a read base with a text base (cost 0 if equal and not N, else 1),
    leaves a read base unpaired (1) or skips a text base (1)."""
    best = [len(read)]

    def rec(i, j, cost):
        if cost >= best[0]:
            return
        if i == len(read):
            best[0] = cost
            return
        if j < len(text):
            rec(i + 1, j + 1, cost + (0 if read[i] == text[j] and read[i] != "N" else 1))
            rec(i, j + 1, cost + 1)
        rec(i + 1, j, cost + 1)

    rec(0, 0, 0)
    return best[0]


def test_edit_distance_vs_exhaustive_alignments(oracle_mod):
    rnd = random.Random(1234)
    for trial in range(400):
        L = rnd.randint(0, 7)
        T = rnd.randint(0, 9)
        alpha = "ACGT" if trial % 4 else "ACGTN"
        read = "".join(rnd.choice(alpha) for _ in range(L))
        text = "".join(rnd.choice(alpha) for _ in range(T))
        D = brute_alignment_distance(read, text)
        for lim in range(-1, 9):
            got = oracle_mod.edit_distance(read, text, lim)
            assert got == (D if D <= lim else oracle_mod.INF), (read, text, lim, D, got)


def test_edit_distance_related_reads(oracle_mod):
    """Reads that differ from the text by a few edits (the common case)."""
    rnd = random.Random(99)
    for _ in range(150):
        text = "".join(rnd.choice("ACGT") for _ in range(9))
        r = list(text[: rnd.randint(4, 8)])
        for _ in range(rnd.randint(0, 2)):
            k = rnd.randrange(len(r))
            op = rnd.randrange(3)
            if op == 0:
                r[k] = rnd.choice("ACGT")
            elif op == 1:
                del r[k]
                if not r:
                    r = ["A"]
            else:
                r.insert(k, rnd.choice("ACGT"))
        read = "".join(r)
        D = brute_alignment_distance(read, text)
        assert oracle_mod.edit_distance(read, text, 10) == D


def test_edit_distance_closed_forms(oracle_mod):
    rnd = random.Random(5)
    g = "".join(rnd.choice("ACGT") for _ in range(400))
    read = g[:100]
    ED = oracle_mod.edit_distance
    assert ED(read, g[:100], 0) == 0
    assert ED(read, g, 0) == 0                       # end is free: longer text costs nothing
    # k spaced substitutions cost k
    for k in range(1, 8):
        r = list(read)
        for i in range(k):
            j = 5 + 12 * i
            r[j] = {"A": "C", "C": "G", "G": "T", "T": "A"}[r[j]]
        assert ED("".join(r), g, 20) == k
    # an interior deletion or insertion of length l costs l
    for l in range(1, 6):
        dele = g[:40] + g[40 + l:100 + l]
        assert ED(dele, g, 20) == l
        ins = g[:40] + "".join(rnd.choice("ACGT") for _ in range(l)) + g[40:100 - l]
        assert ED(ins, g, 20) <= l
    # the distance never exceeds the substitutions along the main diagonal
    r = "".join(rnd.choice("ACGT") for _ in range(60))
    ham = sum(a != b for a, b in zip(r, g[:60]))
    assert ED(r, g, 200) <= ham
    # N matches nothing, not even N
    assert ED("NNNN", "NNNN", 10) == 4
    assert ED("ACNT", "ACNT", 10) == 1
    assert ED("ACGT", "ACNT", 10) == 1
    # threshold semantics: distance if at most the limit, the special value otherwise
    r = g[:50] + "T" + g[51:100]
    d = ED(r, g, 100)
    assert d in (0, 1)
    for lim in range(0, 5):
        assert ED(r, g, lim) == (d if d <= lim else oracle_mod.INF)
    assert ED(read, g, -1) == oracle_mod.INF


# ------------------------------------------------------------------ index

def test_index_vs_occurrence_scan(oracle_mod, synth_mod):
    g = synth_mod.genome_repeats(60_000, 11, n_frac=0.02, n_run_lo=50, n_run_hi=500)
    gs = g.tobytes().decode()
    for s in (8, 20):
        ix = oracle_mod.Index(g, s)
        free = sum(1 for q in range(len(gs) - s + 1) if "N" not in gs[q:q + s])
        assert ix.windows == free
        rnd = random.Random(s)
        queries = [gs[q:q + s] for q in rnd.sample(range(len(gs) - s), 60)]
        queries += ["".join(rnd.choice("ACGT") for _ in range(s)) for _ in range(20)]
        for qs in queries:
            want = None if "N" in qs else [q for q in range(len(gs) - s + 1) if gs[q:q + s] == qs]
            assert ix.occ(qs) == want
        ix.close()


@pytest.mark.parametrize("s,threads", [(8, 3), (20, 2), (20, 8), (3, 5), (32, 4)])
def test_parallel_index_build_equals_plain(oracle_mod, synth_mod, s, threads):
    """The threaded bucket-sort build gives the same sorted (window, position) array as
    the plain single-thread build, on a repeat genome with N runs (and answers lookups
    the same, against a scan of the genome)."""
    g = synth_mod.genome_repeats(40_000, 13, n_frac=0.02, n_run_lo=50, n_run_hi=500)
    a = oracle_mod.Index(g, s)
    b = oracle_mod.Index(g, s, threads=threads)
    ka, qa = a.entries()
    kb, qb = b.entries()
    assert len(ka) == a.windows > 0
    assert np.array_equal(ka, kb) and np.array_equal(qa, qb)
    gs = g.tobytes().decode()
    rnd = random.Random(s)
    for q in rnd.sample(range(len(gs) - s), 30):
        want = None if "N" in gs[q:q + s] else [x for x in range(len(gs) - s + 1) if gs[x:x + s] == gs[q:q + s]]
        assert b.occ(gs[q:q + s]) == want
    a.close()
    b.close()


def test_index_random_hit_rate(oracle_mod, synth_mod):
    """Section 3.1: a random s-mer hits about G/4^s places by chance (4^6 for
    s = 10 and 4^-4 for s = 20 on a 4^16 genome). Checked at s = 7 where the
    mean, (G - s + 1)/4^7, is measurable."""
    G, s = 200_000, 7
    ix = oracle_mod.Index(synth_mod.genome_uniform(G, 3), s)
    rnd = random.Random(7)
    hits = [len(ix.occ("".join(rnd.choice("ACGT") for _ in range(s)))) for _ in range(3000)]
    expect = (G - s + 1) / 4 ** s
    assert abs(np.mean(hits) - expect) < 0.1 * expect


# ------------------------------------------------------- simulator checks

def test_simulator_seed_probabilities(synth_mod):
    """Section 3.1: at 2% substitutions a 20 bp seed is clean with probability
    0.98^20 = 0.67 and all five disjoint seeds of a 100 bp read carry an error
    with probability (1 - 0.98^20)^5 ~ 0.004 (printed as 0.33^5)."""
    gold = {r[0]: (float(r[1]), float(r[2])) for r in read_golden("seed_probabilities.txt")}
    g = synth_mod.genome_uniform(2_000_000, 21)
    model = synth_mod.ReadModel(len_mode=0, len_a=100, p_sub=0.02, p_indel=0.0)
    rd = synth_mod.simulate_reads(g, 200_000, 22, model)
    gs = g.tobytes()
    clean = 0
    all_dirty = 0
    for i in range(rd.n):
        r = rd.bases[rd.offsets[i]:rd.offsets[i + 1]].tobytes()
        src = gs[rd.truth_pos[i]:rd.truth_pos[i] + 100]
        if rd.truth_strand[i]:
            src = rc(src.decode()).encode()
        seeds = [r[o:o + 20] == src[o:o + 20] for o in range(0, 100, 20)]
        clean += sum(seeds)
        all_dirty += not any(seeds)
    p_clean = clean / (5 * rd.n)
    p_dirty = all_dirty / rd.n
    assert abs(p_clean - 0.98 ** 20) < 0.005
    assert abs(p_clean - gold["p_seed_clean"][0]) <= gold["p_seed_clean"][1] + 0.005
    assert abs(p_dirty - (1 - 0.98 ** 20) ** 5) < 0.0012
    assert abs(p_dirty - gold["p_all_five_dirty"][0]) <= gold["p_all_five_dirty"][1] + 0.0012


def test_simulator_error_rates(synth_mod):
    g = synth_mod.genome_uniform(1_000_000, 0)
    model = synth_mod.ReadModel(len_mode=0, len_a=100, p_sub=0.01, p_indel=0.001, indel_max=5)
    rd = synth_mod.simulate_reads(g, 20_000, 5, model)
    assert np.all(rd.lengths == 100)
    assert 0.4 < rd.truth_strand.mean() < 0.6
    # expected events per read ~ 100 * (0.01 + 0.001 * mean indel length)
    assert 0.9 < rd.truth_edits.mean() < 1.4
    # deterministic by seed and per-read streams
    rd2 = synth_mod.simulate_reads(g, 100, 5, model)
    assert np.array_equal(rd2.bases, rd.bases[:rd2.bases.shape[0]])


def test_family_genome_generator(synth_mod):
    """The high-copy family generator: `copies` copies of one element at distinct,
    non-overlapping places, each differing from the consensus at about `div` of its
    bases (the consensus is the per-column majority over the copies)."""
    G, copies, L, div = 400_000, 600, 300, 0.015
    g = synth_mod.genome_family(G, 17, copies, elem_len=L, div=div)
    assert g.shape == (G,) and set(np.unique(g).tolist()) <= set(b"ACGT")
    # the copies sit in slots of elem_len: find them as the slots closest to the consensus
    slots = g[: (G // L) * L].reshape(-1, L)
    cols = np.stack([(slots == c).sum(0) for c in b"ACGT"])
    consensus = np.frombuffer(b"ACGT", np.uint8)[cols.argmax(0)]
    mism = (slots != consensus).mean(1)
    family = mism < 0.2
    assert family.sum() == copies
    assert abs(mism[family].mean() - div) < 0.004
    assert mism[~family].min() > 0.6    # the rest is uniform sequence
    with pytest.raises(ValueError):
        synth_mod.genome_family(1000, 1, 10, elem_len=300)
