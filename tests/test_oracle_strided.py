"""The strided index of Section 3.1's footnote (a window slid `stride` bases at a time:
a smaller index, more lookups) in the oracle, with hand-derived outcomes.

Reading (the footnote gives no seed schedule): only windows at positions q with
q % stride == 0 are indexed. Each seed slot of the schedule at read offset o looks up
the seeds at o, o + 1, ..., o + stride - 1 that fit the read; for any location p one of
them starts at an indexed position (p + o + j or, reversed, p + L - o - j - s is a
multiple of the stride). The slot is skipped as an N seed if any of its bases is an N;
its h_max count is the sum over its seeds; it votes once per location; and it counts in
t only if it is a round-0 slot whose stride seeds all fit the read. With stride 1 all of
this is the plain algorithm.

Toy genomes as in the other Algorithm 1 scenarios: a 20 kbase uniform random background
with planted copies of a random 100 bp read R; s = 20, n = 10, c = 2, d_max = 8,
h_max = 300, stride 2, seeds at offsets 0, 20, 40, 60, 80, 10, 30, 50, 70, 5. Of the
round-0 slots only 0, 20, 40, 60 are complete (the seed at 81 does not fit), so t <= 4.
"""
import random

import numpy as np
import pytest

COMP = str.maketrans("ACGTN", "TGCAN")


def rc(s):
    return s.translate(COMP)[::-1]


def sub(c):
    return {"A": "C", "C": "G", "G": "T", "T": "A"}[c]


def with_subs(seq, offsets):
    x = list(seq)
    for k in offsets:
        x[k] = sub(x[k])
    return "".join(x)


def plant(g, placements, strand=0):
    for pos, seq in placements:
        seq = rc(seq) if strand else seq
        g = g[:pos] + seq + g[pos + len(seq):]
    return g


@pytest.fixture(scope="module")
def bg(synth_mod):
    return synth_mod.genome_uniform(20_000, 7).tobytes().decode()


@pytest.fixture(scope="module")
def R():
    rng = np.random.default_rng(4242)
    return "".join("ACGT"[i] for i in rng.integers(0, 4, 100))


def run(oracle_mod, g, read, stride=2, **kw):
    p = oracle_mod.make_params(**{"conf_c": 2, "d_max": 8, "max_hits": 300, **kw})
    ix = oracle_mod.Index(g.encode(), 20, stride=stride)
    out = ix.align_one(read, p)
    log = ix.score_log(read, p)
    st = ix.align(read.encode(), np.array([0, len(read)]), np.array([len(read)]), p, 1).stats
    ix.close()
    return out, log, st


@pytest.mark.parametrize("stride,threads", [(2, 1), (2, 4), (3, 1), (3, 5), (4, 2)])
def test_strided_index_holds_the_windows_at_multiples_of_the_stride(oracle_mod, synth_mod, stride, threads):
    """Brute force: the sorted (window, position) pairs of the strided index are those of
    the full index at positions that are multiples of the stride, and lookups return the
    occurrences at such positions only (repeat genome with N runs)."""
    g = synth_mod.genome_repeats(40_000, 17, n_frac=0.02, n_run_lo=50, n_run_hi=500)
    full = oracle_mod.Index(g, 12)
    ix = oracle_mod.Index(g, 12, threads=threads, stride=stride)
    assert ix.stride == stride
    kf, qf = full.entries()
    ks, qs = ix.entries()
    keep = qf % stride == 0
    assert np.array_equal(ks, kf[keep]) and np.array_equal(qs, qf[keep])
    gs = g.tobytes().decode()
    rnd = random.Random(stride)
    for q in rnd.sample(range(len(gs) - 12), 40):
        w = gs[q:q + 12]
        want = None if "N" in w else [x for x in range(0, len(gs) - 11, stride) if gs[x:x + 12] == w]
        assert ix.occ(w) == want
    full.close()
    ix.close()


def test_stride_one_is_the_plain_index(oracle_mod, synth_mod):
    """stride 1 builds the plain index and aligns exactly as it does (mid recipe reads)."""
    from synth.workloads import MID
    w = MID.scaled(genome_len=300_000, n_reads=600)
    g = w.make_genome()
    reads = w.make_reads(g)
    a = oracle_mod.Index(g, 20)
    b = oracle_mod.Index(g, 20, stride=1)
    p = oracle_mod.params_from(w.params)
    ra, rb = a.align_reads(reads, p, threads=2), b.align_reads(reads, p, threads=2)
    for x, y in zip(ra.fields(), rb.fields()):
        assert np.array_equal(x, y)
    assert ra.stats == rb.stats and ra.stats["index_lookups"] == ra.stats["seeds_looked_up"]
    a.close()
    b.close()


@pytest.mark.parametrize("p0", [5000, 5001])
@pytest.mark.parametrize("strand", [0, 1])
def test_exact_read_at_either_parity(oracle_mod, bg, R, p0, strand):
    """An exact copy at an even or an odd position: in every slot exactly one of the two
    seeds starts at an indexed position of it (offset o for an even forward location,
    o + 1 for an odd one), so slot 0 finds it, it is scored at limit 9 -> 0, slot 20 brings
    t = 2 >= 0 + c: single after 2 slots, i.e. 4 index lookups (twice the plain index's)."""
    g = plant(bg, [(p0, R)], strand)
    out, log, st = run(oracle_mod, g, R)
    assert out == (p0, strand, 0, -1, 1)
    assert [(q, s, d, lim) for q, s, d, lim in log] == [(p0, strand, 0, 9)]
    assert st["seeds_looked_up"] == 2 and st["index_lookups"] == 4


def test_incomplete_round0_slot_does_not_count_in_t(oracle_mod, bg, R):
    """The last round-0 slot (offset 80) has one seed only, so it does not count in t.

    X (subs 15, 35, 55) at 5000 (even), D = 3, is found by the seeds at 60, 80 and 70. Y
    (subs 15, 25, 55, 75) at 12001 (odd), D = 4: for an odd location the slots at even
    offsets use their second seed ([o + 1, o + 21)), and only the slot at 30 (seed 31..50)
    misses every substitution; the slot at 80 has no second seed and cannot reach it.
    Slots 0, 20, 40: nothing, t = 3. Slot 60: X at limit 9 -> 3, t = 4 < 3 + c. Slot 80:
    t stays 4. Slot 10: nothing. Slot 30: Y at limit 3 + 1 = 4 -> 4. All 10 slots are
    looked up (19 seeds: the slot at 80 has one). Final: d_second = 4 < 5: multiple.
    Counting the slot at 80 would give t = 5 there and stop before Y: single."""
    g = plant(bg, [(5000, with_subs(R, (15, 35, 55))), (12001, with_subs(R, (15, 25, 55, 75)))])
    out, log, st = run(oracle_mod, g, R)
    assert [(q, s, d, lim) for q, s, d, lim in log] == [(5000, 0, 3, 9), (12001, 0, 4, 4)]
    assert out == (5000, 0, 3, 4, 2)
    assert st["seeds_looked_up"] == 10 and st["index_lookups"] == 19


def test_hmax_sums_a_slots_seeds(oracle_mod, bg, R):
    """A slot's entries for the h_max test are summed over its seeds.

    R exactly at 5000; R's first 20 bases planted 3 more times and bases 1..20 planted 3
    times, all at even positions. Slot 0's seeds have 4 (three plants and 5000) and 3
    indexed entries: 7 > h_max = 5, so the slot is skipped (either seed alone is within
    h_max). Slot 20: 5000 at limit 9 -> 0, t = 1; slot 40: t = 2: single after 3 slots,
    one of them over h_max, one distance computed."""
    g = plant(bg, [(5000, R)] + [(1000 + 400 * k, R[:20]) for k in range(3)] +
              [(3000 + 400 * k, R[1:21]) for k in range(3)])
    out, log, st = run(oracle_mod, g, R, max_hits=5)
    assert out == (5000, 0, 0, -1, 1)
    assert st["seeds_looked_up"] == 3 and st["seeds_over_limit"] == 1 and st["ed_calls"] == 1
    # with h_max 7 the slot is within the limit: it votes for 5000 and the 6 plants
    out, log, st = run(oracle_mod, g, R, max_hits=7)
    assert out == (5000, 0, 0, -1, 1) and st["seeds_over_limit"] == 0 and st["seeds_looked_up"] == 2


def test_n_in_a_slots_second_seed_skips_the_slot(oracle_mod, bg, R):
    """An N at read offset 20 lies outside the seed at 0 but inside the slot's second seed
    (1..20): slot 0 is skipped as an N seed, and so are the slots at 20, 10 and 5 whose
    seeds cover offset 20. R (with the N) at 5000: slot 40 scores 5000 at limit 9 -> 1 (the
    N matches nothing), t = 1; slot 60: t = 2; the slot at 80 does not count; t stays 2 <
    1 + c, so every slot is looked up: 6 lookups, 4 N slots. Single at distance 1."""
    read = R[:20] + "N" + R[21:]
    g = plant(bg, [(5000, R)])
    out, log, st = run(oracle_mod, g, read)
    assert out == (5000, 0, 1, -1, 1)
    assert st["seeds_with_n"] == 4 and st["seeds_looked_up"] == 6
