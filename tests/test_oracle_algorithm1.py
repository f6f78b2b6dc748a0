"""Algorithm 1 of the oracle on toy genomes with hand-derived outcomes.

Background: a 20 kbase uniform random genome, where a random 20-mer occurs by
chance with probability ~4e-8, so the only seed hits are the planted ones.
Parameters: s = 20, n = 10, c = 2, d_max = 8, h_max = 300, bucket 32, so
seeds are tried at offsets 0, 20, 40, 60, 80, 10, 30, 50, 70, 5 of a 100 bp
read. Outputs are (pos, strand, dist, second, call) with call 0 = not found,
1 = single hit, 2 = multiple hits, and -1 for "none".
"""
import numpy as np
import pytest

COMP = {ord("A"): "T", ord("C"): "G", ord("G"): "C", ord("T"): "A", ord("N"): "N"}


def rc(s):
    return s.translate(COMP)[::-1]


def sub(c):
    return {"A": "C", "C": "G", "G": "T", "T": "A"}[c]


@pytest.fixture(scope="module")
def base_genome(synth_mod):
    return synth_mod.genome_uniform(20_000, 7).tobytes().decode()


@pytest.fixture(scope="module")
def P(oracle_mod):
    return oracle_mod.make_params(conf_c=2, d_max=8, max_hits=300)


def align(oracle_mod, genome, read, params):
    ix = oracle_mod.Index(genome.encode(), 20)
    out = ix.align_one(read, params)
    res = ix.align(read.encode(), np.array([0, len(read)]), np.array([len(read)]), params, 1)
    ix.close()
    return out, res.stats


def plant(g, src, dst, seq=None):
    seq = g[src:src + 100] if seq is None else seq
    return g[:dst] + seq + g[dst + len(seq):]


@pytest.mark.parametrize("strand", [0, 1])
def test_exact_unique_read(oracle_mod, base_genome, P, strand):
    """Seed 1 finds the origin, scored at distance 0; seed 2 brings t = 2 >= 0 + c,
    so the loop breaks after exactly c = 2 lookups and one edit-distance call."""
    read = base_genome[5000:5100]
    read = rc(read) if strand else read
    out, st = align(oracle_mod, base_genome, read, P)
    assert out == (5000, strand, 0, -1, 1)
    assert st["seeds_looked_up"] == 2 and st["ed_calls"] == 1


@pytest.mark.parametrize("strand", [0, 1])
def test_two_identical_copies_early_multiple(oracle_mod, base_genome, P, strand):
    """Copies at 5000 and 12000: seed 1 votes for both, the smaller p is scored (0);
    seed 2 scores 12000 with limit 0 + c - 1 = 1 and gets 0, so d_best = 0 < c and
    d_second = 0 < 0 + c: early return of multiple hits."""
    g = plant(base_genome, 5000, 12000)
    read = g[5000:5100]
    read = rc(read) if strand else read
    out, st = align(oracle_mod, g, read, P)
    assert out == (5000, strand, 0, 0, 2)
    assert st["seeds_looked_up"] == 2 and st["ed_calls"] == 2


@pytest.mark.parametrize("strand", [0, 1])
def test_copy_c_or_more_edits_away_is_single(oracle_mod, base_genome, P, strand):
    """The copy carries substitutions at read offsets 10, 50, 90 (inside seeds 1, 3, 5).
    Seed 1 hits only the origin (0); seed 2 hits the copy, scored with limit 1 and
    rejected (3 > 1); t = 2 >= 0 + c, break. Single hit, no second."""
    g0 = base_genome
    copy = list(g0[5000:5100])
    for j in (10, 50, 90):
        copy[j] = sub(copy[j])
    g = plant(g0, 0, 12000, "".join(copy))
    read = g[5000:5100]
    if strand:
        read = rc(read)
        # on the reverse strand the seeds cover read offsets mirrored; keep the
        # copy's substitutions inside seeds 1, 3, 5 of the reversed read
        copy = list(g0[5000:5100])
        for j in (9, 49, 89):
            copy[j] = sub(copy[j])
        g = plant(g0, 0, 12000, "".join(copy))
    out, st = align(oracle_mod, g, read, P)
    assert out == (5000, strand, 0, -1, 1)
    assert st["ed_calls"] == 2 and st["ed_over_limit"] == 1


@pytest.mark.parametrize("strand", [0, 1])
def test_copy_one_edit_away_is_multiple(oracle_mod, base_genome, P, strand):
    """The copy differs at read offset 50 only. Seed 1 votes for both; the origin
    is scored first (0); seed 2 scores the copy with limit 1 and gets 1, so
    d_best = 0 < c and d_second = 1 < 0 + c: multiple hits. With limit rule
    d_best - 1 instead of d_best + c - 1 the copy would be rejected (Single)."""
    copy = list(base_genome[5000:5100])
    copy[50] = sub(copy[50])
    g = plant(base_genome, 0, 12000, "".join(copy))
    read = g[5000:5100]
    read = rc(read) if strand else read
    out, _ = align(oracle_mod, g, read, P)
    assert out == (5000, strand, 0, 1, 2)


@pytest.mark.parametrize("strand", [0, 1])
def test_all_seeds_over_hmax_is_multiple(oracle_mod, base_genome, oracle_mod_params_small_hmax, strand):
    """A tandem array of an 8-base unit over 900 bases: every 20-mer of a read
    inside it occurs > 100 times (h_max = 100 here), so every looked-up seed is
    skipped and the final test reports multiple hits with no location."""
    unit = "ACGTTGCA"
    arr = (unit * 200)[:900]
    g = base_genome[:3000] + arr + base_genome[3900:]
    read = g[3300:3400]
    read = rc(read) if strand else read
    out, st = align(oracle_mod, g, read, oracle_mod_params_small_hmax)
    assert out == (-1, -1, -1, -1, 2)
    assert st["seeds_over_limit"] == st["seeds_looked_up"] == 10


@pytest.fixture(scope="module")
def oracle_mod_params_small_hmax(oracle_mod):
    return oracle_mod.make_params(conf_c=2, d_max=8, max_hits=100)


def test_random_read_not_found(oracle_mod, base_genome, synth_mod, P):
    """No seed hits anything: all 10 seeds are looked up, nothing is scored."""
    read = synth_mod.genome_uniform(100, 99999).tobytes().decode()
    out, st = align(oracle_mod, base_genome, read, P)
    assert out == (-1, -1, -1, -1, 0)
    assert st["seeds_looked_up"] == 10 and st["ed_calls"] == 0


@pytest.mark.parametrize("strand", [0, 1])
def test_too_many_errors(oracle_mod, base_genome, P, strand):
    """Seed 1 is clean, the rest of the read carries k substitutions. With k = 12 >
    K = d_max + c - 1 = 9 the single call returns the special value: not found,
    no location. With k = 9 the distance 9 is within the limit K but above
    d_max = 8: not found, but the tracked location is reported."""
    for k, expect in ((12, (-1, -1, -1, -1, 0)), (9, (5000, strand, 9, -1, 0))):
        r = list(base_genome[5000:5100])
        for i in range(k):
            j = 22 + 6 * i
            r[j] = sub(r[j])
        read = "".join(r)
        if strand:
            read = rc(read)
            # reverse strand: the clean seed must be the first 20 bases of the reversed read
            r = list(base_genome[5000:5100])
            for i in range(k):
                j = 2 + 6 * i
                r[j] = sub(r[j])
            read = rc("".join(r))
        out, _ = align(oracle_mod, base_genome, read, P)
        assert out == (expect[0], expect[1], expect[2], expect[3], expect[4]), k


def test_paper_deletion_example_same_bucket(oracle_mod, base_genome, P):
    """Section 3.2, omitted aspect 1: seed 1 matches at p, seed 2 at p + 21 because
    of a deletion between them, so seeds vote for p and p + 1. Read = genome
    [5000, 5101) without base 5020. p = 5000 scores 1; p + 1 = 5001 scores 2 (one
    read base unpaired at the start, one text base skipped). Both fall in bucket
    5000 // 32 = 156, which keeps only (1, 5000): single hit, no second."""
    g = base_genome
    read = g[5000:5020] + g[5021:5101]
    ix = oracle_mod.Index(g.encode(), 20)
    log = ix.score_log(read, P)
    out = ix.align_one(read, P)
    ix.close()
    assert [(p, s, d) for p, s, d, _ in log] == [(5000, 0, 1), (5001, 0, 2)]
    assert out == (5000, 0, 1, -1, 1)


def test_deletion_example_across_bucket_boundary(oracle_mod, base_genome, P):
    """Same example with p = 5023: p and p + 1 = 5024 straddle the fixed bucket
    boundary (5024 = 157 * 32), so the two results stay separate: d_second = 2 <
    d_best + c = 3 and the read is reported as multiple hits."""
    g = base_genome
    read = g[5023:5043] + g[5044:5124]
    out = align(oracle_mod, g, read, P)[0]
    assert out == (5023, 0, 1, 2, 2)


def test_baeza_yates_break_counts_lookups(oracle_mod, base_genome, P):
    """Section 3.2: after t disjoint seeds are tested, unfound locations are >= t
    away, so the search stops once t >= d_best + c. A read with one substitution
    in seed 5 (offset 90) scores 1 at seed 1 and stops after 3 lookups; with two
    substitutions there (offsets 85, 95) it stops after 4."""
    r = list(base_genome[5000:5100])
    r[90] = sub(r[90])
    out, st = align(oracle_mod, base_genome, "".join(r), P)
    assert out == (5000, 0, 1, -1, 1) and st["seeds_looked_up"] == 3
    r = list(base_genome[5000:5100])
    r[85] = sub(r[85])
    r[95] = sub(r[95])
    out, st = align(oracle_mod, base_genome, "".join(r), P)
    assert out == (5000, 0, 2, -1, 1) and st["seeds_looked_up"] == 4


def test_seed_with_n_is_skipped(oracle_mod, base_genome, P):
    """An N in seed 1 skips that slot (not looked up, t not counted); N never
    matches so the distance counts it; the read still aligns."""
    r = list(base_genome[5000:5100])
    r[3] = "N"
    out, st = align(oracle_mod, base_genome, "".join(r), P)
    assert out == (5000, 0, 1, -1, 1)
    assert st["seeds_with_n"] == 1 and st["seeds_looked_up"] == 3


def test_genome_edges(oracle_mod, base_genome, P):
    """Reads at the very start and end of the genome align; locations with p < 0
    or p + L > G are dropped."""
    G = len(base_genome)
    for a in (0, G - 100):
        out, _ = align(oracle_mod, base_genome, base_genome[a:a + 100], P)
        assert out == (a, 0, 0, -1, 1)
    # a read that would start before 0: its first 5 bases are not in the genome
    read = "ACGTA" + base_genome[0:95]
    out, _ = align(oracle_mod, base_genome, read, P)
    # seeds after offset 5 vote for p = -5 (dropped); nothing is scored
    assert out == (-1, -1, -1, -1, 0)


def test_short_reads(oracle_mod, base_genome, P):
    """A read shorter than s has no seeds: not found. Length exactly s: one seed."""
    assert align(oracle_mod, base_genome, base_genome[100:119], P)[0] == (-1, -1, -1, -1, 0)
    out = align(oracle_mod, base_genome, base_genome[100:120], P)[0]
    assert out[:3] == (100, 0, 0)
