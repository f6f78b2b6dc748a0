"""Algorithm 1 of the oracle at the boundaries of its tests, with hand-derived outcomes.

Each scenario plants copies of one random 100 bp read R (with substitutions, or an
insertion, at chosen read offsets) into a 20 kbase uniform random background, where a
random 20-mer occurs by chance with probability ~4e-8, so the only seed hits are the
planted ones. A copy with substitutions at offsets D is hit by the seed at offset o iff
no offset of D lies in [o, o + 20), and its distance to R is |D|.

Parameters unless stated: s = 20, n = 10, c = 2, d_max = 8, h_max = 300, bucket 32, so
the seeds of a 100 bp read are tried at offsets 0, 20, 40, 60, 80, 10, 30, 50, 70, 5 and
the round-0 (non-overlapping) seeds are the first five. The limit rule of Algorithm 1:
d_max + c - 1 = 9 while d_best > d_max; d_best + c - 1 if d_second >= d_best + c; else
d_best - 1. Outputs are (pos, strand, dist, second, call), call 0 = not found,
1 = single, 2 = multiple, -1 = none; the score log lists (p, strand, D or INF, limit).

Strand 1 versions plant the reverse complement of every copy and align the same read:
the read's seed at offset o then hits the copy in the reverse orientation at the same
location p (p = q - (L - o - s)), so each derivation carries over with strand 1.

Every scenario pins a point where a plausible slip in the oracle (a boundary written as
< instead of <=, a tie broken the other way, a counter that counts too much, an early
return in the wrong phase, a text window one base short) changes the outputs.
"""
import numpy as np
import pytest

INF = 0x3FFFFFFF
L = 100
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


@pytest.fixture(scope="module")
def bg(synth_mod):
    return synth_mod.genome_uniform(20_000, 7).tobytes().decode()


@pytest.fixture(scope="module")
def R():
    rng = np.random.default_rng(4242)
    return "".join("ACGT"[i] for i in rng.integers(0, 4, L))


def plant(g, placements, strand=0):
    """Write each (pos, seq) into the genome, reverse-complemented for strand 1."""
    for pos, seq in placements:
        seq = rc(seq) if strand else seq
        g = g[:pos] + seq + g[pos + len(seq):]
    return g


def run(oracle_mod, g, read, **kw):
    p = oracle_mod.make_params(**{"conf_c": 2, "d_max": 8, "max_hits": 300, **kw})
    ix = oracle_mod.Index(g.encode(), 20)
    out = ix.align_one(read, p)
    log = ix.score_log(read, p)
    st = ix.align(read.encode(), np.array([0, len(read)]), np.array([len(read)]), p, 1).stats
    ix.close()
    return out, [(q, s, d, lim) for q, s, d, lim in log], st


@pytest.mark.parametrize("strand", [0, 1])
def test_third_limit_rejects_a_location_at_d_best(oracle_mod, bg, R, strand):
    """The limit d_best - 1 (third case of the rule) is the only thing that rejects a copy.

    X1 (subs 25, 45) at 5000, D = 2; X2 (subs 65, 85, 95) at 12000, D = 3; X3 (subs 35, 75)
    at 16000, D = 2. Seed 0 votes for all three: X1 (smallest p) is scored with limit 9 -> 2.
    Seed 20 hits X2 only (2 votes): limit 2 + 2 - 1 = 3 (d_second = INF >= 4) -> 3, so
    d_second = 3. Seed 40 hits X2, X3: X3 (2 votes) is the only unscored location; now
    d_second = 3 < d_best + c = 4, so the limit is d_best - 1 = 1 and X3 (D = 2) is
    rejected. Seed 60 brings t = 4 >= 2 + 2: nothing is left to score; stop after 4
    lookups. Final: d_best = 2 <= 8, d_second = 3 < 4: multiple, second 3. A limit of d_best
    or d_best + c - 1 here would accept X3 and report second = 2."""
    g = plant(bg, [(5000, with_subs(R, (25, 45))), (12000, with_subs(R, (65, 85, 95))),
                   (16000, with_subs(R, (35, 75)))], strand)
    out, log, st = run(oracle_mod, g, R)
    assert log == [(5000, strand, 2, 9), (12000, strand, 3, 3), (16000, strand, INF, 1)]
    assert out == (5000, strand, 2, 3, 2)
    assert st["seeds_looked_up"] == 4 and st["ed_calls"] == 3
    # diagonal extensions at each call's own limit, (min(D, limit) + 1)^2: 9 + 16 + 4
    assert st["lv_extensions"] == 29
    # the selection scans the three locations after each of the four seeds, and once more
    # when the remaining phase finds nothing left: 5 x 3
    assert st["select_visits"] == 15


@pytest.mark.parametrize("strand", [0, 1])
def test_early_return_needs_d_best_below_c(oracle_mod, bg, R, strand):
    """No early return while d_best == c.

    X1 (subs 25, 45) at 5000, D = 2; X2 (subs 65, 85, 95) at 12000, D = 3; X3 (sub 35) at
    16000, D = 1. Seed 0: X1 scored (limit 9) -> 2. Seed 20 hits X2: limit 3 -> 3; now
    d_best = 2 = c and d_second = 3 < 2 + c: the early test d_best < c fails, so the loop
    goes on. Seed 40: X3 (hit by seeds 0 and 40) with limit d_best - 1 = 1 -> 1; now
    d_best = 1 < c and d_second = 2 < 1 + c: early return of multiple with X3 best.
    Returning already at d_best == c would report (5000, 2, 3)."""
    g = plant(bg, [(5000, with_subs(R, (25, 45))), (12000, with_subs(R, (65, 85, 95))),
                   (16000, with_subs(R, (35,)))], strand)
    out, log, st = run(oracle_mod, g, R)
    assert log == [(5000, strand, 2, 9), (12000, strand, 3, 3), (16000, strand, 1, 1)]
    assert out == (16000, strand, 1, 2, 2)
    assert st["seeds_looked_up"] == 3


@pytest.mark.parametrize("strand", [0, 1])
def test_second_exactly_c_away_is_single(oracle_mod, bg, R, strand):
    """d_second == d_best + c gives a single hit; the selection tie goes to the smaller p.

    X2 (subs 65, 85) at 5000, D = 2; X1 = R exactly at 12000. Seed 0 votes for both (one
    vote each): the tie goes to the smaller p, so X2 is scored first, with limit 9 -> 2.
    Seed 20: X1 (2 votes) with limit 2 + 1 = 3 -> 0, so d_best = 0 and d_second = 2. The
    early test fails (d_second = 2 is not < 0 + c); t = 2 >= 0 + c ends the loop. Final:
    d_second = 2 >= d_best + c = 2: single, with second 2. With the test d_second >
    d_best + c the read would be multiple; with the tie to the larger p, X1 would be scored
    first and X2 rejected at limit 1 (second -1)."""
    g = plant(bg, [(5000, with_subs(R, (65, 85))), (12000, R)], strand)
    out, log, st = run(oracle_mod, g, R)
    assert log == [(5000, strand, 2, 9), (12000, strand, 0, 3)]
    assert out == (12000, strand, 0, 2, 1)
    assert st["seeds_looked_up"] == 2


def test_hmax_counts_both_orientations(oracle_mod, bg, R):
    """h_max is compared with the entries of the seed plus those of its reverse complement.

    R is planted three times forward (3000, 6000, 9000) and three times reverse
    complemented (12000, 15000, 18000), so every seed has 3 + 3 = 6 entries. With h_max = 4
    every seed is over the limit: all 10 are looked up and skipped, and the final rule
    reports multiple with no location. With h_max = 6 none is: seed 0 votes for all six
    locations, (3000, +) is scored first (limit 9 -> 0), seed 20 scores (6000, +) at limit
    1 -> 0, and d_best = d_second = 0 < c returns multiple early. Counting forward entries
    only (3 <= 4) would give that second outcome at h_max = 4 too."""
    g = plant(bg, [(3000, R), (6000, R), (9000, R)])
    g = plant(g, [(12000, R), (15000, R), (18000, R)], strand=1)
    out, log, st = run(oracle_mod, g, R, max_hits=4)
    assert out == (-1, -1, -1, -1, 2) and log == []
    assert st["seeds_looked_up"] == 10 and st["seeds_over_limit"] == 10
    out, log, st = run(oracle_mod, g, R, max_hits=6)
    assert log == [(3000, 0, 0, 9), (6000, 0, 0, 1)]
    assert out == (3000, 0, 0, 0, 2)
    assert st["seeds_over_limit"] == 0


@pytest.mark.parametrize("strand", [0, 1])
def test_t_counts_round0_seeds_only(oracle_mod, bg, R, strand):
    """t counts the non-overlapping (round-0) seeds only, so with d_best = 4 the loop
    never breaks and a location hit by a later seed is still scored.

    X1 (subs 15, 35, 55, 75) at 5000, D = 4, is hit only by the seed at 80 (the 5th).
    Y (subs 15, 35, 55, 65, 95) at 12000, D = 5, only by the seed at 70 (the 9th). After
    seed 80: X1 scored (limit 9) -> 4, t = 5 < 4 + c. Seeds 10, 30, 50 hit nothing. Seed
    70: Y with limit 4 + 1 = 5 -> 5. All 10 seeds are looked up. Final: d_second = 5 <
    6: multiple. Counting every looked-up seed in t would break at the 6th seed (t = 6)
    before Y is found, and report single."""
    g = plant(bg, [(5000, with_subs(R, (15, 35, 55, 75))), (12000, with_subs(R, (15, 35, 55, 65, 95)))], strand)
    out, log, st = run(oracle_mod, g, R)
    assert log == [(5000, strand, 4, 9), (12000, strand, 5, 5)]
    assert out == (5000, strand, 4, 5, 2)
    assert st["seeds_looked_up"] == 10


@pytest.mark.parametrize("strand", [0, 1])
def test_t_skips_round0_seeds_over_hmax(oracle_mod, bg, R, strand):
    """A round-0 seed skipped for having more than h_max entries does not count in t.

    h_max = 5; R's first 20 bases are planted 10 more times on their own, so seed 0 has
    11 entries and is skipped. X1 (subs 5, 15) at 5000, D = 2, is hit by seeds 20..80; Z
    (subs 30, 50, 70) at 12000, D = 3, among the round-0 seeds only by 80. Seed 20: X1 ->
    2 (limit 9), t = 1; seeds 40, 60: t = 3; seed 80: Z with limit 3 -> 3, t = 4 >=
    2 + c: stop after 5 lookups. Final: multiple, second 3. Counting the skipped seed would
    stop after seed 60 (t = 4) without Z: single."""
    head = R[:20]
    g = plant(bg, [(1000 + 300 * k, head) for k in range(10)], strand)
    g = plant(g, [(5000, with_subs(R, (5, 15))), (12000, with_subs(R, (30, 50, 70)))], strand)
    out, log, st = run(oracle_mod, g, R, max_hits=5)
    assert log == [(5000, strand, 2, 9), (12000, strand, 3, 3)]
    assert out == (5000, strand, 2, 3, 2)
    assert st["seeds_looked_up"] == 5 and st["seeds_over_limit"] == 1


@pytest.mark.parametrize("strand", [0, 1])
def test_no_early_return_while_scoring_remaining(oracle_mod, bg, R, strand):
    """"Score remaining locations" scores every one, even after the multiple-hits test
    would hold, and recomputes the limit before each call.

    X (sub 90) at 1000, D = 1; E1 (subs 45, 65, 85) at 1500, D = 3; E2 (subs 65, 75, 95)
    at 1700, D = 3; B (subs 85, 95) at 2000, D = 2; C = R at 3000, D = 0. Seed 0 votes
    for all: X scored (limit 9) -> 1. Seed 20: E1 (2 votes, smallest p) at limit 2 ->
    INF. Seed 40 (misses E1): E2 at limit 2 -> INF; t = 3 >= 1 + c: score the rest in
    selection order: B (3 votes, p 2000) at limit 2 -> 2, so d_best = 1 < c and d_second
    = 2 < 1 + c, yet scoring goes on: C at limit d_best - 1 = 0 -> 0. Final: d_best 0 (C),
    d_second 1: multiple at 3000. An early return inside this phase would report X."""
    g = plant(bg, [(1000, with_subs(R, (90,))), (1500, with_subs(R, (45, 65, 85))),
                   (1700, with_subs(R, (65, 75, 95))), (2000, with_subs(R, (85, 95))), (3000, R)], strand)
    out, log, st = run(oracle_mod, g, R)
    assert log == [(1000, strand, 1, 9), (1500, strand, INF, 2), (1700, strand, INF, 2),
                   (2000, strand, 2, 2), (3000, strand, 0, 0)]
    assert out == (3000, strand, 0, 1, 2)
    assert st["seeds_looked_up"] == 3


def test_bucket_keeps_the_lower_p_on_equal_distance(oracle_mod, bg):
    """A bucket keeps its lowest (D, p), not the first result scored in it.

    A tandem array of a random 10-base unit V from a0 = 5000 to 5108; the base at 5005 is
    changed and the bases around the array are chosen to differ from the unit's
    continuation. The read is V repeated 10 times. Location 5010 matches except its last
    base (5109 lies outside the array): D = 1; location 5000 matches except offset 5: D =
    1; both lie in bucket 5000 // 32 = 5010 // 32 = 156. The phase-0 seed V V occurs at
    5010, ..., 5080 (not at 5000, which holds the change). Seed 0 votes for 5010..5080 and
    scores 5010 (limit 9) -> 1. Seed 20 adds votes to 4990..5060: 5020 (2 votes) at limit 2
    -> INF. Seed 40: 5030 (3 votes) at limit 2 -> INF; t = 3 >= 1 + c: the rest in
    selection order: 5040 -> INF, then the 2-vote locations 4990 -> INF and 5000 -> 1 at
    limit 2, ... The bucket then holds (1, 5000): single at 5000. Keeping the first result
    of a bucket would report 5010."""
    rng = np.random.default_rng(77)
    while True:
        V = "".join("ACGT"[i] for i in rng.integers(0, 4, 10))
        if len({V[k:] + V[:k] for k in range(10)}) == 10:   # no shorter period
            break
    a0 = 5000
    cont = lambda j: V[(j - a0) % 10]   # the array's unit continued over any position
    g = list(bg)
    for j in range(a0 - 40, a0 + 140):
        g[j] = cont(j) if a0 <= j < a0 + 109 else sub(cont(j))
    g[a0 + 5] = sub(cont(a0 + 5))
    g = "".join(g)
    read = V * 10
    out, log, st = run(oracle_mod, g, read)
    assert log[:7] == [(5010, 0, 1, 9), (5020, 0, INF, 2), (5030, 0, INF, 2), (5040, 0, INF, 2),
                       (4990, 0, INF, 2), (5000, 0, 1, 2), (5050, 0, INF, 2)]
    assert all(d == INF for _, _, d, _ in log[7:])
    assert out == (5000, 0, 1, -1, 1)


def test_best_location_tie_prefers_the_forward_strand(oracle_mod, bg):
    """Equal distance and equal p on both strands: the forward strand is reported.

    R = X + rc(X) (X a random 50-mer) equals its own reverse complement, planted at 5000:
    both (+, 5000) and (-, 5000) are at distance 0 and every seed votes for both. The
    selection tie goes to + (scored with limit 9 -> 0), then - at limit 1 -> 0: two
    buckets at distance 0, early return of multiple; the best of the equal (D, p) pair is
    the forward one."""
    rng = np.random.default_rng(99)
    X = "".join("ACGT"[i] for i in rng.integers(0, 4, 50))
    read = X + rc(X)
    assert rc(read) == read
    g = plant(bg, [(5000, read)])
    out, log, st = run(oracle_mod, g, read)
    assert log == [(5000, 0, 0, 9), (5000, 1, 0, 1)]
    assert out == (5000, 0, 0, 0, 2)


@pytest.mark.parametrize("strand", [0, 1])
def test_text_window_holds_read_length_plus_limit(oracle_mod, bg, R, strand):
    """The text compared with a read is L + limit bases long: a location the read
    reaches only with `limit` deletions needs all of them.

    X1 (sub 50) at 5000, D = 1. X2 is R with two extra bases inserted (after read offset
    90 for strand 0, after offset 10 for strand 1, so that the seeds on the read's own side
    of the insertion vote for X2's start): the read reaches it with 2 deletions, using 102
    text bases. Seed 0: X1 -> 1 (limit 9). Seed 20: X2 at limit 1 + c - 1 = 2 with a
    102-base text -> 2; d_best = 1 < c and d_second = 2 < 1 + c: multiple. With a text one
    base shorter (L + limit - 1) X2 would cost 3 -> INF, and the read would be single."""
    k = 90 if strand == 0 else 10
    ins = sub(R[k]) + sub(sub(R[k]))
    x2 = R[:k] + ins + R[k:]
    g = plant(bg, [(5000, with_subs(R, (50,))), (12000, x2)], strand)
    out, log, st = run(oracle_mod, g, R)
    assert log == [(5000, strand, 1, 9), (12000, strand, 2, 2)]
    assert out == (5000, strand, 1, 2, 2)


def test_locations_past_either_genome_end_are_dropped(oracle_mod, bg):
    """A location whose read span would leave the genome (p < 0 or p + L > G) gets no vote,
    on either strand. Each read below is 95 genome bases plus 5 bases outside: its seeds
    hit only at a location with p = -5 or p + L = G + 5, so nothing is scored and the read
    is not found (with the edges kept, each would be scored and found at distance 5)."""
    G = len(bg)
    extra = "ACGTA"
    reads = {
        "forward, past the end": bg[G - 95:] + extra,
        "forward, before the start": extra + bg[:95],
        "reverse, past the end": rc(bg[G - 95:] + extra),
        "reverse, before the start": rc(extra + bg[:95]),
    }
    for what, read in reads.items():
        out, log, st = run(oracle_mod, bg, read)
        assert out == (-1, -1, -1, -1, 0) and log == [], what
        assert st["candidates"] == 0 and st["seeds_looked_up"] == 10, what
