"""Exact-duplicate classes (Section 4.2, "Approach": identical substrings of a read's
length, so that a read is compared with each repeated string once) in the oracle.

Reading: a read of length L is compared at location p with the window G[p, p + L + K)
(K = d_max + c - 1, the largest limit), so locations whose W-base windows (W >= L + K)
are identical have the same distance at every limit; rep[p] is the smallest position
with p's W-base window. Pinned by brute force (all pairs of windows) and by the
distance being equal across a class for reads of that length."""
import numpy as np
import pytest


@pytest.mark.parametrize("W", [1, 5, 12, 40])
def test_dup_classes_brute_force(oracle_mod, synth_mod, W):
    """Every pair of windows compared directly, on a tandem-rich genome with N runs and
    mixed case (N equals N, case does not matter)."""
    g = synth_mod.genome_repeats(1_500, 3, n_frac=0.05, n_run_lo=5, n_run_hi=30).copy()
    g[700:760] = np.frombuffer((b"ACGTTA" * 10), np.uint8)   # a tandem array
    g[100:110] = g[100:110] + 32
    g[900:905] = ord("R")                                      # another N code
    rep = oracle_mod.dup_classes(g, W)
    norm = ["N" if c not in "ACGT" else c for c in g.tobytes().decode().upper()]
    G = len(norm)
    for p in range(G):
        if p + W > G:
            assert rep[p] == p
            continue
        w = norm[p:p + W]
        want = next(q for q in range(p + 1) if norm[q:q + W] == w)
        assert rep[p] == want, (p, rep[p], want)
    if W <= 12:
        assert (rep != np.arange(G)).sum() > 0   # some duplicates exist


def test_distance_equal_within_a_class(oracle_mod, synth_mod):
    """For reads of length L and every limit up to K, the bounded distance at a location
    equals the distance at its class representative (W = L + K)."""
    from synth.workloads import MID
    w = MID.scaled(genome_len=60_000, n_reads=1)
    g = w.make_genome()
    L, K = 100, 11
    rep = oracle_mod.dup_classes(g, L + K)
    dup = np.nonzero(rep != np.arange(len(g)))[0]
    assert len(dup) > 100
    rng = np.random.default_rng(3)
    for k in rng.choice(len(dup), 40, replace=False):
        p = int(dup[k])
        q = int(rep[p])
        assert q < p and bytes(g[p:p + L + K]).upper() == bytes(g[q:q + L + K]).upper()
        r = g[p:p + L].copy()   # a read from the location, with two substitutions
        for j in (17, 61):
            r[j] = ord("A") if r[j] != ord("A") else ord("C")
        assert oracle_mod.edit_distance(r, g[p:p + L + K], K) <= 2
        for lim in (0, 1, 2, 3, K):
            assert (oracle_mod.edit_distance(r, g[p:p + L + lim], lim) ==
                    oracle_mod.edit_distance(r, g[q:q + L + lim], lim))
