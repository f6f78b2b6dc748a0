"""CPU checks of the HIP library: it loads, exports every declared symbol, and its
host-side index layout and seed order agree with the oracle. No GPU calls."""
import os
import random
import re

import pytest

from conftest import ROOT


@pytest.fixture(scope="session")
def snapgpu():
    import paper_1111_5572_amd as m
    if not os.path.exists(m.LIB_PATH):
        m.build_library()
    return m


def declared_functions():
    names = []
    inc = os.path.join(ROOT, "include")
    for f in sorted(os.listdir(inc)):
        if not f.endswith(".h"):
            continue
        text = open(os.path.join(inc, f)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w\s\*]*?\b(snap_\w+)\s*\(", text, flags=re.M):
            names.append(m.group(1))
    return sorted(set(names))


def test_library_exports_every_declared_symbol(snapgpu):
    import ctypes
    names = declared_functions()
    assert "snap_align" in names and "snap_index_build" in names
    lib = ctypes.CDLL(snapgpu.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_strerror_and_defaults(snapgpu):
    assert snapgpu.strerror(0) == "ok"
    assert "invalid" in snapgpu.strerror(1)
    p = snapgpu.default_params()
    assert (p.n_min, p.n_cap, p.bp_per_seed, p.conf_c, p.max_hits, p.d_max_pct, p.bucket) == (10, 32, 100, 2, 300, 0, 32)
    assert snapgpu.max_limit() >= 16


def test_seed_order_matches_oracle(snapgpu, oracle_mod):
    for s in (1, 5, 8, 12, 20, 31, 32):
        for L in (0, s - 1, s, s + 1, 2 * s - 1, 2 * s, 99, 100, 101, 250, 1000, 9999):
            for n in (1, 5, 10, 14, 32):
                if L < 0:
                    continue
                assert snapgpu.debug_seed_offsets(L, s, n) == oracle_mod.seed_offsets(L, s, n), (s, L, n)


@pytest.mark.parametrize("s", [1, 4, 9, 16, 20, 31, 32])
def test_host_table_lookup_vs_oracle(snapgpu, oracle_mod, synth_mod, s):
    g = synth_mod.genome_repeats(40_000, 3 + s, n_frac=0.01, n_run_lo=30, n_run_hi=300)
    gs = g.tobytes().decode()
    rnd = random.Random(s)
    queries = [gs[q:q + s] for q in rnd.sample(range(len(gs) - s), 150)]
    queries += ["".join(rnd.choice("ACGT") for _ in range(s)) for _ in range(50)]
    # palindromic seeds (equal to their reverse complement) for even s
    if s % 2 == 0:
        half = "".join(rnd.choice("ACGT") for _ in range(s // 2))
        comp = {"A": "T", "C": "G", "G": "C", "T": "A"}
        pal = half + "".join(comp[c] for c in reversed(half))
        queries.append(pal)
        gs2 = gs[:1000] + pal + gs[1000 + s:]
    else:
        gs2 = gs
    windows, got = snapgpu.debug_host_lookup(gs2, s, queries)
    ix = oracle_mod.Index(gs2.encode(), s)
    assert windows == ix.windows
    comp = str.maketrans("ACGTN", "TGCAN")
    for q, (f, r, first) in zip(queries, got):
        occ = ix.occ(q)
        if occ is None:
            assert (f, r, first) == (-1, -1, -1)
            continue
        rocc = ix.occ(q.translate(comp)[::-1])
        assert f == len(occ) and r == len(rocc), q
        assert first == (occ[0] if occ else -1)
    ix.close()


def test_host_table_tandem_counts(snapgpu, oracle_mod, synth_mod):
    """Seeds inside a long tandem array have hundreds of hits; counts stay exact."""
    g = synth_mod.genome_uniform(20_000, 5).tobytes().decode()
    g = g[:5000] + ("ACGTTGCA" * 500)[:3000] + g[8000:]
    q = [g[5100:5120], g[5101:5121], g[6000:6020]]
    _, got = snapgpu.debug_host_lookup(g, 20, q)
    ix = oracle_mod.Index(g.encode(), 20)
    comp = str.maketrans("ACGT", "TGCA")
    for s_, (f, r, _) in zip(q, got):
        assert f == len(ix.occ(s_)) and r == len(ix.occ(s_.translate(comp)[::-1]))
        assert f + r > 300
    ix.close()


def test_host_table_single_key(snapgpu, oracle_mod):
    """A homopolymer genome has one distinct seed: every window groups under one key
    (the build's parallel grouping must not split a run of equal keys)."""
    g = "A" * 12_000 + "C" * 25
    q = ["A" * 20, "T" * 20, "A" * 10 + "C" * 10]
    windows, got = snapgpu.debug_host_lookup(g, 20, q)
    ix = oracle_mod.Index(g.encode(), 20)
    assert windows == ix.windows
    comp = str.maketrans("ACGT", "TGCA")
    for s_, (f, r, first) in zip(q, got):
        occ, rocc = ix.occ(s_), ix.occ(s_.translate(comp)[::-1])
        assert (f, r) == (len(occ), len(rocc)), s_
        assert first == (occ[0] if occ else -1)
    assert got[0][0] == 12_000 - 19
    ix.close()
