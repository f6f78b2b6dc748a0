"""The oracle's pins catch plausible mistakes in Algorithm 1 and in the readings of the
strided index and the exact-duplicate classes: each one-line change below (a wrong limit
case, a boundary test off by one, a dropped orientation, a wrong tie-break, a shorter text
window, an early return where the paper has none, an N test over one seed of a slot, t over
incomplete slots, a class on a shorter window or with the wrong representative) is applied
to a copy of oracle.c, and the copy must fail at least one of the oracle's CPU pin tests."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# (what the change breaks, original line, mutated line)
MUTATIONS = [
    ("d_limit, third case: d_best - 1 (Algorithm 1)",
     "return st->d_best - 1;", "return st->d_best;"),
    ("d_limit, third case taken as the second",
     "return st->d_best - 1;", "return st->d_best + c - 1;"),
    ("early multiple-hits return needs d_best < c",
     "if (st.d_best < c && st.d_second < st.d_best + c) {", "if (st.d_best <= c && st.d_second < st.d_best + c) {"),
    ("single call needs d_second >= d_best + c",
     "if (st.d_best <= dmax && st.d_second >= st.d_best + c) call = 1;",
     "if (st.d_best <= dmax && st.d_second > st.d_best + c) call = 1;"),
    ("h_max counts both orientations",
     "entries += (fhi - flo) + (rhi - rlo);", "entries += (fhi - flo);"),
    ("t counts only round-0 seeds",
     "if (o % s == 0 && np == stride) t++;", "t++;"),
    ("t does not count seeds over h_max",
     "if (entries > hmax) { stt->seeds_over_limit++; continue; }",
     "if (entries > hmax) { stt->seeds_over_limit++; if (o % s == 0) t++; continue; }"),
    ("selection ties go to the smaller p",
     "if (k < 0 || w->c[i].hits > w->c[k].hits) k = i;", "if (k < 0 || w->c[i].hits >= w->c[k].hits) k = i;"),
    ("a bucket keeps the lower p on equal distance",
     "} else if (d < w->b[j].d || (d == w->b[j].d && p < w->b[j].p)) {", "} else if (d < w->b[j].d) {"),
    ("best-location ties: forward before reverse",
     "if (x->d < y->d || (x->d == y->d && (x->p < y->p || (x->p == y->p && x->strand < y->strand)))) bi = j;",
     "if (x->d < y->d || (x->d == y->d && (x->p < y->p || (x->p == y->p && x->strand > y->strand)))) bi = j;"),
    ("text window of L + limit bases",
     "int64_t want = (int64_t)L + (lim > 0 ? lim : 0);", "int64_t want = (int64_t)L + (lim > 0 ? lim - 1 : 0);"),
    # the strided index (reading S1)
    ("a slot is skipped for an N in any of its seeds, not only the first",
     "if (has_n(w->fwd + o, s + np - 1)) { stt->seeds_with_n++; continue; }",
     "if (has_n(w->fwd + o, s)) { stt->seeds_with_n++; continue; }"),
    ("t counts a round-0 slot only when all its seeds fit the read",
     "if (o % s == 0 && np == stride) t++;", "if (o % s == 0) t++;"),
    # exact-duplicate classes (reading S2)
    ("a class needs the whole W-base window identical",
     "if (memcmp(codes + order[k], codes + order[k - 1], (size_t)W) == 0) rep[order[k]] = rep[order[k - 1]];",
     "if (memcmp(codes + order[k], codes + order[k - 1], (size_t)W - 1) == 0) rep[order[k]] = rep[order[k - 1]];"),
    ("a class's representative is its smallest position, not the previous member",
     "if (memcmp(codes + order[k], codes + order[k - 1], (size_t)W) == 0) rep[order[k]] = rep[order[k - 1]];",
     "if (memcmp(codes + order[k], codes + order[k - 1], (size_t)W) == 0) rep[order[k]] = order[k - 1];"),
    ("no early return while scoring the remaining locations",
     "                score(ix, w, &st, k, L, dmax, pr, stt, lg);\n            }",
     "                score(ix, w, &st, k, L, dmax, pr, stt, lg);\n"
     "                if (st.d_best < c && st.d_second < st.d_best + c) { call = 2; break; }\n            }"),
]

PIN_TESTS = ["tests/test_oracle_algorithm1.py", "tests/test_oracle_branches.py", "tests/test_oracle_pins.py",
             "tests/test_oracle_invariants.py", "tests/test_oracle_strided.py", "tests/test_oracle_dups.py"]


@pytest.mark.parametrize("what,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_mutation_fails_a_pin(tmp_path, synth_mod, what, old, new):
    src = open(os.path.join(ROOT, "oracle", "oracle.c")).read()
    assert src.count(old) == 1, f"the line to mutate is not in oracle.c once: {old}"
    for d in ("oracle", "synth", "tests"):
        shutil.copytree(os.path.join(ROOT, d), tmp_path / d,
                        ignore=shutil.ignore_patterns("__pycache__", "liboracle.so", "*.tmp"))
    (tmp_path / "oracle" / "oracle.c").write_text(src.replace(old, new))
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread", "-o",
                           str(tmp_path / "oracle" / "liboracle.so"), str(tmp_path / "oracle" / "oracle.c")])
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider",
                        *PIN_TESTS], cwd=tmp_path, capture_output=True, text=True, timeout=300)
    assert r.returncode == 1, f"mutation survived every pin: {what}\n{r.stdout[-2000:]}"
