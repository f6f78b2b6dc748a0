"""Host-side logic of bench.py, no GPU: the HBM-traffic summary is used only for the
kernel, workload, schedule and kernel source it was taken on; the roofline counts the
first verification's diagonal extensions on their own; the accuracy metrics of the
h_max harness; more than one GPU is refused with a message."""
import importlib.util
import json
import os
import subprocess
import sys
from types import SimpleNamespace

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _summary(tmp_path, **kv):
    p = tmp_path / "traffic.txt"
    p.write_text("# comment: ignored\n" + "".join(f"{k}: {v}\n" for k, v in kv.items()))
    return str(p)


def test_traffic_needs_matching_kernel_source(bench, tmp_path):
    sha = bench.kernel_source_sha1()
    good = dict(kernel="verify", workload="mid", schedule="5,6,6,0,1,0", source_sha1=sha, bytes_per_launch=123)
    assert bench.read_traffic(_summary(tmp_path, **good), "verify", "mid", (5, 6, 6, 0, 1, 0)) == 123
    # the same schedule written with its defaults spelled out, or with another worker count
    assert bench.read_traffic(_summary(tmp_path, **good), "verify", "mid", (5, 6, 6, 0, 1, 0, 0, 0)) == 123
    assert bench.read_traffic(_summary(tmp_path, **good), "verify", "mid", (5, 6, 6, 0, 1, 0, 0, 3)) == 123
    assert bench.read_traffic(_summary(tmp_path, **good), "verify", "mid", (5, 6, 6, 0, 1, 0, 4096, 0)) is None
    for key, bad in (("source_sha1", "0" * 40), ("kernel", "gather"), ("workload", "human"),
                     ("schedule", "5,5,5,0,1,0")):
        assert bench.read_traffic(_summary(tmp_path, **{**good, key: bad}), "verify", "mid", (5, 6, 6, 0, 1, 0)) is None
    missing = {k: v for k, v in good.items() if k != "source_sha1"}
    assert bench.read_traffic(_summary(tmp_path, **missing), "verify", "mid", (5, 6, 6, 0, 1, 0)) is None
    assert bench.read_traffic(str(tmp_path / "absent.txt"), "verify", "mid", (5, 6, 6, 0, 1, 0)) is None


def test_roofline_first_verification_counted_alone(bench):
    # ms totals per kernel over 10 launches each; 1e9 steps in all, 6e8 of them first-verification
    kern = {"verify": (10, 20.0), "verify_request": (10, 5.0), "verify_request_wave": (10, 15.0), "probe": (10, 4.0)}
    ctr = {"lv_steps": 1_000_000_000, "lv_steps_first": 600_000_000, "seed_slots": 0, "hits": 0, "locations": 0,
           "reads": 1_000_000}
    r = bench.roofline_of(kern, ctr, "verify")
    # 6e8 steps x 30 ops / 10 launches / 2 ms a launch
    assert r["achieved"] == pytest.approx(6e8 * 30 / 10 / 2e-3 / 1e12, rel=1e-4)
    assert r["bound"] == "alu" and r["unit"] == "TOP/s"
    q = bench.roofline_of(kern, ctr, "verify_request")
    # the request kernels share the other 4e8 steps by time: 5 of 20 ms
    assert q["achieved"] == pytest.approx(4e8 * 0.25 * 30 / 10 / 0.5e-3 / 1e12, rel=1e-4)
    assert bench.roofline_of(kern, ctr, "absent") is None
    assert bench.roofline_of(kern, ctr)["kernel"] == "verify"   # the largest total
    assert r["extensions_per_read_executed"] == 1000


def test_roofline_counts_algorithm1_own_extensions(bench):
    # the method needs 100 extensions a read (oracle sample); the kernels ran 1000 a read:
    # 60% of them in the first verification, which is credited with 60% of the method's
    kern = {"verify": (10, 20.0), "verify_request": (10, 5.0), "verify_request_wave": (10, 15.0)}
    ctr = {"lv_steps": 1_000_000_000, "lv_steps_first": 600_000_000, "seed_slots": 0, "hits": 0, "locations": 0,
           "reads": 1_000_000}
    method = {"lv_extensions_per_read": 100.0}
    r = bench.roofline_of(kern, ctr, "verify", method)
    assert r["achieved"] == pytest.approx(1e8 * 0.6 * 30 / 10 / 2e-3 / 1e12, rel=1e-4)
    assert r["achieved_executed"] == pytest.approx(6e8 * 30 / 10 / 2e-3 / 1e12, rel=1e-3)
    assert r["extensions_per_read_method"] == 100.0
    ph = bench.phases_of(kern, ctr, method)
    # every verify kernel together: 1e8 extensions x 30 ops over 40 ms
    assert ph["verify_all"]["achieved"] == pytest.approx(1e8 * 30 / 40e-3 / 1e12, rel=1e-3)
    assert ph["verify"]["kernel"] == "verify"


def test_accuracy_metrics(bench):
    truth = SimpleNamespace(n=5, truth_pos=np.array([100, 200, 300, 400, 500]), truth_strand=np.array([0, 1, 0, 1, 0]))
    pos = np.array([100, 232, 340, 400, -1])
    strand = np.array([0, 1, 0, 0, -1], dtype=np.int8)
    call = np.array([1, 1, 1, 1, 0], dtype=np.int8)   # four single calls, one not found
    out = (pos, strand, None, None, call)
    m = bench.accuracy_of(out, truth)
    # read 2 is 40 bases off, read 3 on the wrong strand: 2 errors of 4 aligned
    assert m == {"aligned_pct": 80.0, "error_pct": 50.0}
    assert bench.accuracy_of(out, truth, tol=40)["error_pct"] == 25.0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    line = [l for l in r.stdout.splitlines() if l.startswith("{")]
    assert line and "one GPU" in json.loads(line[-1]).get("error", "") + r.stderr


def test_tuning_table_lookup(tmp_path):
    """Length classes and table entries of the autotuner (no GPU needed)."""
    sys.path.insert(0, ROOT)
    from paper_1111_5572_amd import autotune
    assert autotune.length_class(np.array([], np.int32)) == "empty"
    assert autotune.length_class(np.full(100, 100, np.int32)) == "64-64"
    assert autotune.length_class(np.full(100, 250, np.int32)) == "128-128"
    mixed = np.concatenate([np.full(50, 100), np.full(50, 250)]).astype(np.int32)
    assert autotune.length_class(mixed) == "64-128"
    table = tmp_path / "t.json"
    table.write_text(json.dumps({"plain:64-64": {"tuning": [5, 6, 6, 0, 1, 0, 0, 3]},
                                 "batched:64-64": {"tuning": [1, 2]}}))
    lens = np.full(10, 100, np.int32)
    assert autotune.lookup(lens, batched=False, path=str(table)) == (5, 6, 6, 0, 1, 0, 0, 3)
    assert autotune.lookup(lens, batched=True, path=str(table)) is None   # too few fields
    assert autotune.lookup(np.full(10, 5000, np.int32), batched=False, path=str(table)) is None
    # the committed table has the mid entry the benchmark uses
    assert autotune.lookup(lens, batched=False) is not None


def test_autotune_candidates_for_mixed_lengths():
    """Plain calls on reads of mixed lengths also try pass1_max_len at the length quartiles
    below the longest read; one length, or the batched form, adds nothing."""
    sys.path.insert(0, ROOT)
    from paper_1111_5572_amd import autotune
    base = len(autotune.CANDIDATES)
    mixed = np.concatenate([np.full(50, 100), np.full(50, 250)]).astype(np.int32)
    c = autotune.candidates_for(mixed, batched=False)
    extra = c[base:]
    assert extra and all(len(x) == 10 for x in extra)
    assert sorted({x[9] for x in extra}) == [100, 175]
    assert all(0 < x[9] < 250 for x in extra)
    assert len(autotune.candidates_for(np.full(100, 100, np.int32), batched=False)) == base
    assert len(autotune.candidates_for(mixed, batched=True)) == base
    assert len(autotune.candidates_for(np.array([], np.int32), batched=False)) == base


def test_accuracy_grid_dmax(bench):
    # 1.5 times the expected edits, at least 8, at most the largest limit minus c - 1
    assert bench.grid_dmax(100, 0.02) == 8
    assert bench.grid_dmax(100, 0.10) == 15
    assert bench.grid_dmax(1000, 0.05) == 75
    assert bench.grid_dmax(10000, 0.10) == 1022
    assert [row[1] for row in bench.ACCURACY_GRID].count(10000) == 3


def test_roofline_of_a_replay_kernel(bench):
    # the replays share Algorithm 1's selection scans by time: 3 of 4 ms to the heavy one
    kern = {"replay_heavy": (10, 30.0), "replay": (10, 10.0), "verify": (10, 5.0)}
    ctr = {"lv_steps": 1, "lv_steps_first": 1, "seed_slots": 0, "hits": 0, "locations": 0, "reads": 1_000_000}
    r = bench.roofline_of(kern, ctr, None, {"select_visits_per_read": 50.0, "lv_extensions_per_read": 1.0})
    assert r["kernel"] == "replay_heavy" and r["bound"] == "alu"
    assert r["achieved"] == pytest.approx(50.0 * 1e6 * 0.75 * 4 / 10 / 3e-3 / 1e12, rel=1e-4)
    # without an oracle sample there is no work figure, and nothing is NaN
    q = bench.roofline_of(kern, ctr)
    assert q["achieved"] is None and q["frac"] is None
