"""CPU checks of bench.py's command-line contract and byte accounting."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True)
    assert out.returncode == 2
    assert "one GPU" in out.stderr


# the graded bytes follow the method at FP32 state (X, mask with missing
# data, U read and write, A' read, A write): 21 B per point-feature with a
# mask, 20 without, and 24 B per edge for the point sweep's neighbour slots
# and q factors; the whole iteration adds the edge stage's 8 B per
# point-feature and comes to 60 B per edge
@pytest.mark.parametrize("mask,k1", [(True, 21), (False, 20)])
def test_algorithmic_bytes(mask, k1):
    point, it, per_pf = bench.algorithmic_bytes(2000, 500, 22965, mask)
    assert per_pf == k1
    assert point == 2000 * 500 * k1 + 24 * 22965
    assert it == 2000 * 500 * (k1 + 8) + 60 * 22965


# what this implementation moves: the mixed precision keeps FP64 U and A as
# hi + lo (the FP32 gather copy and an FP32 low half); without a mask U is
# neither read nor written (it follows from X and A'); with a mask and one
# item per wave U is read and written in full, with several items per wave
# only at the missing entries
@pytest.mark.parametrize("prec,mask,expect", [("mixed", True, 37), ("f32", True, 21),
                                              ("f64", True, 41), ("mixed", False, 20),
                                              ("f32", False, 12), ("f64", False, 24)])
def test_implementation_bytes(prec, mask, expect):
    b, per_pf = bench.implementation_bytes(2000, 500, 22965, prec, mask)
    assert per_pf == expect
    assert b == 2000 * 500 * expect + 24 * 22965


def test_implementation_bytes_side_array():
    b, per_pf = bench.implementation_bytes(2000, 500, 22965, "mixed", True, missing=50000)
    assert per_pf == 21
    assert b == 2000 * 500 * 21 + 16 * 50000 + 24 * 22965


def test_host_cpu_description():
    h = bench.host_cpu()
    assert h["nproc"] >= 1 and 1 <= h["usable"] <= h["nproc"]
    assert isinstance(h["model"], str)


def _fake_counters(path, counter, copy_kib, kp_kib):
    import csv
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writerow([1, "__amd_rocclr_copyBuffer", counter, copy_kib])
        w.writerow([2, "void ccmi::k_point<1, 4, false>(ccmi::PointArgs)", counter, kp_kib])
        w.writerow([3, "void ccmi::k_point<1, 4, false>(ccmi::PointArgs)", counter, kp_kib + 2])
        w.writerow([4, "void ccmi::k_edge_items<1, 8>(ccmi::EdgeArgs)", counter, 7])


def test_counter_summary_scales_by_the_copy_and_checks_the_source_hash(tmp_path, capsys, monkeypatch):
    f, w = tmp_path / "f.csv", tmp_path / "w.csv"
    _fake_counters(f, "FETCH_SIZE", 131072.0, 1000.0)   # the copy reads half: factor 2
    _fake_counters(w, "WRITE_SIZE", 262144.0, 500.0)
    bench.pmc_summary(str(f), str(w), 256, "rocprofv3 --pmc {counter} -- x")
    text = capsys.readouterr().out
    assert "factors 2.0000 and 1.0000" in text
    prof = tmp_path / "traffic.md"
    prof.write_text(text)
    monkeypatch.setattr(bench, "TRAFFIC_PROFILES", {("expression", "mixed"): str(prof)})
    got = bench.stored_traffic("expression", "mixed")
    assert got == pytest.approx((1001.0 * 2.0 + 501.0) * 1024)
    assert bench.stored_traffic("genotype", "mixed") is None
    assert bench.stored_traffic("expression", "f64") is None
    prof.write_text(text.replace(bench.kernel_source_hash(), "0" * 64))
    assert bench.stored_traffic("expression", "mixed") is None


def test_malformed_counter_summary_gives_no_traffic(tmp_path, monkeypatch):
    prof = tmp_path / "traffic.md"
    prof.write_text("```json\n{not json\n```\n")
    monkeypatch.setattr(bench, "TRAFFIC_PROFILES", {("expression", "mixed"): str(prof)})
    assert bench.stored_traffic("expression", "mixed") is None
    monkeypatch.setattr(bench, "TRAFFIC_PROFILES", {("expression", "mixed"): str(tmp_path / "missing.md")})
    assert bench.stored_traffic("expression", "mixed") is None


def test_committed_counter_summaries_parse():
    # each committed summary holds a record for the point sweep; whether its
    # source hash is current decides only whether the bench reports it
    import json
    import re
    for (wl, prec), path in bench.TRAFFIC_PROFILES.items():
        rec = json.loads(re.search(r"```json\n(.*?)\n```", open(path).read(), re.S).group(1))
        assert "k_point" in rec["kernel"], path
        assert rec["fetch_kib_per_launch"] > 0 and rec["write_kib_per_launch"] > 0, path
        assert 1.5 < rec["fetch_factor"] < 2.5 and 0.5 < rec["write_factor"] < 1.5, path
