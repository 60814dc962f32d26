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


@pytest.mark.parametrize("prec,mask,expect", [("mixed", True, 45), ("f32", True, 21),
                                              ("f64", True, 41), ("mixed", False, 44)])
def test_point_sweep_bytes(prec, mask, expect):
    b, per_pf = bench.point_sweep_bytes(2000, 500, 22965, prec, mask)
    assert per_pf == expect
    assert b == 2000 * 500 * expect + 40 * 22965
