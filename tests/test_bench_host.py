"""Host-side contract of bench.py: one GPU only, and strict JSON lines."""
import json
import math
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


def test_study_lines_are_strict_json():
    sys.path.insert(0, ROOT)
    import bench
    out = bench._finite({"a": math.nan, "b": [1.0, math.inf, {"c": -math.inf}], "d": (2, "x")})
    assert out == {"a": None, "b": [1.0, None, {"c": None}], "d": [2, "x"]}
    json.loads(json.dumps(out, allow_nan=False))
