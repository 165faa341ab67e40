"""Host checks of bench.py (no GPU): the one-GPU contract, the algorithmic
byte count it prices the roofline with, and its amortisation of the
regrouping pass's HBM bytes."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_exits_with_a_message(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_algorithmic_bytes():
    sys.path.insert(0, ROOT)
    import bench
    # FP32, 64^3 x 64 ppc x 2 species: 28 B read + 28 B written per particle,
    # E, B^n, B^{n+1} read and J, M written per node (4 B each)
    assert bench.algorithmic_bytes("f32", 33554432, 262144) == 2 * 28 * 33554432 + 4 * 138 * 262144 == 2023751680
    assert bench.algorithmic_bytes("f64", 33554432, 262144) == 2 * 48 * 33554432 + 8 * 138 * 262144
    # a per-particle charge adds one read per particle
    assert bench.algorithmic_bytes("f32", 10, 1, q_read=10) - bench.algorithmic_bytes("f32", 10, 1) == 40


def test_traffic_record_matches_its_profile():
    """The byte counts bench.py reports are the ones its profile summary states."""
    sys.path.insert(0, ROOT)
    import bench
    prof = open(os.path.join(ROOT, bench.TRAFFIC["profile"])).read()
    assert bench.TRAFFIC["sources_sha256"] in prof
    assert f"{bench.TRAFFIC['plain_call'] / 1e9:.3f} GB" in prof
    assert f"{bench.TRAFFIC['regroup_call'] / 1e9:.3f} GB" in prof
