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


def test_host_cpu_reports_threads():
    sys.path.insert(0, ROOT)
    import bench
    info = bench.host_cpu()
    assert info["threads"] >= 1 and info["cpus_allowed"] >= info["threads"]


def test_mass_blocks_27_from_14_round_trip(oracle, inputs):
    """The CPU leg rebuilds the 27 blocks of every node from the 14 stored
    ones for the oracle's field solve: the oracle's own 27 blocks, which obey
    M_{g,g+o} = M_{g+o,g} (Eq. 3) to the rounding of the order of the two
    weights in each product."""
    import numpy as np
    sys.path.insert(0, ROOT)
    import bench
    p = inputs.uniform_plasma(31, (5, 4, 3), 6)
    rng = np.random.default_rng(2)
    BN = np.array([[0.01], [0.02], [0.2]]) + 0.05 * rng.standard_normal((3, p.nn))
    M27 = np.zeros((27, 9, p.nn))
    for s in p.species:
        oracle.moments(p.n, p.h, p.dt, s.x, s.v, s.q, s.qom, BN, None, M27)
    back = bench._m27_from_m14(oracle, p.n, oracle.m14(p.n, M27))
    assert np.max(np.abs(back - M27)) <= 1e-14 * np.max(np.abs(M27))


def test_oracle_error_leg_on_a_small_run(oracle, inputs):
    """The oracle-error leg recovers a zero error when the 'GPU' results are
    the oracle's own (an FP32 state run through the oracle), and a nonzero
    one when J is perturbed."""
    import numpy as np
    sys.path.insert(0, ROOT)
    import bench
    p = inputs.uniform_plasma(33, (6, 6, 4), 5)
    st = inputs.to_f32_state(p)
    rng = np.random.default_rng(3)
    Et = (1e-3 * rng.standard_normal((3, p.nn))).astype(np.float32)
    Bm = (np.array([[0.0], [0.0], [0.2]]) + 0.01 * rng.standard_normal((3, p.nn))).astype(np.float32)
    Bd = (Bm + 1e-3 * rng.standard_normal((3, p.nn))).astype(np.float32)
    J = np.zeros((3, p.nn))
    M27 = np.zeros((27, 9, p.nn))
    J0 = np.zeros((3, p.nn))
    M0 = np.zeros((27, 9, p.nn))
    species = []
    for s, f in zip(p.species, st):
        oracle.moments(p.n, p.h, p.dt, f["x64"], f["v64"], f["q64"], s.qom, Bm.astype(np.float64), J0, M0)
        _, _, J, M27, _ = oracle.move_moments_threads(p.n, p.h, p.dt, f["x64"], f["v64"], f["q64"], s.qom,
                                                      Et.astype(np.float64), Bm.astype(np.float64),
                                                      Bd.astype(np.float64), J, M27, 2)
        species.append(dict(cell=f["cell"], off=f["off"], v=f["v"], q=f["q"], q_const=0.0, qom=s.qom))
    M14 = oracle.m14(p.n, M27)
    sol = oracle.field_solve(p.n, p.h, p.dt, M0, J0, p.E, p.B_C, 1e-10)
    rec = [dict(species=species, Et=Et, Bmove=Bm, Bdep=Bd, J1=J, M1=M14, J=J0, M=oracle.m14(p.n, M0), E=p.E,
                BC=p.B_C, E1=sol["E_next"])]
    out = bench.oracle_error(oracle, p, rec, threads=2, nnodes=4)
    assert out["J"] < 1e-13 and out["M"] < 1e-13 and out["E"] < 1e-9
    rec[0]["J1"] = J * (1.0 + 1e-4)
    assert bench.oracle_error(oracle, p, rec, threads=2, nnodes=4)["J"] > 5e-5
