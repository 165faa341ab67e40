"""Writes tests/golden/oracle_small_cases.json from the FP64 oracle alone.

The paper prints no worked numeric example of the method, so the stored
values are the oracle's, for two small cases whose inputs are given in the
file: a lone particle gyrating in a uniform B (Eqs. 2, 4, 5, 8; its velocities
also have a closed form, the Cayley rotation, checked by the test), and the
moments (Eqs. 1, 3) of a few particles on a 3 x 2 x 2 grid (whose sums obey
the partition-of-unity rules, also checked). Run from the repository root:
    python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
from oracle import oracle as O  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_small_cases.json")


def gyration_case():
    n, h, dt, qom = (4, 4, 4), (0.5, 0.5, 0.5), 0.1, -1.0
    x = np.array([[1.1], [0.7], [1.3]])
    v = np.array([[0.03], [-0.02], [0.01]])
    nn = int(np.prod(n))
    E = np.zeros((3, nn))
    B = np.zeros((3, nn))
    B[2] = 0.2
    xs, vs = [], []
    for _ in range(8):
        x, v = O.move(n, h, dt, x, v, qom, E, B)
        xs.append(x[:, 0].tolist())
        vs.append(v[:, 0].tolist())
    return {"n": n, "h": h, "dt": dt, "qom": qom, "x0": [1.1, 0.7, 1.3], "v0": [0.03, -0.02, 0.01],
            "B": [0.0, 0.0, 0.2], "x": xs, "v": vs}


def moments_case():
    n, h, dt, qom = (3, 2, 2), (0.5, 0.5, 0.5), 0.1, -1.0
    x = np.array([[0.1, 0.9, 1.4, 0.6], [0.2, 0.7, 0.05, 0.95], [0.3, 0.45, 0.8, 0.1]])
    v = np.array([[0.05, -0.02, 0.01, 0.03], [0.0, 0.04, -0.03, 0.02], [-0.01, 0.02, 0.05, -0.04]])
    q = np.array([-1e-3, -2e-3, -1.5e-3, -0.5e-3])
    nn = int(np.prod(n))
    B = np.zeros((3, nn))
    B[0], B[1], B[2] = 0.05, -0.1, 0.2
    J, M27 = O.moments(n, h, dt, x, v, q, qom, B)
    M14 = O.m14(n, M27)
    return {"n": n, "h": h, "dt": dt, "qom": qom, "x": x.tolist(), "v": v.tolist(), "q": q.tolist(),
            "B": [0.05, -0.1, 0.2], "J": J.tolist(), "M14": M14.tolist()}


if __name__ == "__main__":
    data = {"about": "FP64 oracle outputs for two small cases (see make_golden.py); regression pins",
            "gyration": gyration_case(), "moments": moments_case()}
    with open(OUT, "w") as f:
        json.dump(data, f, indent=1)
    print("wrote", OUT)
