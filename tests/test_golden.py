"""Pins of the oracle to the stored fixture tests/golden/oracle_small_cases.json
(written by tests/golden/make_golden.py from the oracle alone; the paper prints
no worked example): the oracle reproduces it bit for bit, and the stored values
themselves obey what the mathematics fixes -- the lone particle's velocities are
the Cayley rotation about B by 2 atan(beta |B|) per step (Eqs. 2, 4, 5) and its
positions the push of Eq. 8; the moments obey the sum rules of Eqs. 1 and 3
with alpha obtained by solving the implicit velocity equation."""
import json
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "oracle_small_cases.json")))


def _rot_z(w, ang):
    c, s = math.cos(ang), math.sin(ang)
    return np.array([c * w[0] - s * w[1], s * w[0] + c * w[1], w[2]])


def test_oracle_reproduces_fixture(oracle):
    import importlib.util
    spec = importlib.util.spec_from_file_location("make_golden", os.path.join(HERE, "golden", "make_golden.py"))
    mg = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mg)
    g, m = mg.gyration_case(), mg.moments_case()
    assert g["x"] == GOLD["gyration"]["x"] and g["v"] == GOLD["gyration"]["v"]
    assert m["J"] == GOLD["moments"]["J"] and m["M14"] == GOLD["moments"]["M14"]


def test_fixture_gyration_is_the_cayley_rotation():
    g = GOLD["gyration"]
    beta = g["qom"] * g["dt"] / 2
    phi = 2 * math.atan(beta * g["B"][2])
    v0 = np.array(g["v0"])
    L = np.array(g["n"]) * np.array(g["h"])
    x = np.array(g["x0"])
    for k, (xs, vs) in enumerate(zip(g["x"], g["v"]), start=1):
        assert np.max(np.abs(np.array(vs) - _rot_z(v0, -k * phi))) < 1e-15
        x = np.mod(x + g["dt"] * np.array(vs), L)
        assert np.max(np.abs(np.array(xs) - x)) < 1e-14


def test_fixture_moments_obey_sum_rules():
    m = GOLD["moments"]
    V = float(np.prod(m["h"]))
    beta = m["qom"] * m["dt"] / 2
    B = np.array(m["B"])
    cross = np.array([[0.0, -B[2], B[1]], [B[2], 0.0, -B[0]], [-B[1], B[0], 0.0]])   # [B x] u = B x u
    # alpha u solves vbar - beta vbar x B = u, i.e. (I + beta [B x]) vbar = u
    alpha = np.linalg.solve(np.eye(3) + beta * cross, np.eye(3))
    q, v = np.array(m["q"]), np.array(m["v"])
    J, M14 = np.array(m["J"]), np.array(m["M14"])
    assert np.max(np.abs(V * J.sum(axis=1) - (alpha @ v) @ q)) < 1e-17
    # sum over every node pair of the blocks (offset 0 once, the 13 others twice) = sum_p q beta alpha
    total = M14[0].sum(axis=1) + 2 * M14[1:].sum(axis=(0, 2))
    assert np.max(np.abs(V * total - beta * q.sum() * alpha.reshape(9))) < 1e-17
