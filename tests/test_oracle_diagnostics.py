"""Pins of the oracle's diagnostic moments (Sec. III, diagnostics for I/O:
charge density, the current without the velocity rotation, and the
charge-weighted second velocity moment as the pressure tensor).

Each is checked against something other than itself: sum rules, the first
moment that linear interpolation reproduces, a textbook numpy CIC scatter,
numbers worked out by hand for one particle, and the hatted current of
Eq. 1 at B = 0 (where alpha is the identity).
"""
import numpy as np

from tests.helpers import cic_nodes_weights, relerr

PAIRS = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]   # P component order: xx, xy, xz, yy, yz, zz


def _plasma(inputs, n=(5, 4, 3), ppc=7, seed=11):
    return inputs.uniform_plasma(60 + seed, n, ppc)


def test_sum_rules(oracle, inputs):
    """V sum_N rho = sum_p q_p, V sum_N J = sum_p q_p v_p, V sum_N P_ij = sum_p q_p v_i v_j
    (partition of unity), for every species and component."""
    p = _plasma(inputs)
    V = np.prod(p.h)
    for s in p.species:
        rho, Jd, P = oracle.diagnostics(p.n, p.h, s.x, s.v, s.q)
        assert relerr(V * rho.sum(), s.q.sum()) < 1e-13
        assert relerr(V * Jd.sum(axis=1), (s.q * s.v).sum(axis=1)) < 1e-13
        ref = np.array([(s.q * s.v[i] * s.v[j]).sum() for i, j in PAIRS])
        assert relerr(V * P.sum(axis=1), ref) < 1e-13


def test_first_moment(oracle, inputs):
    """Linear interpolation reproduces x: V sum_N x_N rho_N = sum_p q_p x_p (and with
    v for J), for particles whose 8 nodes do not wrap. A corner paired with the
    wrong weight fails this."""
    p = _plasma(inputs, n=(6, 5, 4), ppc=9, seed=12)
    V = np.prod(p.h)
    L = np.array(p.L)
    for s in p.species:
        keep = np.all(s.x < (L - np.array(p.h))[:, None], axis=0)
        x, v, q = s.x[:, keep], s.v[:, keep], s.q[keep]
        rho, Jd, _ = oracle.diagnostics(p.n, p.h, x, v, q)
        idx = np.arange(p.nn)
        xn = np.stack([(idx % p.n[0]) * p.h[0], ((idx // p.n[0]) % p.n[1]) * p.h[1],
                       (idx // (p.n[0] * p.n[1])) * p.h[2]])
        assert relerr(V * (xn * rho).sum(axis=1), (q * x).sum(axis=1)) < 1e-12
        for c in range(3):
            assert relerr(V * (xn * Jd[c]).sum(axis=1), (q * v[c] * x).sum(axis=1)) < 1e-12


def test_textbook_cic_scatter(oracle, inputs):
    """Against a numpy CIC scatter written separately (node index and weight per corner)."""
    p = _plasma(inputs, n=(3, 4, 2), ppc=5, seed=13)
    V = np.prod(p.h)
    s = p.species[1]
    rho, Jd, P = oracle.diagnostics(p.n, p.h, s.x, s.v, s.q)
    nodes, w = cic_nodes_weights(s.x, p.n, p.h)
    r_rho = np.zeros(p.nn)
    np.add.at(r_rho, nodes.ravel(), (w * s.q[:, None]).ravel() / V)
    assert relerr(rho, r_rho) < 1e-13
    for c in range(3):
        r = np.zeros(p.nn)
        np.add.at(r, nodes.ravel(), (w * (s.q * s.v[c])[:, None]).ravel() / V)
        assert relerr(Jd[c], r) < 1e-13
    for k, (i, j) in enumerate(PAIRS):
        r = np.zeros(p.nn)
        np.add.at(r, nodes.ravel(), (w * (s.q * s.v[i] * s.v[j])[:, None]).ravel() / V)
        assert relerr(P[k], r) < 1e-13


def test_single_particle_by_hand(oracle):
    """One particle at x = (0.3, 0.6, 0.1) on a 3^3 grid with h = 0.5: cell (0, 1, 0),
    fractions (0.6, 0.2, 0.2). Charge 2, velocity (1, -2, 3), V = 0.125."""
    n, h = (3, 3, 3), (0.5, 0.5, 0.5)
    rho, Jd, P = oracle.diagnostics(n, h, np.array([[0.3], [0.6], [0.1]]), np.array([[1.0], [-2.0], [3.0]]),
                                    np.array([2.0]))
    # node (1, 1, 0) = index 1 + 3 * 1 = 4: weight 0.6 * 0.8 * 0.8 = 0.384
    # node (0, 2, 1) = index 0 + 3 * (2 + 3 * 1) = 15: weight 0.4 * 0.2 * 0.2 = 0.016
    assert abs(rho[4] - 2 * 0.384 / 0.125) < 1e-13
    assert abs(rho[15] - 2 * 0.016 / 0.125) < 1e-13
    assert abs(Jd[1, 4] - 2 * -2.0 * 0.384 / 0.125) < 1e-13
    assert abs(P[2, 15] - 2 * 1.0 * 3.0 * 0.016 / 0.125) < 1e-13   # xz
    assert abs(P[3, 4] - 2 * 4.0 * 0.384 / 0.125) < 1e-13          # yy
    assert np.count_nonzero(rho) == 8


def test_current_equals_hatted_current_at_B0(oracle, inputs):
    """With B = 0, alpha = I and the hatted current of Eq. 1 is the plain current."""
    p = _plasma(inputs, seed=14)
    BN = np.zeros((3, p.nn))
    for s in p.species:
        J, _ = oracle.moments(p.n, p.h, p.dt, s.x, s.v, s.q, s.qom, BN)
        _, Jd, _ = oracle.diagnostics(p.n, p.h, s.x, s.v, s.q)
        assert relerr(Jd, J) < 1e-13
