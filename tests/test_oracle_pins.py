"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a closed
form, an invariant stated in the paper, an independent textbook
implementation, a library routine, or brute force on a tiny grid.
"""
import math

import numpy as np
import pytest

from tests.helpers import alpha_by_solve, cic_nodes_weights, cross_matrix, periodic_relerr, relerr

H = (0.5, 0.5, 0.5)
DT = 0.1


# ---------------------------------------------------------------------------
# P2: interpolation weights (linear in each dimension, 8 nodes)
# ---------------------------------------------------------------------------

def test_partition_of_unity_and_linear_reproduction(oracle):
    g = np.random.default_rng(11)
    n = (5, 4, 3)
    for _ in range(200):
        x = g.random(3) * np.array([n[d] * H[d] for d in range(3)])
        lo, W = oracle.weights(n, H, x)
        assert abs(W.sum() - 1.0) < 1e-15
        assert np.all(W >= 0.0)
        # first moment: sum_a W_a X_a = x with X_a the (unwrapped) node position
        first = np.zeros(3)
        for a in range(8):
            ad = (a & 1, (a >> 1) & 1, (a >> 2) & 1)
            first += W[a] * np.array([(lo[d] + ad[d]) * H[d] for d in range(3)])
        assert np.max(np.abs(first - x)) < 1e-14


def test_weights_match_textbook_cic(oracle):
    g = np.random.default_rng(12)
    n = (6, 5, 4)
    x = g.random((3, 50)) * np.array([[n[d] * H[d]] for d in range(3)])
    nodes, w = cic_nodes_weights(x, n, H)
    for p in range(50):
        lo, W = oracle.weights(n, H, x[:, p])
        assert np.allclose(W, w[p], rtol=0, atol=1e-15)


def test_gather_reproduces_linear_field(oracle):
    n = (8, 8, 8)
    nn = 512
    idx = np.arange(nn)
    pos = np.stack([(idx % 8) * H[0], (idx // 8 % 8) * H[1], (idx // 64) * H[2]])
    c0 = np.array([0.3, -0.2, 0.1])
    G = np.array([[0.5, -1.0, 0.25], [0.1, 0.2, -0.3], [-0.7, 0.05, 0.9]])
    F = c0[:, None] + G @ pos
    g = np.random.default_rng(13)
    # stay away from the periodic seam where the linear field jumps
    x = 0.2 + g.random((3, 100)) * 3.0
    out = oracle.gather(n, H, x, F)
    assert relerr(out, c0[:, None] + G @ x) < 1e-14


# ---------------------------------------------------------------------------
# Eq. 2: the rotation matrix solves the implicit velocity equation
# ---------------------------------------------------------------------------

def test_alpha_solves_implicit_equation(oracle):
    g = np.random.default_rng(14)
    for _ in range(50):
        B = g.standard_normal(3)
        beta = g.standard_normal()
        a = oracle.alpha(B, beta)
        assert relerr(a, alpha_by_solve(B, beta)) < 1e-14
        u = g.standard_normal(3)
        vb = a @ u
        assert np.max(np.abs(vb - beta * np.cross(vb, B) - u)) < 1e-14
        # parallel direction is left unchanged
        bh = B / np.linalg.norm(B)
        assert np.max(np.abs(a @ bh - bh)) < 1e-14


# ---------------------------------------------------------------------------
# P1: exact gyration of a lone particle (mover, Eqs. 4, 5, 8)
# ---------------------------------------------------------------------------

def _rot_z(v, ang):
    c, s = math.cos(ang), math.sin(ang)
    return np.array([c * v[0] - s * v[1], s * v[0] + c * v[1], v[2]])


@pytest.mark.parametrize("qom", [-1.0, 1.0 / 25.0])
def test_gyration_closed_form(oracle, inputs, qom):
    p = inputs.single_particle(qom=qom, v=(0.03, -0.02, 0.01))
    s = p.species[0]
    BN = oracle.centres_to_nodes(p.n, p.B_C)
    x, v = s.x.copy(), s.v.copy()
    beta = qom * p.dt / 2
    Bz = 0.2
    phi = 2.0 * math.atan(beta * Bz)
    nsteps = 1000
    xs = []
    for _ in range(nsteps):
        x, v = oracle.move(p.n, p.h, p.dt, x, v, qom, p.E, BN)
        xs.append(x[:, 0].copy())
    v0 = s.v[:, 0]
    # v_perp rotates by -phi per step about z; |v| and v_par are invariant
    v_exact = _rot_z(v0, -nsteps * phi)
    assert np.max(np.abs(v[:, 0] - v_exact)) / np.linalg.norm(v0) < 1e-12
    assert abs(np.linalg.norm(v[:, 0]) - np.linalg.norm(v0)) / np.linalg.norm(v0) < 1e-12
    # position: x^N = x^0 + dt sum_{k=1..N} v^k with v^k = R(-k phi) v^0
    z = complex(v0[0], v0[1])
    rot = complex(math.cos(-phi), math.sin(-phi))
    geo = rot * (1 - rot ** nsteps) / (1 - rot)
    disp = p.dt * z * geo
    L = p.L
    x_exact = np.array([s.x[0, 0] + disp.real, s.x[1, 0] + disp.imag, s.x[2, 0] + p.dt * nsteps * v0[2]])
    assert periodic_relerr(x, x_exact[:, None], L) < 1e-12
    # every position lies on the circle of radius dt |v_perp| / (2 sin(phi/2))
    xs = np.array(xs)
    r = p.dt * abs(z) / (2 * abs(math.sin(phi / 2)))
    # centre: mean of a full number of turns is not available; fit from 3 points
    c = _circumcentre(xs[0, :2], xs[1, :2], xs[2, :2])
    rr = np.hypot(xs[:50, 0] - c[0], xs[:50, 1] - c[1])
    assert np.max(np.abs(rr - r)) / r < 1e-10


def _circumcentre(a, b, c):
    d = 2 * (a[0] * (b[1] - c[1]) + b[0] * (c[1] - a[1]) + c[0] * (a[1] - b[1]))
    ux = ((a @ a) * (b[1] - c[1]) + (b @ b) * (c[1] - a[1]) + (c @ c) * (a[1] - b[1])) / d
    uy = ((a @ a) * (c[0] - b[0]) + (b @ b) * (a[0] - c[0]) + (c @ c) * (b[0] - a[0])) / d
    return np.array([ux, uy])


def test_exb_drift_and_parallel_acceleration(oracle, inputs):
    qom = -1.0
    e = (0.004, -0.003, 0.002)   # perpendicular part drives E x B, parallel part accelerates
    p = inputs.single_particle(qom=qom, v=(0.02, 0.01, -0.01), e=e)
    BN = oracle.centres_to_nodes(p.n, p.B_C)
    x, v = p.species[0].x.copy(), p.species[0].v.copy()
    beta = qom * p.dt / 2
    B = np.array([0.0, 0.0, 0.2])
    E = np.array(e)
    vd = np.cross(E, B) / (B @ B)            # E_perp x B / |B|^2
    phi = 2 * math.atan(beta * 0.2)
    n = 200
    for _ in range(n):
        x, v = oracle.move(p.n, p.h, p.dt, x, v, qom, p.E, BN)
    v0 = p.species[0].v[:, 0]
    w0 = v0 - vd
    w0[2] = 0.0
    exact = vd + _rot_z(w0, -n * phi)
    exact[2] = v0[2] + n * qom * p.dt * E[2]
    assert np.max(np.abs(v[:, 0] - exact)) / np.linalg.norm(v0) < 1e-12


# ---------------------------------------------------------------------------
# P3: J-hat (Eq. 1): sum rule and the B = 0 textbook deposit
# ---------------------------------------------------------------------------

def _small_plasma(inputs, n=(4, 3, 5), ppc=6, seed=3, bscale=0.2):
    p = inputs.uniform_plasma(50 + seed, n, ppc)
    nn = p.nn
    BN = inputs.random_node_field(nn, 100 + seed, scale=bscale, mean=(0.05, -0.1, 0.2))
    return p, BN


def test_current_sum_rule(oracle, inputs):
    p, BN = _small_plasma(inputs)
    V = np.prod(p.h)
    for s in p.species:
        J, _ = oracle.moments(p.n, p.h, p.dt, s.x, s.v, s.q, s.qom, BN)
        Bp = oracle.gather(p.n, p.h, s.x, BN)
        beta = s.qom * p.dt / 2
        tot = np.zeros(3)
        for i in range(s.np):
            tot += s.q[i] * alpha_by_solve(Bp[:, i], beta) @ s.v[:, i]
        assert relerr(V * J.sum(axis=1), tot) < 1e-12


def test_current_b0_is_textbook_cic(oracle, inputs):
    p, _ = _small_plasma(inputs)
    BN = np.zeros((3, p.nn))
    V = np.prod(p.h)
    s = p.species[0]
    J, _ = oracle.moments(p.n, p.h, p.dt, s.x, s.v, s.q, s.qom, BN)
    nodes, w = cic_nodes_weights(s.x, p.n, p.h)
    ref = np.zeros((3, p.nn))
    for c in range(3):
        np.add.at(ref[c], nodes.ravel(), (w * (s.q * s.v[c])[:, None]).ravel() / V)
    assert relerr(J, ref) < 1e-13


# ---------------------------------------------------------------------------
# P4, P5, P9: mass matrices (Eq. 3)
# ---------------------------------------------------------------------------

def _opp(k27):
    ox, oy, oz = k27 % 3 - 1, k27 // 3 % 3 - 1, k27 // 9 - 1
    return (-ox + 1) + 3 * (-oy + 1) + 9 * (-oz + 1), (ox, oy, oz)


def _shift(n, ox, oy, oz):
    nn = n[0] * n[1] * n[2]
    idx = np.arange(nn)
    gx, gy, gz = idx % n[0], idx // n[0] % n[1], idx // (n[0] * n[1])
    return ((gx + ox) % n[0]) + n[0] * (((gy + oy) % n[1]) + n[1] * ((gz + oz) % n[2]))


def test_mass_matrix_symmetry_not_transposed(oracle, inputs):
    """M_{N N'} = M_{N' N} as identical 3x3 blocks (Eq. 3 and the text after it)."""
    p, BN = _small_plasma(inputs)
    _, M = oracle.species_moments(p, [s.x for s in p.species], [s.v for s in p.species], BN)
    scale = np.max(np.abs(M))
    worst_T = 0.0
    for k in range(27):
        ko, (ox, oy, oz) = _opp(k)
        nb = _shift(p.n, ox, oy, oz)
        # M27[g][o] == M27[g+o][-o]
        assert np.max(np.abs(M[k] - M[ko][:, nb])) / scale < 1e-15
        # and not, in general, its transpose (B != 0 gives alpha an antisymmetric part)
        Mt = M[ko][:, nb].reshape(3, 3, -1).transpose(1, 0, 2).reshape(9, -1)
        worst_T = max(worst_T, np.max(np.abs(M[k] - Mt)) / scale)
    assert worst_T > 1e-4


def test_mass_matrix_reversed_B_is_transpose(oracle, inputs):
    p, BN = _small_plasma(inputs)
    xs = [s.x for s in p.species]
    vs = [s.v for s in p.species]
    _, Mp = oracle.species_moments(p, xs, vs, BN)
    _, Mm = oracle.species_moments(p, xs, vs, -BN)
    MmT = Mm.reshape(27, 3, 3, -1).transpose(0, 2, 1, 3).reshape(27, 9, -1)
    assert relerr(Mp, MmT) < 1e-14


def test_mass_matrix_B0_is_isotropic(oracle, inputs):
    p, _ = _small_plasma(inputs)
    BN = np.zeros((3, p.nn))
    _, M = oracle.species_moments(p, [s.x for s in p.species], [s.v for s in p.species], BN)
    Mb = M.reshape(27, 3, 3, -1)
    scale = np.max(np.abs(M))
    for i in range(3):
        for j in range(3):
            if i != j:
                assert np.max(np.abs(Mb[:, i, j])) / scale < 1e-16
    assert np.max(np.abs(Mb[:, 0, 0] - Mb[:, 1, 1])) / scale < 1e-15
    assert np.max(np.abs(Mb[:, 0, 0] - Mb[:, 2, 2])) / scale < 1e-15


def test_single_particle_blocks_closed_form(oracle, inputs):
    n = (4, 4, 4)
    h = H
    x = np.array([[1.13], [0.41], [1.77]])
    v = np.array([[0.01], [0.02], [-0.03]])
    q, qom = -2e-3, -1.0
    BN = inputs.random_node_field(64, 5, scale=0.1, mean=(0, 0, 0.2))
    J, M = oracle.moments(n, h, DT, x, v, np.array([q]), qom, BN)
    nodes, w = cic_nodes_weights(x, n, h)
    Bp = sum(w[0, a] * BN[:, nodes[0, a]] for a in range(8))
    beta = qom * DT / 2
    al = alpha_by_solve(Bp, beta)
    V = np.prod(h)
    ref = np.zeros_like(M)
    for a in range(8):
        for b in range(8):
            da = np.array([a & 1, (a >> 1) & 1, (a >> 2) & 1])
            db = np.array([b & 1, (b >> 1) & 1, (b >> 2) & 1])
            o = db - da
            k = (o[0] + 1) + 3 * (o[1] + 1) + 9 * (o[2] + 1)
            ref[k, :, nodes[0, a]] += (q * beta / V) * w[0, a] * w[0, b] * al.ravel()
    assert relerr(M, ref) < 1e-14


def test_row_sum_rule(oracle, inputs):
    p, BN = _small_plasma(inputs)
    V = np.prod(p.h)
    _, M = oracle.species_moments(p, [s.x for s in p.species], [s.v for s in p.species], BN)
    lhs = V * M.sum(axis=0)      # (9, Nn)
    rhs = np.zeros_like(lhs)
    for s in p.species:
        nodes, w = cic_nodes_weights(s.x, p.n, p.h)
        Bp = np.einsum("pa,cpa->cp", w, BN[:, nodes])
        beta = s.qom * p.dt / 2
        for i in range(s.np):
            al = alpha_by_solve(Bp[:, i], beta).ravel()
            for a in range(8):
                rhs[:, nodes[i, a]] += s.q[i] * beta * w[i, a] * al
    assert relerr(lhs, rhs) < 1e-13


def test_mass_operator_positive_semidefinite(oracle, inputs):
    p, BN = _small_plasma(inputs)
    _, M = oracle.species_moments(p, [s.x for s in p.species], [s.v for s in p.species], BN)
    g = np.random.default_rng(7)
    for _ in range(20):
        E = g.standard_normal((3, p.nn))
        y = oracle.mass_apply27(p.n, M, E)
        assert float(np.sum(E * y)) >= -1e-15 * float(np.sum(E * E)) * np.max(np.abs(M))


# ---------------------------------------------------------------------------
# P6: dense brute force on 2x2x2 and 3x3x3 periodic grids
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [(2, 2, 2), (3, 3, 3), (2, 3, 4)])
def test_dense_brute_force_apply(oracle, inputs, n):
    p = inputs.uniform_plasma(60, n, 5)
    nn = p.nn
    BN = inputs.random_node_field(nn, 61, scale=0.2, mean=(0.0, 0.1, 0.2))
    _, M27 = oracle.species_moments(p, [s.x for s in p.species], [s.v for s in p.species], BN)
    V = np.prod(p.h)
    dense = np.zeros((3 * nn, 3 * nn))
    for s in p.species:
        nodes, w = cic_nodes_weights(s.x, p.n, p.h)
        Bp = np.einsum("pa,cpa->cp", w, BN[:, nodes])
        beta = s.qom * p.dt / 2
        for i in range(s.np):
            al = alpha_by_solve(Bp[:, i], beta)
            for a in range(8):
                for b in range(8):
                    ga, gb = nodes[i, a], nodes[i, b]
                    for ci in range(3):
                        for cj in range(3):
                            dense[ci * nn + ga, cj * nn + gb] += s.q[i] * beta / V * w[i, a] * w[i, b] * al[ci, cj]
    cols = np.zeros((3 * nn, 3 * nn))
    for j in range(3 * nn):
        e = np.zeros(3 * nn)
        e[j] = 1.0
        cols[:, j] = oracle.mass_apply27(p.n, M27, e.reshape(3, nn)).ravel()
    assert relerr(cols, dense) < 1e-13


# ---------------------------------------------------------------------------
# P7: mover-moment consistency  (1/V) sum q W vbar = J + M E
# ---------------------------------------------------------------------------

def test_vbar_deposit_equals_current_plus_mass_apply(oracle, inputs):
    p, BN = _small_plasma(inputs, n=(5, 4, 4), ppc=8)
    E = inputs.random_node_field(p.nn, 77, scale=0.01)
    xs = [s.x for s in p.species]
    vs = [s.v for s in p.species]
    J, M27 = oracle.species_moments(p, xs, vs, BN)
    lhs = J + oracle.mass_apply27(p.n, M27, E)
    V = np.prod(p.h)
    rhs = np.zeros((3, p.nn))
    for s in p.species:
        _, v1 = oracle.move(p.n, p.h, p.dt, s.x, s.v, s.qom, E, BN)
        vbar = 0.5 * (v1 + s.v)
        nodes, w = cic_nodes_weights(s.x, p.n, p.h)
        for c in range(3):
            np.add.at(rhs[c], nodes.ravel(), (w * (s.q * vbar[c])[:, None]).ravel() / V)
    assert relerr(lhs, rhs) < 1e-12


# ---------------------------------------------------------------------------
# P11: staggered curls
# ---------------------------------------------------------------------------

def test_curl_adjointness(oracle, inputs):
    n = (5, 4, 6)
    g = np.random.default_rng(21)
    for _ in range(5):
        E = g.standard_normal((3, 120))
        B = g.standard_normal((3, 120))
        lhs = np.sum(oracle.curl_C(n, H, E) * B)
        rhs = np.sum(E * oracle.curl_N(n, H, B))
        assert abs(lhs - rhs) <= 1e-13 * (abs(lhs) + np.sum(np.abs(E)) + np.sum(np.abs(B)))


def test_curl_of_plane_wave_closed_form(oracle):
    """E = (0, 0, sin kx): curl_C E at centres = (0, -k cos(k x_c) * sinc, 0) exactly."""
    n = (16, 4, 4)
    h = (0.5, 0.5, 0.5)
    k = 2 * math.pi / (n[0] * h[0])
    idx = np.arange(np.prod(n))
    gx = idx % n[0]
    E = np.zeros((3, idx.size))
    E[2] = np.sin(k * gx * h[0])
    cc = oracle.curl_C(n, h, E)
    xc = (gx + 0.5) * h[0]
    sinc = math.sin(k * h[0] / 2) / (k * h[0] / 2)
    assert np.max(np.abs(cc[0])) < 1e-14
    assert np.max(np.abs(cc[2])) < 1e-14
    assert np.max(np.abs(cc[1] - (-k * np.cos(k * xc) * sinc))) < 1e-13
    # node curl of B = (0, sin k x_c, 0) at centres: curl_N B = (0, 0, k cos(k x_g) sinc)
    B = np.zeros((3, idx.size))
    B[1] = np.sin(k * xc)
    cn = oracle.curl_N(n, h, B)
    assert np.max(np.abs(cn[2] - k * np.cos(k * gx * h[0]) * sinc)) < 1e-13
    assert np.max(np.abs(cn[:2])) < 1e-14


def test_centres_to_nodes_average(oracle):
    n = (3, 4, 5)
    g = np.random.default_rng(3)
    BC = g.standard_normal((3, 60))
    BN = oracle.centres_to_nodes(n, BC)
    ref = np.zeros_like(BC)
    for a in range(8):
        ox, oy, oz = -(a & 1), -((a >> 1) & 1), -((a >> 2) & 1)
        ref += BC[:, _shift(n, ox, oy, oz)] / 8
    assert relerr(BN, ref) < 1e-15


# ---------------------------------------------------------------------------
# P12: GMRES against a dense library solve
# ---------------------------------------------------------------------------

def test_gmres_matches_dense_solve(oracle, inputs):
    p = inputs.uniform_plasma(70, (3, 2, 4), 6)
    BN = inputs.random_node_field(p.nn, 71, scale=0.1, mean=(0, 0, 0.2))
    J, M27 = oracle.species_moments(p, [s.x for s in p.species], [s.v for s in p.species], BN)
    En = inputs.random_node_field(p.nn, 72, scale=1e-3)
    BC = inputs.random_node_field(p.nn, 73, scale=1e-3, mean=(0, 0, 0.2))
    sol = oracle.field_solve(p.n, p.h, p.dt, M27, J, En, BC, tol=1e-13)
    n3 = 3 * p.nn
    A = np.zeros((n3, n3))
    for j in range(n3):
        e = np.zeros(n3)
        e[j] = 1.0
        A[:, j] = oracle.field_operator(p.n, p.h, p.dt, M27, e.reshape(3, -1)).ravel()
    b = oracle.field_rhs(p.n, p.h, p.dt, J, En, BC).ravel()
    ref = np.linalg.solve(A, b)
    assert sol["iters"] > 0
    assert relerr(sol["E_theta"].ravel(), ref) < 1e-11
    # the operator itself: identity + (c theta dt)^2 curl curl + 4 pi theta dt M
    CC = np.zeros((n3, n3))
    MM = np.zeros((n3, n3))
    for j in range(n3):
        e = np.zeros(n3)
        e[j] = 1.0
        CC[:, j] = oracle.curl_N(p.n, p.h, oracle.curl_C(p.n, p.h, e.reshape(3, -1))).ravel()
        MM[:, j] = oracle.mass_apply27(p.n, M27, e.reshape(3, -1)).ravel()
    th = 0.5
    assert relerr(A, np.eye(n3) + (th * p.dt) ** 2 * CC + 4 * math.pi * th * p.dt * MM) < 1e-14
    # curl curl is symmetric positive semidefinite (curl_N = curl_C^T)
    assert relerr(CC, CC.T) < 1e-14


# ---------------------------------------------------------------------------
# P8: energy conservation with theta = 1/2 (Sec. I and Sec. II)
# ---------------------------------------------------------------------------

def test_energy_conservation_small_workload(oracle, inputs):
    p = inputs.config0()
    _, hist = oracle.run_steps(p, 10, tol=1e-10)
    e0 = hist[0]["total"]
    drift = max(abs(h["total"] - e0) / e0 for h in hist)
    assert drift <= 1e-10
    # initial magnetic energy follows from the workload's definition: V_box B0^2 / (8 pi)
    vol = 64.0
    assert abs(hist[0]["WB"] - vol / (8 * math.pi) * 0.2 ** 2) < 1e-14
    # the field did work: kinetic and field energy both changed by far more than the drift
    assert abs(hist[-1]["K"] - hist[0]["K"]) > 1e-6 * e0
    assert all(h["iters"] > 0 for h in hist[1:])


def test_energy_not_conserved_with_inconsistent_mover(oracle, inputs):
    """Sensitivity of the energy pin: moving with an electric field that differs
    by 1% from the implicit solution breaks conservation far above rounding."""
    p = inputs.config0()
    x = [s.x.copy() for s in p.species]
    v = [s.v.copy() for s in p.species]
    E, BC = p.E.copy(), p.B_C.copy()
    K0, WE0, WB0 = oracle.total_energy(p, v, E, BC)
    BN = oracle.centres_to_nodes(p.n, BC)
    J, M27 = oracle.species_moments(p, x, v, BN)
    sol = oracle.field_solve(p.n, p.h, p.dt, M27, J, E, BC)
    for i, s in enumerate(p.species):
        x[i], v[i] = oracle.move(p.n, p.h, p.dt, x[i], v[i], s.qom, sol["E_theta"] * 1.01, BN)
    K1, WE1, WB1 = oracle.total_energy(p, v, sol["E_next"], sol["BC_next"])
    # the work done on the particles no longer matches the field energy change
    e0 = K0 + WE0 + WB0
    assert abs(K1 + WE1 + WB1 - e0) / e0 > 1e-9


# ---------------------------------------------------------------------------
# Reference gradient: dual numbers against central differences of the
# per-particle loss, and the per-particle loss against the moments
# ---------------------------------------------------------------------------

def _grad_case(inputs, n=(4, 4, 3), ppc=3):
    p = inputs.uniform_plasma(80, n, ppc)
    g = np.random.default_rng(81)
    E = 1e-2 * g.standard_normal((3, p.nn))
    BN = 0.05 * g.standard_normal((3, p.nn)) + np.array([[0.0], [0.05], [0.2]])
    gJ = g.standard_normal((3, p.nn))
    gM = g.standard_normal((14, 9, p.nn))
    return p, E, BN, gJ, gM


def test_particle_loss_matches_moments(oracle, inputs):
    p, E, BN, gJ, gM = _grad_case(inputs)
    tot = 0.0
    J = np.zeros((3, p.nn))
    M27 = np.zeros((27, 9, p.nn))
    for s in p.species:
        x1, v1 = oracle.move(p.n, p.h, p.dt, s.x, s.v, s.qom, E, BN)
        oracle.moments(p.n, p.h, p.dt, x1, v1, s.q, s.qom, BN, J, M27)
        tot += oracle.particle_loss(p.n, p.h, p.dt, s.x, s.v, s.q, s.qom, E, BN, gJ, gM).sum()
    L = np.sum(gJ * J) + np.sum(gM * oracle.m14(p.n, M27))
    assert abs(L - tot) <= 1e-12 * (abs(L) + 1e-30)


def test_dual_gradient_matches_central_differences(oracle, inputs):
    p, E, BN, gJ, gM = _grad_case(inputs)
    s = p.species[0]
    gx, gv, gE, gB = oracle.grad(p.n, p.h, p.dt, s.x, s.v, s.q, s.qom, E, BN, gJ, gM)
    eps = 1e-6

    def lp(x, v, E_, B_):
        return oracle.particle_loss(p.n, p.h, p.dt, x, v, s.q, s.qom, E_, B_, gJ, gM)

    # particle inputs: per-particle loss differences
    for c in range(3):
        for arr, gref in ((s.x, gx), (s.v, gv)):
            up = arr.copy(); up[c] += eps
            dn = arr.copy(); dn[c] -= eps
            if arr is s.x:
                fd = (lp(up, s.v, E, BN) - lp(dn, s.v, E, BN)) / (2 * eps)
            else:
                fd = (lp(s.x, up, E, BN) - lp(s.x, dn, E, BN)) / (2 * eps)
            assert relerr(gref[c], fd) < 1e-6
    # grid inputs: a few nodes, summed over the particles of the species
    g = np.random.default_rng(9)
    for node in g.choice(p.nn, 6, replace=False):
        for c in range(3):
            for F, gref in ((E, gE), (BN, gB)):
                up = F.copy(); up[c, node] += eps
                dn = F.copy(); dn[c, node] -= eps
                if F is E:
                    fd = (lp(s.x, s.v, up, BN) - lp(s.x, s.v, dn, BN)).sum() / (2 * eps)
                else:
                    fd = (lp(s.x, s.v, E, up) - lp(s.x, s.v, E, dn)).sum() / (2 * eps)
                assert abs(gref[c, node] - fd) <= 1e-6 * max(np.max(np.abs(gref)), 1e-30)


def test_threaded_particle_pass_matches_serial(oracle, inputs):
    """The host-threaded particle pass (the CPU baseline's form: mover, then the
    moments at the moved positions, thread-private grids added in thread
    order) is the serial mover followed by the serial moments: positions and
    velocities bit for bit, J and M to rounding of the changed summation
    order, and bit for bit on one thread."""
    p = inputs.uniform_plasma(7, (6, 5, 4), 9)
    rng = np.random.default_rng(11)
    En = 1e-2 * rng.standard_normal((3, p.nn))
    BN = np.array([[0.02], [0.0], [0.2]]) + 0.05 * rng.standard_normal((3, p.nn))
    Bn = BN + 0.01 * rng.standard_normal((3, p.nn))
    for s in p.species:
        x1, v1 = oracle.move(p.n, p.h, p.dt, s.x, s.v, s.qom, En, BN)
        J, M27 = oracle.moments(p.n, p.h, p.dt, x1, v1, s.q, s.qom, Bn)
        for th in (1, 3, 4):
            x2, v2, J2, M2, used = oracle.move_moments_threads(p.n, p.h, p.dt, s.x, s.v, s.q, s.qom, En, BN, Bn,
                                                               threads=th)
            assert used == th
            assert np.array_equal(x1, x2) and np.array_equal(v1, v2)
            if th == 1:
                assert np.array_equal(J, J2) and np.array_equal(M27, M2)
            assert relerr(J2, J) < 1e-14
            assert relerr(M2, M27) < 1e-14


def test_threaded_step_loop_matches_step_loop(oracle, inputs):
    """The step loop with the threaded particle pass reaches the same state as
    the plain step loop (moments -> solve -> mover), to rounding, and also
    conserves the energy."""
    p = inputs.config0()
    ref, hist = oracle.run_steps(p, 3)
    out, hist_t, used = oracle.run_steps_threads(p, 3, threads=4)
    assert used == 4
    for a, b in zip(ref["v"], out["v"]):
        assert relerr(b, a) < 1e-12
    assert relerr(out["E"], ref["E"]) < 1e-9
    e0 = hist[0]["total"]
    assert max(abs(h["total"] - e0) for h in hist_t) / e0 < 1e-10
