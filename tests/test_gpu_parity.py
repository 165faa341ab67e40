"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

Tolerances (relative max-norm over each output array): 1e-12 for the FP64
path and 1e-5 for the FP32 path. Atomic accumulation order makes the
results non-deterministic at the rounding level, so bit-exactness is not
asked for; FP32 inputs are compared against the oracle fed the same FP32
values widened exactly to FP64.
"""
import dataclasses

import numpy as np
import pytest

from tests.gpu_common import (dev, fp32_drift_bound, host, kinetic0, need_gpu, periodic_rel, rel, round32,
                              say, torch)

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


@pytest.fixture(scope="module")
def E():
    need_gpu()
    from paper_2603_16624_amd import ecsim
    ecsim.lib()
    return ecsim


@pytest.fixture(scope="module")
def O():
    from oracle import oracle
    oracle.lib()
    return oracle


@pytest.fixture(scope="module")
def I():
    from paper_2603_16624_amd import inputs
    return inputs


CASES = [((5, 4, 3), 7), ((2, 2, 2), 5), ((1, 3, 2), 6), ((8, 8, 8), 27), ((13, 7, 5), 3)]


def make_case(I, n, ppc, seed):
    p = I.uniform_plasma(200 + seed, n, ppc)
    rng = np.random.default_rng(300 + seed)
    En = 1e-2 * rng.standard_normal((3, p.nn))
    BN = np.array([[0.02], [-0.03], [0.2]]) + 0.05 * rng.standard_normal((3, p.nn))
    return p, En, BN


# ---------------------------------------------------------------------------
# mover
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,ppc", CASES)
def test_move_f64(E, O, I, n, ppc):
    say("move f64", n, ppc)
    p, En, BN = make_case(I, n, ppc, 1)
    grid = E.Grid(p.n, p.h, p.dt)
    for s in p.species:
        sp = E.Species.from_f64(s.qom, s.x, s.v, s.q)
        E.move(grid, sp, dev(En), dev(BN))
        xo, vo = O.move(p.n, p.h, p.dt, s.x, s.v, s.qom, En, BN)
        assert rel(host(sp.vel), vo) < TOL64
        assert periodic_rel(host(sp.pos), xo, p.L) < TOL64


@pytest.mark.parametrize("n,ppc", CASES)
def test_move_f32(E, O, I, n, ppc):
    say("move f32", n, ppc)
    p, En, BN = make_case(I, n, ppc, 2)
    grid = E.Grid(p.n, p.h, p.dt)
    for s, f in zip(p.species, I.to_f32_state(p)):
        sp = E.Species.from_f32(s.qom, f["cell"], f["off"], f["v"], f["q"])
        E.move(grid, sp, dev(En, torch.float32), dev(BN, torch.float32))
        xo, vo = O.move(p.n, p.h, p.dt, f["x64"], f["v64"], s.qom, round32(En), round32(BN))
        assert rel(host(sp.vel), vo) < TOL32
        x32 = I.decode_f32(host(sp.cell), host(sp.pos), p.n, p.h)
        assert periodic_rel(x32, xo, p.L) < TOL32
        off = host(sp.pos)
        assert np.all((off >= 0) & (off < 1))


def test_move_kinetic_energy_and_edge_positions(E, O, I):
    """Particles exactly on node planes and crossing the periodic boundary."""
    say("move edges")
    n = (4, 3, 5)
    h = (0.5, 0.5, 0.5)
    L = [n[d] * h[d] for d in range(3)]
    x = np.array([[0.0, 0.5, L[0] - 1e-9, 1.0, L[0] - 0.01],
                  [0.0, 1.0, 0.7, L[1] - 1e-12, 0.01],
                  [0.0, 2.0, 1.1, 0.25, L[2] - 0.001]])
    v = np.array([[0.01, -0.3, 0.5, -0.2, 0.4],
                  [0.02, 0.1, -0.4, 0.3, -0.3],
                  [-0.03, 0.2, 0.1, -0.5, 0.2]])
    q = np.array([1e-3, 2e-3, -1e-3, 5e-4, 3e-3])
    rng = np.random.default_rng(5)
    nn = int(np.prod(n))
    En = 1e-2 * rng.standard_normal((3, nn))
    BN = 0.1 * rng.standard_normal((3, nn))
    grid = E.Grid(n, h, 0.1)
    sp = E.Species.from_f64(-1.0, x, v, q)
    ke = torch.zeros(1, dtype=torch.float64, device="cuda")
    E.move(grid, sp, dev(En), dev(BN), ke)
    xo, vo = O.move(n, h, 0.1, x, v, -1.0, En, BN)
    assert rel(host(sp.vel), vo) < TOL64
    assert periodic_rel(host(sp.pos), xo, L) < TOL64
    assert np.all((host(sp.pos) >= 0) & (host(sp.pos) < np.array(L)[:, None]))
    assert abs(host(ke)[0] - O.kinetic(vo, q, -1.0)) <= 1e-14 * abs(O.kinetic(vo, q, -1.0))


def test_empty_species(E, I):
    say("empty species")
    grid = E.Grid((3, 3, 3), (0.5,) * 3, 0.1)
    sp = E.Species.from_f64(-1.0, np.zeros((3, 0)), np.zeros((3, 0)), 1.0)
    B = torch.zeros((3, 27), dtype=torch.float64, device="cuda")
    E.move(grid, sp, B, B)
    J = torch.ones((3, 27), dtype=torch.float64, device="cuda")
    M = torch.ones((14, 9, 27), dtype=torch.float64, device="cuda")
    E.moments(grid, [sp], B, J, M)
    assert np.all(host(J) == 0) and np.all(host(M) == 0)


# ---------------------------------------------------------------------------
# moments
# ---------------------------------------------------------------------------

def oracle_moments(O, p, xs, vs, qs, BN):
    J = np.zeros((3, p.nn))
    M27 = np.zeros((27, 9, p.nn))
    for s, x, v, q in zip(p.species, xs, vs, qs):
        O.moments(p.n, p.h, p.dt, x, v, q, s.qom, BN, J, M27)
    return J, O.m14(p.n, M27)


@pytest.mark.parametrize("n,ppc", CASES)
def test_moments_f64_any_order(E, O, I, n, ppc):
    say("moments f64 atomic", n, ppc)
    p, _, BN = make_case(I, n, ppc, 3)
    grid = E.Grid(p.n, p.h, p.dt)
    sp = [E.Species.from_f64(s.qom, s.x, s.v, s.q) for s in p.species]
    J = torch.empty((3, p.nn), dtype=torch.float64, device="cuda")
    M = torch.empty((14, 9, p.nn), dtype=torch.float64, device="cuda")
    E.moments(grid, sp, dev(BN), J, M)
    Jo, Mo = oracle_moments(O, p, [s.x for s in p.species], [s.v for s in p.species], [s.q for s in p.species], BN)
    assert rel(host(J), Jo) < TOL64
    assert rel(host(M), Mo) < TOL64


@pytest.mark.parametrize("n,ppc", CASES)
def test_moments_f32_any_order(E, O, I, n, ppc):
    say("moments f32 atomic", n, ppc)
    p, _, BN = make_case(I, n, ppc, 4)
    grid = E.Grid(p.n, p.h, p.dt)
    st = I.to_f32_state(p)
    sp = [E.Species.from_f32(s.qom, f["cell"], f["off"], f["v"], f["q"]) for s, f in zip(p.species, st)]
    J = torch.empty((3, p.nn), dtype=torch.float32, device="cuda")
    M = torch.empty((14, 9, p.nn), dtype=torch.float32, device="cuda")
    E.moments(grid, sp, dev(BN, torch.float32), J, M)
    Jo, Mo = oracle_moments(O, p, [f["x64"] for f in st], [f["v64"] for f in st], [f["q64"] for f in st],
                            round32(BN))
    assert rel(host(J), Jo) < TOL32
    assert rel(host(M), Mo) < TOL32


def sorted_species(E, grid, sp, perms=None):
    out = []
    for s in sp:
        d = s.empty_like()
        cs = torch.empty(grid.nn + 1, dtype=torch.int32, device="cuda")
        perm = torch.empty(max(s.np, 1), dtype=torch.int32, device="cuda")
        E.sort(grid, s, d, cs, perm[: s.np] if s.np else None)
        if perms is not None:
            perms.append(host(perm)[: s.np].astype(np.int64))
        out.append(d)
    return out


@pytest.mark.parametrize("n,ppc", CASES + [((16, 8, 4), 40), ((4, 4, 4), 130)])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_moments_sorted_tiled(E, O, I, n, ppc, prec):
    """The tiled LDS deposit over cell-sorted particles (cells with > 64 particles included)."""
    say("moments tiled", prec, n, ppc)
    p, _, BN = make_case(I, n, ppc, 16)
    grid = E.Grid(p.n, p.h, p.dt)
    if prec == "f64":
        sp = [E.Species.from_f64(s.qom, s.x, s.v, s.q) for s in p.species]
        xs, vs, qs, B = [s.x for s in p.species], [s.v for s in p.species], [s.q for s in p.species], BN
        tdt, tol = torch.float64, TOL64
    else:
        st = I.to_f32_state(p)
        sp = [E.Species.from_f32(s.qom, f["cell"], f["off"], f["v"], f["q"]) for s, f in zip(p.species, st)]
        xs, vs, qs, B = [f["x64"] for f in st], [f["v64"] for f in st], [f["q64"] for f in st], round32(BN)
        tdt, tol = torch.float32, TOL32
    sp = sorted_species(E, grid, sp)
    J = torch.full((3, p.nn), 7.0, dtype=tdt, device="cuda")
    M = torch.full((14, 9, p.nn), 7.0, dtype=tdt, device="cuda")
    E.moments(grid, sp, dev(B, tdt), J, M, flags=E.SORTED)
    Jo, Mo = oracle_moments(O, p, xs, vs, qs, B)
    assert rel(host(J), Jo) < tol
    assert rel(host(M), Mo) < tol


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_moments_tiled_node_plane_positions(E, O, I, prec):
    """The tiled deposit with particles exactly on node planes (weights exactly
    0 and 1, so class-weight factors vanish), just below the next plane, and
    on the periodic boundary, more than 64 to a cell."""
    import types
    say("moments tiled, node-plane positions", prec)
    n, h, dt = (4, 3, 5), (0.5, 0.25, 0.4), 0.1
    nn = int(np.prod(n))
    rng = np.random.default_rng(21)
    npart = 300
    cells = np.stack([rng.integers(0, n[d], npart) for d in range(3)])
    cells[:, :100] = np.array([[1], [2], [3]])   # 100 particles in one cell
    frac = rng.random((3, npart))
    pick = rng.integers(0, 4, (3, npart))
    frac = np.where(pick == 0, 0.0, np.where(pick == 1, 1.0 - 2.0 ** -30, frac))
    v = 0.3 * rng.standard_normal((3, npart))
    q = 1e-3 * (1.0 + rng.random(npart))
    B = np.array([[0.02], [-0.03], [0.2]]) + 0.05 * rng.standard_normal((3, nn))
    grid = E.Grid(n, h, dt)
    if prec == "f64":
        x = (cells + frac) * np.array(h)[:, None]
        sp = E.Species.from_f64(-1.0, x, v, q)
        tdt, tol, Bo = torch.float64, TOL64, B
    else:
        off = frac.astype(np.float32)
        off = np.where(off >= 1.0, np.float32(1.0) - np.finfo(np.float32).epsneg, off).astype(np.float32)
        lin = (cells[0] + n[0] * (cells[1] + n[1] * cells[2])).astype(np.int32)
        v32, q32 = v.astype(np.float32), q.astype(np.float32)
        sp = E.Species.from_f32(-1.0, lin, off, v32, q32)
        x = (cells + off.astype(np.float64)) * np.array(h)[:, None]
        v, q = v32.astype(np.float64), q32.astype(np.float64)
        tdt, tol, Bo = torch.float32, TOL32, round32(B)
    sp = sorted_species(E, grid, [sp])
    J = torch.full((3, nn), 7.0, dtype=tdt, device="cuda")
    M = torch.full((14, 9, nn), 7.0, dtype=tdt, device="cuda")
    E.moments(grid, sp, dev(Bo, tdt), J, M, flags=E.SORTED)
    p = types.SimpleNamespace(n=n, h=h, dt=dt, nn=nn, species=[types.SimpleNamespace(qom=-1.0)])
    Jo, Mo = oracle_moments(O, p, [x], [v], [q], Bo)
    assert rel(host(J), Jo) < tol
    assert rel(host(M), Mo) < tol


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n,shift", [((9, 7, 6), (1, 2, 1)), ((8, 8, 4), (3, 1, 1)), ((10, 6, 1), (5, 3, 0))])
def test_deposit_invariant_under_brick_placement(E, O, I, prec, n, shift):
    """The tiled deposit does not depend on where the bricks of its
    workgroups, the cells of its wavefronts or their list packing fall: the
    plasma and the deposit field translated by whole cells (periodic; grids
    that are not multiples of the brick, so the bricks are clipped
    differently) give J and M translated by the same cells, within the parity
    tolerance (only the order of summation differs). In the FP32 form each
    particle keeps its in-cell offsets, so its record is bit for bit the same."""
    say("translation invariance", prec, n, shift)
    p, _, BN = make_case(I, n, 20, 41)
    grid = E.Grid(p.n, p.h, p.dt)
    nx, ny, nz = p.n

    def roll_nodes(F):
        a = np.asarray(F).reshape(F.shape[:-1] + (nz, ny, nx))
        a = np.roll(a, (shift[2], shift[1], shift[0]), axis=(-3, -2, -1))
        return a.reshape(F.shape)

    def deposit(xs_abs, B):
        if prec == "f64":
            sp = [E.Species.from_f64(s.qom, x, s.v, s.q) for s, x in zip(p.species, xs_abs)]
            tdt = torch.float64
        else:
            sp = []
            for s, x in zip(p.species, xs_abs):
                cell, off = I.encode_f32(x, p.n, p.h)
                sp.append(E.Species.from_f32(s.qom, cell, off, np.asarray(s.v, np.float32).astype(np.float64),
                                             np.asarray(s.q, np.float32).astype(np.float64) if np.ndim(s.q)
                                             else float(np.float32(s.q))))
            tdt = torch.float32
        sp = sorted_species(E, grid, sp)
        J = torch.empty((3, p.nn), dtype=tdt, device="cuda")
        M = torch.empty((14, 9, p.nn), dtype=tdt, device="cuda")
        E.moments(grid, sp, dev(B, tdt), J, M, flags=E.SORTED)
        return host(J), host(M)

    B = BN if prec == "f64" else round32(BN)
    xs = [s.x for s in p.species]
    J0, M0 = deposit(xs, B)
    L = np.asarray(p.L)[:, None]
    xs1 = [np.mod(x + np.asarray(shift)[:, None] * np.asarray(p.h)[:, None], L) for x in xs]
    J1, M1 = deposit(xs1, roll_nodes(B))
    tol = TOL64 if prec == "f64" else TOL32
    assert rel(J1, roll_nodes(J0)) < tol
    assert rel(M1, roll_nodes(M0)) < tol


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n,ppc,vscale", [((8, 8, 8), 27, 1.0), ((6, 5, 4), 9, 40.0), ((2, 3, 2), 7, 20.0),
                                           ((13, 7, 5), 3, 5.0), ((8, 6, 1), 12, 10.0), ((16, 1, 1), 20, 10.0),
                                           ((8, 4, 1), 300, 2.0), ((4, 4, 2), 150, 2.0)])
def test_move_moments_fused(E, O, I, prec, n, ppc, vscale):
    """Fused mover + deposit (two passes on one stale grouping) against the oracle's move then moments.

    Scaled velocities make many particles leave their cell (the stray path),
    some by more than one cell. The last two cases put 19,200 particles in one
    brick, more than the grouping pass maps position by position (8192), so
    it locates their ranges by binary search."""
    say("move+moments fused", prec, n, ppc, vscale)
    p, En, BN = make_case(I, n, ppc, 17)
    for s in p.species:
        s.v = s.v * vscale
    rng = np.random.default_rng(18)
    Bnext = BN + 0.01 * rng.standard_normal(BN.shape)
    grid = E.Grid(p.n, p.h, p.dt)
    if prec == "f64":
        sp = [E.Species.from_f64(s.qom, s.x, s.v, s.q) for s in p.species]
        xs, vs, qs = [s.x for s in p.species], [s.v for s in p.species], [s.q for s in p.species]
        Ec, Bc, Bnc = En, BN, Bnext
        tdt, tol = torch.float64, TOL64
    else:
        st = I.to_f32_state(p)
        sp = [E.Species.from_f32(s.qom, f["cell"], f["off"], f["v"], f["q"]) for s, f in zip(p.species, st)]
        xs, vs, qs = [f["x64"] for f in st], [f["v64"] for f in st], [f["q64"] for f in st]
        Ec, Bc, Bnc = round32(En), round32(BN), round32(Bnext)
        tdt, tol = torch.float32, TOL32
    perms = []
    sp = sorted_species(E, grid, sp, perms)
    J = torch.empty((3, p.nn), dtype=tdt, device="cuda")
    M = torch.empty((14, 9, p.nn), dtype=tdt, device="cuda")
    ke = torch.zeros(1, dtype=torch.float64, device="cuda")
    # the oracle follows every particle through the same two passes
    for it in range(2):
        E.move_moments(grid, sp, dev(Ec, tdt), dev(Bc, tdt), dev(Bnc, tdt), J, M, ke if it == 1 else None)
        x1s, v1s = [], []
        for s, x, v in zip(p.species, xs, vs):
            x1, v1 = O.move(p.n, p.h, p.dt, x, v, s.qom, Ec, Bc)
            x1s.append(x1)
            v1s.append(v1)
        xs, vs = x1s, v1s
        Jo, Mo = oracle_moments(O, p, xs, vs, qs, Bnc)
        assert rel(host(J), Jo) < tol
        assert rel(host(M), Mo) < tol
    # the particle states themselves, matched through the sort permutation
    K = 0.0
    for s, sd, x, v, q, perm in zip(p.species, sp, xs, vs, qs, perms):
        K += O.kinetic(v, q, s.qom)
        assert rel(host(sd.vel), v[:, perm]) < tol
        if prec == "f64":
            xd = host(sd.pos)
        else:
            xd = I.decode_f32(host(sd.cell), host(sd.pos), p.n, p.h)
        assert periodic_rel(xd, x[:, perm], p.L) < tol
    assert abs(host(ke)[0] - K) <= (1e-12 if prec == "f64" else 1e-6) * K


def species_state(sd, prec):
    """Rows (cell or position, velocity, charge) of a species' particles, in a fixed order."""
    cols = [host(sd.cell).astype(np.float64)] if prec == "f32" else []
    cols += list(host(sd.pos).astype(np.float64)) + list(host(sd.vel).astype(np.float64))
    if sd.q is not None:
        cols.append(host(sd.q).astype(np.float64))
    rows = np.stack(cols)
    return rows[:, np.lexsort(rows[::-1])]


def check_grouping(I, p, sd, prec):
    """dst ranges: 0 .. np, non-decreasing, and every particle inside its range's cell."""
    cs = host(sd.cell_start).astype(np.int64)
    assert cs[0] == 0 and cs[-1] == sd.np and np.all(np.diff(cs) >= 0)
    if prec == "f32":
        cells = host(sd.cell).astype(np.int64)
    else:
        x = host(sd.pos)
        ijk = [np.floor(x[d] / p.h[d]).astype(np.int64) for d in range(3)]
        cells = ijk[0] + p.n[0] * (ijk[1] + p.n[1] * ijk[2])
    assert np.array_equal(cells, np.repeat(np.arange(p.nn), np.diff(cs)))


def regroup_case(E, I, p, prec):
    if prec == "f64":
        sp = [E.Species.from_f64(s.qom, s.x, s.v, s.q) for s in p.species]
        xs, vs, qs = [s.x for s in p.species], [s.v for s in p.species], [s.q for s in p.species]
        return sp, xs, vs, qs, torch.float64, TOL64
    st = I.to_f32_state(p)
    sp = [E.Species.from_f32(s.qom, f["cell"], f["off"], f["v"], f["q"]) for s, f in zip(p.species, st)]
    xs, vs, qs = [f["x64"] for f in st], [f["v64"] for f in st], [f["q64"] for f in st]
    return sp, xs, vs, qs, torch.float32, TOL32


def run_regroup_passes(E, O, I, p, prec, En, BN, Bnext, passes=2, plain_first=False):
    """Regrouping fused passes against the oracle: J, M and the kinetic energy
    each pass, the targets' grouping, the targets holding exactly the moved
    particles, and the final states (matched through their whole velocities).
    With plain_first, a fused pass without regrouping goes first, so the first
    regrouping starts from a stale grouping."""
    grid = E.Grid(p.n, p.h, p.dt)
    sp, xs, vs, qs, tdt, tol = regroup_case(E, I, p, prec)
    if prec == "f64":
        Ec, Bc, Bnc = En, BN, Bnext
    else:
        Ec, Bc, Bnc = round32(En), round32(BN), round32(Bnext)
    sp = sorted_species(E, grid, sp)
    dst = [s.empty_like() for s in sp]
    J = torch.full((3, p.nn), 7.0, dtype=tdt, device="cuda")
    M = torch.full((14, 9, p.nn), 7.0, dtype=tdt, device="cuda")
    if plain_first:
        E.move_moments(grid, sp, dev(Ec, tdt), dev(Bc, tdt), dev(Bnc, tdt), J, M)
        x1s, v1s = [], []
        for s, x, v in zip(p.species, xs, vs):
            x1, v1 = O.move(p.n, p.h, p.dt, x, v, s.qom, Ec, Bc)
            x1s.append(x1)
            v1s.append(v1)
        xs, vs = x1s, v1s
    for it in range(passes):
        ke = torch.zeros(1, dtype=torch.float64, device="cuda")
        E.move_moments_regroup(grid, sp, dst, dev(Ec, tdt), dev(Bc, tdt), dev(Bnc, tdt), J, M, ke)
        x1s, v1s = [], []
        for s, x, v in zip(p.species, xs, vs):
            x1, v1 = O.move(p.n, p.h, p.dt, x, v, s.qom, Ec, Bc)
            x1s.append(x1)
            v1s.append(v1)
        xs, vs = x1s, v1s
        Jo, Mo = oracle_moments(O, p, xs, vs, qs, Bnc)
        assert rel(host(J), Jo) < tol
        assert rel(host(M), Mo) < tol
        K = sum(O.kinetic(v, q, s.qom) for s, v, q in zip(p.species, vs, qs))
        assert abs(host(ke)[0] - K) <= (1e-12 if prec == "f64" else 1e-6) * max(K, 1e-300)
        for s, d in zip(sp, dst):
            check_grouping(I, p, d, prec)
            assert np.array_equal(species_state(s, prec), species_state(d, prec))
        sp, dst = dst, sp
    # match each particle to the oracle's through its whole velocity (nearest
    # neighbour; one component alone can tie within FP32 rounding)
    from scipy.spatial import cKDTree
    for d, x, v in zip(sp, xs, vs):
        if d.np == 0:
            continue
        vg = host(d.vel).astype(np.float64)
        idx = cKDTree(v.T).query(vg.T)[1]
        assert np.unique(idx).size == d.np
        assert rel(vg, v[:, idx]) < tol
        xd = host(d.pos) if prec == "f64" else I.decode_f32(host(d.cell), host(d.pos), p.n, p.h)
        assert periodic_rel(xd, x[:, idx], p.L) < tol


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n,ppc,vscale", [((8, 8, 8), 27, 1.0), ((6, 5, 4), 9, 40.0), ((2, 3, 2), 7, 20.0),
                                           ((13, 7, 5), 3, 5.0), ((9, 5, 1), 12, 10.0), ((16, 1, 1), 20, 10.0),
                                           ((8, 4, 1), 300, 2.0), ((4, 4, 2), 150, 2.0)])
def test_move_moments_regroup(E, O, I, prec, n, ppc, vscale):
    """ecsim_move_moments_regroup: two passes, each regrouping into the other
    set of arrays. Scaled velocities send many particles out of their cell,
    some beyond the workgroup's box (moved by the stray mover), some back."""
    say("move+moments regroup", prec, n, ppc, vscale)
    p, En, BN = make_case(I, n, ppc, 23)
    for s in p.species:
        s.v = s.v * vscale
    rng = np.random.default_rng(24)
    run_regroup_passes(E, O, I, p, prec, En, BN, BN + 0.01 * rng.standard_normal(BN.shape))


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n,ppc,vscale", [((6, 5, 4), 9, 40.0), ((9, 5, 1), 12, 10.0), ((4, 4, 2), 150, 2.0)])
def test_move_moments_regroup_from_stale_grouping(E, O, I, prec, n, ppc, vscale):
    """A fused pass without regrouping, then two regrouping passes: the first
    regroups particles that left their ranges a pass earlier (as every
    sort_every-th pass of the loop does)."""
    say("regroup from stale", prec, n, ppc, vscale)
    p, En, BN = make_case(I, n, ppc, 27)
    for s in p.species:
        s.v = s.v * vscale
    rng = np.random.default_rng(28)
    run_regroup_passes(E, O, I, p, prec, En, BN, BN + 0.01 * rng.standard_normal(BN.shape), plain_first=True)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_move_moments_regroup_four_species_and_empty(E, O, I, prec):
    """Four species (per-particle charges on two of them), then a case with an empty species."""
    import dataclasses
    say("regroup four species", prec)
    p, En, BN = make_case(I, (7, 6, 5), 8, 25)
    rng = np.random.default_rng(26)
    e, i = p.species
    extra = [dataclasses.replace(e, name="e2", qom=-0.5, q=e.q * (1.0 + 0.5 * rng.random(e.np)),
                                 v=e.v[:, ::-1].copy() * 8.0),
             dataclasses.replace(i, name="i2", qom=0.1, q=i.q * (1.0 + 0.5 * rng.random(i.np)), v=i.v * 3.0)]
    p.species = [e, i] + extra
    run_regroup_passes(E, O, I, p, prec, En, BN, BN + 0.01 * rng.standard_normal(BN.shape))
    p.species = [e, dataclasses.replace(i, q=i.q[:0], x=i.x[:, :0], v=i.v[:, :0])]
    run_regroup_passes(E, O, I, p, prec, En, BN, BN, passes=1)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_moments_stale_grouping(E, O, I, prec):
    """ecsim_moments with a cell_start left stale by a move (the stray path of the plain deposit)."""
    say("moments stale grouping", prec)
    p, En, BN = make_case(I, (6, 6, 5), 10, 19)
    for s in p.species:
        s.v = s.v * 30.0
    grid = E.Grid(p.n, p.h, p.dt)
    if prec == "f64":
        sp = [E.Species.from_f64(s.qom, s.x, s.v, s.q) for s in p.species]
        xs, vs, qs = [s.x for s in p.species], [s.v for s in p.species], [s.q for s in p.species]
        Ec, Bc, tdt, tol = En, BN, torch.float64, TOL64
    else:
        st = I.to_f32_state(p)
        sp = [E.Species.from_f32(s.qom, f["cell"], f["off"], f["v"], f["q"]) for s, f in zip(p.species, st)]
        xs, vs, qs = [f["x64"] for f in st], [f["v64"] for f in st], [f["q64"] for f in st]
        Ec, Bc, tdt, tol = round32(En), round32(BN), torch.float32, TOL32
    sp = sorted_species(E, grid, sp)
    for s in sp:
        cs = s.cell_start
        E.move(grid, s, dev(Ec, tdt), dev(Bc, tdt))
        s.cell_start = cs          # keep the pre-move grouping
    J = torch.empty((3, p.nn), dtype=tdt, device="cuda")
    M = torch.empty((14, 9, p.nn), dtype=tdt, device="cuda")
    E.moments(grid, sp, dev(Bc, tdt), J, M, flags=E.SORTED)
    x1s, v1s = [], []
    for s, x, v in zip(p.species, xs, vs):
        x1, v1 = O.move(p.n, p.h, p.dt, x, v, s.qom, Ec, Bc)
        x1s.append(x1)
        v1s.append(v1)
    Jo, Mo = oracle_moments(O, p, x1s, v1s, qs, Bc)
    assert rel(host(J), Jo) < tol
    assert rel(host(M), Mo) < tol


def test_moments_tiled_variable_charge(E, O, I):
    """Per-particle charges (the double-Harris layout) through the tiled deposit."""
    say("moments tiled variable q")
    p = I.harris(n=(8, 32, 4), ppc=6)
    BN = O.centres_to_nodes(p.n, p.B_C)
    grid = E.Grid(p.n, p.h, p.dt)
    st = I.to_f32_state(p)
    sp = [E.Species.from_f32(s.qom, f["cell"], f["off"], f["v"], f["q"]) for s, f in zip(p.species, st)]
    assert sp[0].q is not None
    sp = sorted_species(E, grid, sp)
    J = torch.empty((3, p.nn), dtype=torch.float32, device="cuda")
    M = torch.empty((14, 9, p.nn), dtype=torch.float32, device="cuda")
    E.moments(grid, sp, dev(BN, torch.float32), J, M, flags=E.SORTED)
    Jo, Mo = oracle_moments(O, p, [f["x64"] for f in st], [f["v64"] for f in st], [f["q64"] for f in st],
                            round32(BN))
    assert rel(host(J), Jo) < TOL32
    assert rel(host(M), Mo) < TOL32


def test_moments_accumulate_flag(E, O, I):
    say("moments accumulate")
    p, _, BN = make_case(I, (4, 4, 4), 5, 5)
    grid = E.Grid(p.n, p.h, p.dt)
    sp = [E.Species.from_f64(s.qom, s.x, s.v, s.q) for s in p.species]
    J = torch.empty((3, p.nn), dtype=torch.float64, device="cuda")
    M = torch.empty((14, 9, p.nn), dtype=torch.float64, device="cuda")
    E.moments(grid, sp[:1], dev(BN), J, M)
    E.moments(grid, sp[1:], dev(BN), J, M, flags=E.ACCUMULATE)
    Jo, Mo = oracle_moments(O, p, [s.x for s in p.species], [s.v for s in p.species], [s.q for s in p.species], BN)
    assert rel(host(J), Jo) < TOL64 and rel(host(M), Mo) < TOL64


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n", [(5, 6, 3), (9, 5, 1)])
def test_clear_and_accumulate_grouped(E, O, I, prec, n):
    """The grouped calls clear J and M over the whole grid (bricks that the grid
    cuts short included) unless ECSIM_ACCUMULATE is set, when they add to them:
    outputs prefilled with 7 are overwritten, and an accumulating second call
    doubles the first. Moments-only and fused calls."""
    say("clear / accumulate", prec, n)
    p, En, BN = make_case(I, n, 6, 41)
    grid = E.Grid(p.n, p.h, p.dt)
    if prec == "f64":
        mk = lambda: [E.Species.from_f64(s.qom, s.x, s.v, s.q) for s in p.species]
        xs, vs, qs = [s.x for s in p.species], [s.v for s in p.species], [s.q for s in p.species]
        Bc, Ec, tdt, tol = BN, En, torch.float64, TOL64
    else:
        st = I.to_f32_state(p)
        mk = lambda: [E.Species.from_f32(s.qom, f["cell"], f["off"], f["v"], f["q"]) for s, f in zip(p.species, st)]
        xs, vs, qs = [f["x64"] for f in st], [f["v64"] for f in st], [f["q64"] for f in st]
        Bc, Ec, tdt, tol = round32(BN), round32(En), torch.float32, TOL32
    Bd, Ed = dev(Bc, tdt), dev(Ec, tdt)
    full = lambda shape: torch.full(shape, 7.0, dtype=tdt, device="cuda")
    # moments only
    sp = sorted_species(E, grid, mk())
    J, M = full((3, p.nn)), full((14, 9, p.nn))
    E.moments(grid, sp, Bd, J, M, flags=E.SORTED)
    Jo, Mo = oracle_moments(O, p, xs, vs, qs, Bc)
    assert rel(host(J), Jo) < tol and rel(host(M), Mo) < tol
    E.moments(grid, sp, Bd, J, M, flags=E.SORTED | E.ACCUMULATE)
    assert rel(host(J), 2 * Jo) < tol and rel(host(M), 2 * Mo) < tol
    # fused: two copies of the same state
    J1, M1 = full((3, p.nn)), full((14, 9, p.nn))
    E.move_moments(grid, sorted_species(E, grid, mk()), Ed, Bd, Bd, J1, M1)
    xo, vo = [], []
    for s, x, v in zip(p.species, xs, vs):
        a, b = O.move(p.n, p.h, p.dt, x, v, s.qom, Ec, Bc)
        xo.append(a)
        vo.append(b)
    Jo, Mo = oracle_moments(O, p, xo, vo, qs, Bc)
    assert rel(host(J1), Jo) < tol and rel(host(M1), Mo) < tol
    J2, M2 = J1.clone(), M1.clone()
    E.move_moments(grid, sorted_species(E, grid, mk()), Ed, Bd, Bd, J2, M2, flags=E.ACCUMULATE)
    assert rel(host(J2), 2 * host(J1)) < tol and rel(host(M2), 2 * host(M1)) < tol


# ---------------------------------------------------------------------------
# sort
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("f32", [False, True])
def test_sort(E, I, f32):
    say("sort", f32)
    p = I.config1(ppc=4, n=(16, 8, 4))
    grid = E.Grid(p.n, p.h, p.dt)
    s = p.species[0]     # electrons: random order
    if f32:
        f = I.to_f32_state(p)[0]
        src = E.Species.from_f32(s.qom, f["cell"], f["off"], f["v"], f["q"])
        key = f["cell"].astype(np.int64)
    else:
        src = E.Species.from_f64(s.qom, s.x, s.v, s.q)
        ijk = [np.floor(s.x[d] / p.h[d]).astype(np.int64) for d in range(3)]
        key = ijk[0] + p.n[0] * (ijk[1] + p.n[1] * ijk[2])
    dst = src.empty_like()
    cs = torch.empty(p.nn + 1, dtype=torch.int32, device="cuda")
    perm = torch.empty(s.np, dtype=torch.int32, device="cuda")
    E.sort(grid, src, dst, cs, perm)
    perm_h = host(perm).astype(np.int64)
    assert np.array_equal(np.sort(perm_h), np.arange(s.np))
    # keys are non-decreasing in the output and cell_start brackets each cell
    kd = key[perm_h]
    assert np.all(np.diff(kd) >= 0)
    cs_h = host(cs).astype(np.int64)
    assert cs_h[0] == 0 and cs_h[-1] == s.np
    assert np.array_equal(cs_h[:-1], np.searchsorted(kd, np.arange(p.nn), side="left"))
    # payload moved with its key
    assert np.array_equal(host(dst.pos), host(src.pos)[:, perm_h])
    assert np.array_equal(host(dst.vel), host(src.vel)[:, perm_h])
    if f32:
        assert np.array_equal(host(dst.cell), host(src.cell)[perm_h])


# ---------------------------------------------------------------------------
# mass-matrix apply
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,ppc", CASES)
@pytest.mark.parametrize("mprec", ["f64", "f32"])
def test_mass_apply(E, O, I, n, ppc, mprec):
    say("mass apply", mprec, n, ppc)
    p, _, BN = make_case(I, n, ppc, 6)
    _, M27 = O.species_moments(p, [s.x for s in p.species], [s.v for s in p.species], BN)
    M14 = O.m14(p.n, M27)
    if mprec == "f32":
        M14 = round32(M14)
        M27 = round32(M27)
    x = np.random.default_rng(7).standard_normal((3, p.nn))
    y0 = np.random.default_rng(8).standard_normal((3, p.nn))
    grid = E.Grid(p.n, p.h, p.dt)
    Mt = dev(M14, torch.float32 if mprec == "f32" else torch.float64)
    y = dev(y0)
    E.mass_apply(grid, Mt, dev(x), y, a=0.7, b=-0.3)
    ref = 0.7 * O.mass_apply27(p.n, M27, x) - 0.3 * y0
    assert rel(host(y), ref) < TOL64


def test_mass_apply_dense_2x2x2(E, O, I):
    """Every unit vector through the 14-block apply equals the dense brute-force operator."""
    say("mass apply dense 2x2x2")
    p, _, BN = make_case(I, (2, 2, 2), 5, 9)
    _, M27 = O.species_moments(p, [s.x for s in p.species], [s.v for s in p.species], BN)
    grid = E.Grid(p.n, p.h, p.dt)
    Mt = dev(O.m14(p.n, M27))
    n3 = 3 * p.nn
    eye = np.eye(n3)
    cols = np.zeros((n3, n3))
    for j in range(n3):
        y = torch.zeros((3, p.nn), dtype=torch.float64, device="cuda")
        E.mass_apply(grid, Mt, dev(eye[j].reshape(3, -1)), y)
        cols[:, j] = host(y).ravel()
    ref = np.stack([O.mass_apply27(p.n, M27, eye[j].reshape(3, -1)).ravel() for j in range(n3)], axis=1)
    assert rel(cols, ref) < TOL64


# ---------------------------------------------------------------------------
# field solve and the full step
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("mprec,n", [("f64", (6, 5, 4)), ("f32", (6, 5, 4)), ("f64", (32, 16, 16)),
                                     ("f32", (13, 11, 9)), ("f64", (2, 2, 2)), ("f64", (1, 3, 2))])
def test_field_solve(E, O, I, mprec, n):
    """One workgroup (120 nodes), eight (8192 nodes: the XCD-contiguous block
    order of the operator kernels), two with a ragged tail (1287 nodes), and
    grids where the periodic images of g + o and g - o coincide (2 cells) or
    equal g (1 cell), which the curl-curl stencil must count once per offset."""
    say("field solve", mprec, n)
    p, _, BN = make_case(I, n, 6, 10)
    J, M27 = O.species_moments(p, [s.x for s in p.species], [s.v for s in p.species], BN)
    rng = np.random.default_rng(11)
    En = 1e-3 * rng.standard_normal((3, p.nn))
    BC = BN + 1e-3 * rng.standard_normal((3, p.nn))
    M14 = O.m14(p.n, M27)
    tdt = torch.float64
    if mprec == "f32":
        M14, M27, J = round32(M14), round32(M27), round32(J)
        tdt = torch.float32
    ref = O.field_solve(p.n, p.h, p.dt, M27, J, En, BC, tol=1e-13)
    grid = E.Grid(p.n, p.h, p.dt)
    Et, En1, Bn1 = (torch.empty((3, p.nn), dtype=torch.float64, device="cuda") for _ in range(3))
    it, res = E.field_solve(grid, dev(M14, tdt), dev(J, tdt), dev(En), dev(BC), Et, En1, Bn1, tol=1e-10)
    assert it > 0 and res <= 1e-10
    assert rel(host(Et), ref["E_theta"]) < 1e-9
    assert rel(host(En1), ref["E_next"]) < 1e-9
    assert rel(host(Bn1), ref["BC_next"]) < 1e-9
    # independent residual check with the oracle's operator
    b = O.field_rhs(p.n, p.h, p.dt, J, En, BC)
    r = b - O.field_operator(p.n, p.h, p.dt, M27, host(Et))
    assert np.linalg.norm(r) <= 2e-10 * np.linalg.norm(b)


def solve_inputs(E, O, I, n=(6, 5, 4)):
    p, _, BN = make_case(I, n, 6, 10)
    J, M27 = O.species_moments(p, [s.x for s in p.species], [s.v for s in p.species], BN)
    rng = np.random.default_rng(11)
    En = 1e-3 * rng.standard_normal((3, p.nn))
    BC = BN + 1e-3 * rng.standard_normal((3, p.nn))
    return p, J, M27, En, BC


@pytest.mark.parametrize("restart", [1, 2, 3])
def test_field_solve_restarted(E, O, I, restart):
    """GMRES(1..3): several restart cycles, each closed by the true residual;
    the result is the same solution."""
    say("field solve restarted", restart)
    p, J, M27, En, BC = solve_inputs(E, O, I)
    ref = O.field_solve(p.n, p.h, p.dt, M27, J, En, BC, tol=1e-13)
    grid = E.Grid(p.n, p.h, p.dt)
    Et, En1, Bn1 = (torch.empty((3, p.nn), dtype=torch.float64, device="cuda") for _ in range(3))
    it, res = E.field_solve(grid, dev(O.m14(p.n, M27)), dev(J), dev(En), dev(BC), Et, En1, Bn1, tol=1e-10,
                            restart=restart, maxit=500)
    assert it > restart and res <= 1e-10
    assert rel(host(Et), ref["E_theta"]) < 1e-9
    assert rel(host(Bn1), ref["BC_next"]) < 1e-9
    b = O.field_rhs(p.n, p.h, p.dt, J, En, BC)
    r = b - O.field_operator(p.n, p.h, p.dt, M27, host(Et))
    assert np.linalg.norm(r) <= 2e-10 * np.linalg.norm(b)


def test_field_solve_batches_of_one_cycle(E, O, I):
    """After a GMRES(1) solve the first batch of the next solve is one step
    long, so a GMRES(30) solve continues its cycle over several batches, each
    closed by moving E by V times the change in y: the same solution."""
    say("field solve, one cycle over several batches")
    p, J, M27, En, BC = solve_inputs(E, O, I)
    grid = E.Grid(p.n, p.h, p.dt)
    M14 = dev(O.m14(p.n, M27))
    Et, En1, Bn1 = (torch.empty((3, p.nn), dtype=torch.float64, device="cuda") for _ in range(3))
    E.field_solve(grid, M14, dev(J), dev(En), dev(BC), Et, En1, Bn1, tol=1e-10, restart=1, maxit=500)
    it, res = E.field_solve(grid, M14, dev(J), dev(En), dev(BC), Et, En1, Bn1, tol=1e-10, restart=30, maxit=500)
    ref = O.field_solve(p.n, p.h, p.dt, M27, J, En, BC, tol=1e-13)
    assert 1 < it <= 30 and res <= 1e-10
    assert rel(host(Et), ref["E_theta"]) < 1e-9
    assert rel(host(En1), ref["E_next"]) < 1e-9
    assert rel(host(Bn1), ref["BC_next"]) < 1e-9


def test_field_solve_no_convergence(E, O, I):
    """maxit below what tol needs: ENOCONV, and the outputs hold the last
    iterate advanced consistently (E^{n+1} = 2 E^{n+theta} - E^n)."""
    say("field solve, no convergence")
    p, J, M27, En, BC = solve_inputs(E, O, I)
    grid = E.Grid(p.n, p.h, p.dt)
    Et, En1, Bn1 = (torch.empty((3, p.nn), dtype=torch.float64, device="cuda") for _ in range(3))
    with pytest.raises(E.EcsimError) as ex:
        E.field_solve(grid, dev(O.m14(p.n, M27)), dev(J), dev(En), dev(BC), Et, En1, Bn1, tol=1e-14, restart=30,
                      maxit=2)
    assert ex.value.status == E.ENOCONV
    et = host(Et)
    assert np.isfinite(et).all()
    assert rel(host(En1), 2.0 * et - En) < 1e-14
    b = O.field_rhs(p.n, p.h, p.dt, J, En, BC)
    r = b - O.field_operator(p.n, p.h, p.dt, M27, et)
    r0 = b - O.field_operator(p.n, p.h, p.dt, M27, En)
    assert 1e-14 * np.linalg.norm(b) < np.linalg.norm(r) < np.linalg.norm(r0)


def test_field_solve_long_cycle(E, O, I):
    """A 30 times longer time step makes the system harder: one GMRES(60)
    cycle takes more than 40 columns, beyond the least-squares triangle the
    last kernel of a batch stages in LDS, and must still give the oracle's
    solution."""
    say("field solve, more than 40 columns in one cycle")
    p, J, M27, En, BC = solve_inputs(E, O, I)
    dt = 30 * p.dt
    grid = E.Grid(p.n, p.h, dt)
    Et, En1, Bn1 = (torch.empty((3, p.nn), dtype=torch.float64, device="cuda") for _ in range(3))
    it, res = E.field_solve(grid, dev(O.m14(p.n, M27)), dev(J), dev(En), dev(BC), Et, En1, Bn1, tol=1e-12,
                            restart=60, maxit=200)
    assert 40 < it <= 60 and res <= 1e-12
    ref = O.field_solve(p.n, p.h, dt, M27, J, En, BC, tol=1e-14, restart=120, maxit=400)
    assert rel(host(Et), ref["E_theta"]) < 1e-10
    assert rel(host(Bn1), ref["BC_next"]) < 1e-10
    b = O.field_rhs(p.n, p.h, dt, J, En, BC)
    r = b - O.field_operator(p.n, p.h, dt, M27, host(Et))
    assert np.linalg.norm(r) <= 2e-12 * np.linalg.norm(b)


def test_field_solve_zero_rhs(E, O, I):
    """b = 0 (E^n, J and B^n zero): E^{n+theta} = 0 after no iterations."""
    say("field solve, zero right-hand side")
    p, J, M27, En, BC = solve_inputs(E, O, I)
    grid = E.Grid(p.n, p.h, p.dt)
    z = torch.zeros((3, p.nn), dtype=torch.float64, device="cuda")
    Et, En1, Bn1 = (torch.full((3, p.nn), 7.0, dtype=torch.float64, device="cuda") for _ in range(3))
    it, res = E.field_solve(grid, dev(O.m14(p.n, M27)), z, z, z, Et, En1, Bn1, tol=1e-10)
    assert it == 0 and res == 0.0
    for t in (Et, En1, Bn1):
        assert not host(t).any()


@pytest.mark.parametrize("where", ["M", "J"])
def test_field_solve_nonfinite(E, O, I, where):
    """A NaN in M or J ends the solve with ENONFINITE."""
    say("field solve, NaN in", where)
    p, J, M27, En, BC = solve_inputs(E, O, I)
    M14 = O.m14(p.n, M27)
    if where == "M":
        M14 = M14.copy()
        M14.flat[37] = np.nan
    else:
        J = J.copy()
        J[1, 5] = np.nan
    grid = E.Grid(p.n, p.h, p.dt)
    Et, En1, Bn1 = (torch.empty((3, p.nn), dtype=torch.float64, device="cuda") for _ in range(3))
    with pytest.raises(E.EcsimError) as ex:
        E.field_solve(grid, dev(M14), dev(J), dev(En), dev(BC), Et, En1, Bn1, tol=1e-10)
    assert ex.value.status == E.ENONFINITE


def test_centres_to_nodes_and_energy(E, O, I):
    say("centres to nodes, field energy")
    n = (5, 6, 7)
    rng = np.random.default_rng(12)
    BC = rng.standard_normal((3, 210))
    grid = E.Grid(n, (0.5,) * 3, 0.1)
    BN = torch.empty((3, 210), dtype=torch.float64, device="cuda")
    BN32 = torch.empty((3, 210), dtype=torch.float32, device="cuda")
    E.centres_to_nodes(grid, dev(BC), BN, BN32)
    ref = O.centres_to_nodes(n, BC)
    assert rel(host(BN), ref) < 1e-15
    assert rel(host(BN32), ref) < 1e-7
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    E.field_energy(grid, dev(BC), out)
    assert abs(host(out)[0] - O.field_energy(n, (0.5,) * 3, BC)) < 1e-13 * O.field_energy(n, (0.5,) * 3, BC)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_two_dimensional_run(E, O, I, prec):
    """A reduced run, 8 x 8 x 1 cells x 27 ppc x 2 species, fused path, 8 steps:
    positions along z stay put (fixPosition), energy is conserved (FP64) and
    the state matches the oracle's run."""
    say("2D run", prec)
    p = I.uniform_plasma(95, (8, 8, 1), 27)
    P = E.F64 if prec == "f64" else E.F32
    sim = E.Simulation(p, prec=P, tol=1e-10, fused=True, sort_every=3)
    if prec == "f32":
        for s, f in zip(p.species, I.to_f32_state(p)):
            s.x, s.v, s.q = f["x64"], f["v64"], f["q64"]
    z0 = [s.x[2].copy() for s in p.species]
    K0 = kinetic0(E, O, p, prec)
    WE0, WB0 = sim.energy()
    e0 = K0 + WE0 + WB0
    drift = 0.0
    for step in range(8):
        sim.step()
        WE, WB = sim.energy()
        drift = max(drift, abs(host(sim.scal)[0] + WE + WB - e0) / e0)
    if prec == "f64":
        assert drift <= 1e-10
        ref, _ = O.run_steps(p, 8, tol=1e-13)
        assert rel(host(sim.E), ref["E"]) < 1e-9
    else:
        # 3,456 particles: the once-per-step rounding of v averages less
        say("drift", drift, "bound", fp32_drift_bound(p, 8, e0))
        assert drift <= fp32_drift_bound(p, 8, e0)
    for s, z in zip(sim.species, z0):
        if prec == "f64":
            zs = host(s.pos)[2]
        else:
            zs = I.decode_f32(host(s.cell), host(s.pos), p.n, p.h)[2]
        assert np.array_equal(np.sort(zs), np.sort(z))


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("sort", [False, True, "fused", "regroup"])
def test_small_workload_ten_steps(E, O, I, prec, sort):
    """8^3 cells, 27 ppc x 2 species, 10 steps: state parity and energy drift."""
    say("config-0 ten steps", prec, sort)
    p = I.config0()
    P = E.F64 if prec == "f64" else E.F32
    if sort == "fused":
        sim = E.Simulation(p, prec=P, tol=1e-10, fused=True, sort_every=3)
    elif sort == "regroup":
        sim = E.Simulation(p, prec=P, tol=1e-10, fused=True, regroup=True)
    else:
        sim = E.Simulation(p, prec=P, tol=1e-10, sort=sort)
    if prec == "f32":
        st = I.to_f32_state(p)
        for s, f in zip(p.species, st):
            s.x, s.v, s.q = f["x64"], f["v64"], f["q64"]
    K0 = kinetic0(E, O, p, prec)
    WE0, WB0 = sim.energy()
    e0 = K0 + WE0 + WB0
    drift = 0.0
    for step in range(10):
        sim.step()
        K = host(sim.scal)[0]
        WE, WB = sim.energy()
        drift = max(drift, abs(K + WE + WB - e0) / e0)
        assert sim.last_resid <= 1e-10
    say("drift", drift)
    if prec == "f64":
        assert drift <= 1e-10
        ref, _ = O.run_steps(p, 10, tol=1e-13)
        assert rel(host(sim.E), ref["E"]) < 1e-9
        if not sort:
            for s, x, v in zip(sim.species, ref["x"], ref["v"]):
                assert rel(host(s.vel), v) < 1e-9
                assert periodic_rel(host(s.pos), x, p.L) < 1e-9
        else:
            # the sort permutes particles: match them through their x velocity, whose
            # gaps (~1e-8) are far above the accumulated rounding (~1e-13)
            for s, x, v in zip(sim.species, ref["x"], ref["v"]):
                ka = np.argsort(host(s.vel)[0])
                kb = np.argsort(v[0])
                assert rel(host(s.vel)[:, ka], v[:, kb]) < 1e-9
                assert periodic_rel(host(s.pos)[:, ka], x[:, kb], p.L) < 1e-9
    else:
        # FP32 particle state: each stored velocity is rounded once per step (the
        # update itself is formed in FP64), an unbiased error that averages over
        # the 27,648 particles to a few 1e-10 over ten steps
        say("bound", fp32_drift_bound(p, 10, e0))
        assert drift <= fp32_drift_bound(p, 10, e0)


# ---------------------------------------------------------------------------
# adjoint
# ---------------------------------------------------------------------------

def grad_case(I, n=(5, 4, 4), ppc=4, seed=13):
    p = I.uniform_plasma(400 + seed, n, ppc)
    rng = np.random.default_rng(500 + seed)
    En = 1e-2 * rng.standard_normal((3, p.nn))
    BN = np.array([[0.0], [0.05], [0.2]]) + 0.05 * rng.standard_normal((3, p.nn))
    gJ = rng.standard_normal((3, p.nn))
    gM = rng.standard_normal((14, 9, p.nn))
    return p, En, BN, gJ, gM


@pytest.mark.parametrize("n,ppc", [((5, 4, 4), 4), ((2, 2, 2), 6), ((3, 1, 2), 5)])
def test_backward_f64_matches_dual_oracle(E, O, I, n, ppc):
    say("backward f64", n, ppc)
    p, En, BN, gJ, gM = grad_case(I, n, ppc)
    grid = E.Grid(p.n, p.h, p.dt)
    gE = torch.zeros((3, p.nn), dtype=torch.float64, device="cuda")
    gB = torch.zeros((3, p.nn), dtype=torch.float64, device="cuda")
    gEo = np.zeros((3, p.nn))
    gBo = np.zeros((3, p.nn))
    for s in p.species:
        sp = E.Species.from_f64(s.qom, s.x, s.v, s.q)
        gx = torch.empty_like(sp.pos)
        gv = torch.empty_like(sp.vel)
        E.moments_backward(grid, sp, dev(En), dev(BN), dev(gJ), dev(gM), gx, gv, gE, gB, through_mover=True)
        gxo, gvo, _, _ = O.grad(p.n, p.h, p.dt, s.x, s.v, s.q, s.qom, En, BN, gJ, gM, gEo, gBo)
        assert rel(host(gx), gxo) < TOL64
        assert rel(host(gv), gvo) < TOL64
    assert rel(host(gE), gEo) < TOL64
    assert rel(host(gB), gBo) < TOL64


@pytest.mark.parametrize("order", ["cells", "shuffled", "interleaved"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_backward_particle_order(E, O, I, prec, order):
    """The grid gradients do not depend on particle order: cell-ordered
    particles (long runs of lanes on one node), a random order, and two cells'
    particles alternating (the same node coming back in separate runs)."""
    say("backward order", prec, order)
    p, En, BN, gJ, gM = grad_case(I, (6, 5, 4), 9, 21)
    grid = E.Grid(p.n, p.h, p.dt)
    tdt, tol = (torch.float64, TOL64) if prec == "f64" else (torch.float32, TOL32)
    rng = np.random.default_rng(22)
    gE = torch.zeros((3, p.nn), dtype=tdt, device="cuda")
    gB = torch.zeros((3, p.nn), dtype=tdt, device="cuda")
    gEo = np.zeros((3, p.nn))
    gBo = np.zeros((3, p.nn))
    Ec, Bc, gJc, gMc = (En, BN, gJ, gM) if prec == "f64" else (round32(En), round32(BN), round32(gJ), round32(gM))
    states = I.to_f32_state(p) if prec == "f32" else [None] * len(p.species)
    for s, f in zip(p.species, states):
        x = s.x if f is None else f["x64"]
        cells = np.floor(x[0] / p.h[0]).astype(np.int64) + p.n[0] * (np.floor(x[1] / p.h[1]).astype(np.int64)
                                                                      + p.n[1] * np.floor(x[2] / p.h[2]).astype(np.int64))
        if order == "cells":
            perm = np.argsort(cells, kind="stable")
        elif order == "shuffled":
            perm = rng.permutation(s.np)
        else:
            srt = np.argsort(cells, kind="stable")
            half = (len(srt) + 1) // 2
            perm = np.empty_like(srt)
            perm[0::2] = srt[:half]
            perm[1::2] = srt[half:]
        if f is None:
            sp = E.Species.from_f64(s.qom, s.x[:, perm], s.v[:, perm], s.q[perm])
            xs, vs, qs = s.x[:, perm], s.v[:, perm], s.q[perm]
        else:
            sp = E.Species.from_f32(s.qom, f["cell"][perm], f["off"][:, perm], f["v"][:, perm], f["q"][perm])
            xs, vs, qs = f["x64"][:, perm], f["v64"][:, perm], f["q64"][perm]
        gx = torch.empty_like(sp.pos)
        gv = torch.empty_like(sp.vel)
        E.moments_backward(grid, sp, dev(Ec, tdt), dev(Bc, tdt), dev(gJc, tdt), dev(gMc, tdt), gx, gv, gE, gB,
                           through_mover=True)
        gxo, gvo, _, _ = O.grad(p.n, p.h, p.dt, xs, vs, qs, s.qom, Ec, Bc, gJc, gMc, gEo, gBo)
        assert rel(host(gx), gxo) < tol
        assert rel(host(gv), gvo) < tol
    assert rel(host(gE), gEo) < tol
    assert rel(host(gB), gBo) < tol


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n,ppc,vscale,stale,through", [
    ((6, 5, 4), 9, 1.0, False, True), ((6, 5, 4), 9, 30.0, False, True), ((6, 5, 4), 9, 3.0, True, True),
    ((9, 5, 1), 12, 5.0, False, True), ((3, 1, 2), 5, 5.0, False, True), ((8, 8, 4), 27, 1.0, False, True)])
def test_backward_grouped_matches_dual_oracle(E, O, I, prec, n, ppc, vscale, stale, through):
    """The brick-tiled adjoint (particles grouped by cell: every cell's
    gradient blocks formed once in LDS) against the oracle's dual-number
    gradient. Scaled velocities send particles out of their cell in the move,
    and a stale grouping (the particles moved once after the grouping) leaves
    particles outside their range's cell: both go through the listed general
    path. (Without the mover: test_backward_moments_only_matches_fd.)"""
    say("backward grouped", prec, n, ppc, vscale, stale, through)
    p, En, BN, gJ, gM = grad_case(I, n, ppc, 31)
    for sp_ in p.species:
        sp_.v = sp_.v * vscale
    grid = E.Grid(p.n, p.h, p.dt)
    tdt, tol = (torch.float64, TOL64) if prec == "f64" else (torch.float32, TOL32)
    Ec, Bc, gJc, gMc = (En, BN, gJ, gM) if prec == "f64" else (round32(En), round32(BN), round32(gJ), round32(gM))
    gE = torch.zeros((3, p.nn), dtype=tdt, device="cuda")
    gB = torch.zeros((3, p.nn), dtype=tdt, device="cuda")
    gEo = np.zeros((3, p.nn))
    gBo = np.zeros((3, p.nn))
    states = I.to_f32_state(p) if prec == "f32" else [None] * len(p.species)
    for s, f in zip(p.species, states):
        if f is None:
            sp = E.Species.from_f64(s.qom, s.x, s.v, s.q)
        else:
            sp = E.Species.from_f32(s.qom, f["cell"], f["off"], f["v"], f["q"])
        d = sp.empty_like()
        cs = torch.empty(grid.nn + 1, dtype=torch.int32, device="cuda")
        perm = torch.empty(sp.np, dtype=torch.int32, device="cuda")
        E.sort(grid, sp, d, cs, perm)
        d.cell_start = cs
        if stale:   # the grouping goes stale: one move with small fields
            E.move(grid, d, dev(0.1 * Ec, tdt), dev(Bc, tdt))
        if f is None:
            xs, vs = host(d.pos), host(d.vel)
            qs = s.q[host(perm).astype(np.int64)]
        else:
            xs = I.decode_f32(host(d.cell), host(d.pos), p.n, p.h)
            vs = host(d.vel).astype(np.float64)
            qs = f["q64"][host(perm).astype(np.int64)]
        gx = torch.empty_like(d.pos)
        gv = torch.empty_like(d.vel)
        E.moments_backward(grid, d, dev(Ec, tdt), dev(Bc, tdt), dev(gJc, tdt), dev(gMc, tdt), gx, gv, gE, gB,
                           through_mover=True)
        gxo, gvo, _, _ = O.grad(p.n, p.h, p.dt, xs, vs, qs, s.qom, Ec, Bc, gJc, gMc, gEo, gBo)
        assert rel(host(gx), gxo) < tol
        assert rel(host(gv), gvo) < tol
    assert rel(host(gE), gEo) < tol
    assert rel(host(gB), gBo) < tol


def test_backward_f32_matches_dual_oracle(E, O, I):
    say("backward f32")
    p, En, BN, gJ, gM = grad_case(I, (5, 4, 4), 4, 14)
    grid = E.Grid(p.n, p.h, p.dt)
    gE = torch.zeros((3, p.nn), dtype=torch.float32, device="cuda")
    gB = torch.zeros((3, p.nn), dtype=torch.float32, device="cuda")
    gEo = np.zeros((3, p.nn))
    gBo = np.zeros((3, p.nn))
    E32, B32, gJ32, gM32 = round32(En), round32(BN), round32(gJ), round32(gM)
    for s, f in zip(p.species, I.to_f32_state(p)):
        sp = E.Species.from_f32(s.qom, f["cell"], f["off"], f["v"], f["q"])
        gx = torch.empty_like(sp.pos)
        gv = torch.empty_like(sp.vel)
        E.moments_backward(grid, sp, dev(E32, torch.float32), dev(B32, torch.float32), dev(gJ32, torch.float32),
                           dev(gM32, torch.float32), gx, gv, gE, gB, through_mover=True)
        gxo, gvo, _, _ = O.grad(p.n, p.h, p.dt, f["x64"], f["v64"], f["q64"], s.qom, E32, B32, gJ32, gM32, gEo, gBo)
        assert rel(host(gx), gxo) < TOL32
        assert rel(host(gv), gvo) < TOL32
    assert rel(host(gE), gEo) < TOL32
    assert rel(host(gB), gBo) < TOL32


@pytest.mark.parametrize("grouped", [False, True])
def test_backward_moments_only_matches_fd(E, O, I, grouped):
    """Without the mover: dL/dx, dL/dv of <gJ,J> + <gM,M> by central differences of the oracle's moments,
    for particles in any order and grouped by cell (the brick-tiled kernel); dL/dB at sampled nodes by
    central differences of the whole loss."""
    say("backward moments-only", "grouped" if grouped else "any order")
    p, En, BN, gJ, gM = grad_case(I, (4, 4, 3), 2, 15)
    grid = E.Grid(p.n, p.h, p.dt)
    s = p.species[0]
    sp = E.Species.from_f64(s.qom, s.x, s.v, s.q)
    if grouped:
        d = sp.empty_like()
        cs = torch.empty(grid.nn + 1, dtype=torch.int32, device="cuda")
        perm = torch.empty(sp.np, dtype=torch.int32, device="cuda")
        E.sort(grid, sp, d, cs, perm)
        d.cell_start = cs
        sp = d
        k = host(perm).astype(np.int64)
        s = dataclasses.replace(s, x=s.x[:, k], v=s.v[:, k], q=s.q[k])
    gx = torch.empty_like(sp.pos)
    gv = torch.empty_like(sp.vel)
    gB = torch.zeros((3, p.nn), dtype=torch.float64, device="cuda")
    E.moments_backward(grid, sp, None, dev(BN), dev(gJ), dev(gM), gx, gv, None, gB, through_mover=False)
    gx, gv = host(gx), host(gv)

    def loss_one(x, v, i):
        J, M27 = O.moments(p.n, p.h, p.dt, x[:, i:i + 1], v[:, i:i + 1], s.q[i:i + 1], s.qom, BN)
        return np.sum(gJ * J) + np.sum(gM * O.m14(p.n, M27))

    def loss_all(B):
        J, M27 = O.moments(p.n, p.h, p.dt, s.x, s.v, s.q, s.qom, B)
        return np.sum(gJ * J) + np.sum(gM * O.m14(p.n, M27))

    gBh = host(gB)
    for node in range(0, p.nn, max(1, p.nn // 6)):
        for c in range(3):
            up = BN.copy(); up[c, node] += 1e-6
            dn = BN.copy(); dn[c, node] -= 1e-6
            fd = (loss_all(up) - loss_all(dn)) / 2e-6
            assert abs(gBh[c, node] - fd) <= 1e-6 * max(np.max(np.abs(gBh)), 1e-30)

    eps = 1e-6
    for i in range(0, s.np, max(1, s.np // 12)):
        for c in range(3):
            for arr, g in ((s.x, gx), (s.v, gv)):
                up = arr.copy(); up[c, i] += eps
                dn = arr.copy(); dn[c, i] -= eps
                if arr is s.x:
                    fd = (loss_one(up, s.v, i) - loss_one(dn, s.v, i)) / (2 * eps)
                else:
                    fd = (loss_one(s.x, up, i) - loss_one(s.x, dn, i)) / (2 * eps)
                assert abs(g[c, i] - fd) <= 1e-6 * max(np.max(np.abs(g)), 1e-30)
