"""GPU checks of the boundary's conventions: the non-finite flag, and sizes
past the single-level scan (grids of more than 2^20 cells).

Non-finite values: a NaN placed in one node of E reaches the velocities of
the particles around that node; the mover records it in the device's flag,
ecsim_check_finite reports ECSIM_ENONFINITE once and clears the flag. The
same for a NaN charge in the moment gather and a NaN in B in the fused pass.
NaN inputs cannot send an index out of bounds: a NaN offset or position
converts to cell 0 of its dimension in the stencil and the push keeps the
cell index in range.

Large grids: the exclusive scan over cells (and over species x cells when
regrouping) takes more than one level of 1024-value tiles beyond 2^20
entries; a counting sort and a regrouping fused pass on 1,179,648 cells check
the ranges exactly and J-hat and M against the oracle.
"""
import numpy as np
import pytest

from tests.gpu_common import dev, host, need_gpu, rel, round32, say, torch

pytestmark = pytest.mark.gpu


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


def expect_nonfinite(E):
    with pytest.raises(E.EcsimError) as ex:
        E.check_finite()
    assert ex.value.status == E.ENONFINITE
    E.check_finite()   # cleared: a second check passes


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_nan_in_E_sets_the_flag(E, I, prec):
    say("nonfinite flag, NaN in E", prec)
    p = I.uniform_plasma(501, (6, 5, 4), 4)
    grid = E.Grid(p.n, p.h, p.dt)
    tdt = torch.float64 if prec == "f64" else torch.float32
    if prec == "f64":
        sp = [E.Species.from_f64(s.qom, s.x, s.v, s.q) for s in p.species]
    else:
        sp = [E.Species.from_f32(s.qom, f["cell"], f["off"], f["v"], f["q"])
              for s, f in zip(p.species, I.to_f32_state(p))]
    En = np.zeros((3, p.nn))
    BN = np.zeros((3, p.nn))
    BN[2] = 0.2
    E.check_finite()   # nothing recorded before
    for s in sp:
        E.move(grid, s, dev(En, tdt), dev(BN, tdt))
    E.check_finite()   # finite fields: nothing recorded
    En[1, 17] = np.nan
    for s in sp:
        E.move(grid, s, dev(En, tdt), dev(BN, tdt))
    expect_nonfinite(E)
    # the asynchronous read: 1, then 0 after the clear
    flag = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    for s in sp:
        E.move(grid, s, dev(En, tdt), dev(BN, tdt))
    E.nonfinite_read(flag)
    assert int(host(flag)[0]) == 1
    E.nonfinite_read(flag)
    assert int(host(flag)[0]) == 0
    E.check_finite()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_nan_charge_in_moments_and_nan_B_in_fused_pass(E, I, prec):
    say("nonfinite flag, moments and fused pass", prec)
    p = I.uniform_plasma(502, (8, 4, 4), 6)
    grid = E.Grid(p.n, p.h, p.dt)
    tdt = torch.float64 if prec == "f64" else torch.float32
    if prec == "f64":
        sp = [E.Species.from_f64(s.qom, s.x, s.v, s.q) for s in p.species]
    else:
        sp = [E.Species.from_f32(s.qom, f["cell"], f["off"], f["v"], f["q"])
              for s, f in zip(p.species, I.to_f32_state(p))]
    BN = np.zeros((3, p.nn))
    BN[2] = 0.2
    J = torch.empty((3, p.nn), dtype=tdt, device="cuda")
    M = torch.empty((14, 9, p.nn), dtype=tdt, device="cuda")
    E.check_finite()
    q = torch.full((sp[0].np,), sp[0].q_const, dtype=tdt, device="cuda")
    q[5] = float("nan")
    bad = E.Species(sp[0].prec, sp[0].qom, sp[0].pos, sp[0].vel, sp[0].cell, q, 0.0)
    E.moments(grid, [bad, sp[1]], dev(BN, tdt), J, M)
    expect_nonfinite(E)
    # the grouped (tiled) deposit and the fused pass
    grouped = []
    for s in sp:
        d = s.empty_like()
        E.sort(grid, s, d, torch.empty(grid.nn + 1, dtype=torch.int32, device="cuda"))
        grouped.append(d)
    E.moments(grid, grouped, dev(BN, tdt), J, M, flags=E.SORTED)
    E.check_finite()
    Bbad = BN.copy()
    Bbad[0, 3] = np.nan
    E.move_moments(grid, grouped, dev(np.zeros((3, p.nn)), tdt), dev(Bbad, tdt), dev(BN, tdt), J, M)
    expect_nonfinite(E)


def test_sort_beyond_one_scan_level(E, I):
    """ecsim_sort on 1,179,648 cells (1152 tiles of the cell scan)."""
    say("sort, 128x96x96 cells")
    n = (128, 96, 96)
    nn = n[0] * n[1] * n[2]
    p = I.uniform_plasma(503, n, 1)
    s = p.species[0]
    st = I.to_f32_state(p)[0]
    grid = E.Grid(p.n, p.h, p.dt)
    src = E.Species.from_f32(s.qom, st["cell"], st["off"], st["v"], st["q"])
    # a random order, so that the sort has work to do
    perm = np.random.default_rng(5).permutation(src.np)
    src = E.Species.from_f32(s.qom, st["cell"][perm], st["off"][:, perm], st["v"][:, perm], st["q"])
    dst = src.empty_like()
    cs = torch.empty(nn + 1, dtype=torch.int32, device="cuda")
    E.sort(grid, src, dst, cs)
    want = np.concatenate([[0], np.cumsum(np.bincount(st["cell"], minlength=nn))])
    assert np.array_equal(host(cs).astype(np.int64), want)
    cells = host(dst.cell).astype(np.int64)
    assert np.array_equal(cells, np.repeat(np.arange(nn), np.diff(want)))


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_regroup_beyond_one_scan_level(E, O, I, prec):
    """A regrouping fused pass on 128x96x96 cells x 2 species x 2 particles per
    cell (2,359,296 species x cells entries: three scan levels): the new
    ranges exactly, J-hat and M against the oracle."""
    say("regroup, 128x96x96 cells", prec)
    n = (128, 96, 96)
    p = I.uniform_plasma(504, n, 2)
    rng = np.random.default_rng(505)
    for s in p.species:
        s.v = s.v * 5.0   # a few percent of the particles change cell
    En = 1e-3 * rng.standard_normal((3, p.nn))
    BN = np.array([[0.0], [0.0], [0.2]]) + 0.01 * rng.standard_normal((3, p.nn))
    Bn = BN + 1e-3 * rng.standard_normal((3, p.nn))
    grid = E.Grid(p.n, p.h, p.dt)
    if prec == "f64":
        sp = [E.Species.from_f64(s.qom, s.x, s.v, s.q) for s in p.species]
        xs, vs, qs = [s.x for s in p.species], [s.v for s in p.species], [s.q for s in p.species]
        Ec, Bc, Bnc, tdt, tol = En, BN, Bn, torch.float64, 1e-12
    else:
        st = I.to_f32_state(p)
        sp = [E.Species.from_f32(s.qom, f["cell"], f["off"], f["v"], f["q"]) for s, f in zip(p.species, st)]
        xs, vs, qs = [f["x64"] for f in st], [f["v64"] for f in st], [f["q64"] for f in st]
        Ec, Bc, Bnc, tdt, tol = round32(En), round32(BN), round32(Bn), torch.float32, 1e-5
    grouped = []
    for s in sp:
        d = s.empty_like()
        E.sort(grid, s, d, torch.empty(grid.nn + 1, dtype=torch.int32, device="cuda"))
        grouped.append(d)
    dst = [s.empty_like() for s in grouped]
    J = torch.empty((3, p.nn), dtype=tdt, device="cuda")
    M = torch.empty((14, 9, p.nn), dtype=tdt, device="cuda")
    E.move_moments_regroup(grid, grouped, dst, dev(Ec, tdt), dev(Bc, tdt), dev(Bnc, tdt), J, M)
    Jo = np.zeros((3, p.nn))
    M27 = np.zeros((27, 9, p.nn))
    for s, x, v, q, d in zip(p.species, xs, vs, qs, dst):
        x1, v1 = O.move(p.n, p.h, p.dt, x, v, s.qom, Ec, Bc)
        O.moments(p.n, p.h, p.dt, x1, v1, q, s.qom, Bnc, Jo, M27)
        ijk = [np.floor(x1[k] / p.h[k]).astype(np.int64) for k in range(3)]
        cells = ijk[0] + p.n[0] * (ijk[1] + p.n[1] * ijk[2])
        want = np.concatenate([[0], np.cumsum(np.bincount(cells, minlength=p.nn))])
        got = host(d.cell_start).astype(np.int64)
        if prec == "f64":
            assert np.array_equal(got, want)
        else:
            # cells from the FP32 state; a particle within rounding of a face may differ
            assert got[-1] == want[-1] and np.abs(got - want).max() <= 2
    assert rel(host(J), Jo) < tol
    Mo = O.m14(p.n, M27)
    del M27
    assert rel(host(M), Mo) < tol
    E.check_finite()
