"""GPU parity of the diagnostic moments (ecsim_diagnostics) against the FP64
oracle: charge density, current without rotation, charge-weighted second
velocity moment. Relative max-norm over each output array, 1e-12 (FP64) and
1e-5 (FP32, oracle fed the FP32 values widened exactly)."""
import numpy as np
import pytest

from tests.gpu_common import dev, host, need_gpu, rel, say, torch

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}
CASES = [((5, 4, 3), 7), ((2, 2, 2), 5), ((1, 3, 2), 6), ((8, 8, 8), 27), ((13, 7, 5), 3), ((4, 4, 4), 130)]


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


def species_and_reference(E, I, p, prec):
    if prec == "f64":
        sp = [E.Species.from_f64(s.qom, s.x, s.v, s.q) for s in p.species]
        ref = [(s.x, s.v, s.q) for s in p.species]
        return sp, ref, torch.float64
    st = I.to_f32_state(p)
    sp = [E.Species.from_f32(s.qom, f["cell"], f["off"], f["v"], f["q"]) for s, f in zip(p.species, st)]
    ref = [(f["x64"], f["v64"], f["q64"]) for f in st]
    return sp, ref, torch.float32


def oracle_diag(O, p, ref):
    rho, Jd, P = np.zeros(p.nn), np.zeros((3, p.nn)), np.zeros((6, p.nn))
    for x, v, q in ref:
        O.diagnostics(p.n, p.h, x, v, q, rho, Jd, P)
    return rho, Jd, P


def outputs(nn, tdt):
    return (torch.full((nn,), 7.0, dtype=tdt, device="cuda"), torch.full((3, nn), 7.0, dtype=tdt, device="cuda"),
            torch.full((6, nn), 7.0, dtype=tdt, device="cuda"))


def check(out, refs, tol):
    for a, b in zip(out, refs):
        assert rel(host(a), b) < tol


def grouped(E, grid, sp):
    out = []
    for s in sp:
        d = s.empty_like()
        E.sort(grid, s, d, torch.empty(grid.nn + 1, dtype=torch.int32, device="cuda"))
        out.append(d)
    return out


@pytest.mark.parametrize("n,ppc", CASES)
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_diagnostics_any_order(E, O, I, prec, n, ppc):
    say("diagnostics any order", prec, n, ppc)
    p = I.uniform_plasma(700, n, ppc)
    grid = E.Grid(p.n, p.h, p.dt)
    sp, ref, tdt = species_and_reference(E, I, p, prec)
    out = outputs(p.nn, tdt)
    E.diagnostics(grid, sp, *out)
    check(out, oracle_diag(O, p, ref), TOL[prec])


@pytest.mark.parametrize("n,ppc", CASES)
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_diagnostics_grouped(E, O, I, prec, n, ppc):
    """The tiled kernel over cell-grouped particles (cells of more than 64 included)."""
    say("diagnostics grouped", prec, n, ppc)
    p = I.uniform_plasma(710, n, ppc)
    grid = E.Grid(p.n, p.h, p.dt)
    sp, ref, tdt = species_and_reference(E, I, p, prec)
    out = outputs(p.nn, tdt)
    E.diagnostics(grid, grouped(E, grid, sp), *out, flags=E.SORTED)
    check(out, oracle_diag(O, p, ref), TOL[prec])


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_diagnostics_stale_grouping_and_accumulate(E, O, I, prec):
    """Particles moved after grouping (many out of their range's cell) are still
    counted; a second call with ECSIM_ACCUMULATE adds to the first."""
    say("diagnostics stale", prec)
    p = I.uniform_plasma(720, (6, 5, 4), 11)
    for s in p.species:
        s.v = s.v * 30.0
    grid = E.Grid(p.n, p.h, p.dt)
    sp, _, tdt = species_and_reference(E, I, p, prec)
    sp = grouped(E, grid, sp)
    rng = np.random.default_rng(721)
    En = dev(1e-2 * rng.standard_normal((3, p.nn)), tdt)
    BN = dev(0.2 * rng.standard_normal((3, p.nn)), tdt)
    for s in sp:
        E.move(grid, s, En, BN)        # the cell_start of each species is now stale
    ref = []
    for s in sp:
        x = host(s.pos).astype(np.float64)
        if prec == "f32":
            x = I.decode_f32(host(s.cell), host(s.pos), p.n, p.h)
        q = host(s.q).astype(np.float64) if s.q is not None else np.full(s.np, float(s.q_const))
        if prec == "f32":
            q = q.astype(np.float32).astype(np.float64)
        ref.append((x, host(s.vel).astype(np.float64), q))
    out = outputs(p.nn, tdt)
    E.diagnostics(grid, sp, *out, flags=E.SORTED)
    refs = oracle_diag(O, p, ref)
    check(out, refs, TOL[prec])
    E.diagnostics(grid, sp, *out, flags=E.SORTED | E.ACCUMULATE)
    check(out, [2 * r for r in refs], TOL[prec])


def test_diagnostics_empty_species(E, I):
    say("diagnostics empty")
    grid = E.Grid((3, 3, 3), (0.5,) * 3, 0.1)
    sp = E.Species.from_f64(-1.0, np.zeros((3, 0)), np.zeros((3, 0)), 1.0)
    out = outputs(27, torch.float64)
    E.diagnostics(grid, [sp], *out)
    assert all(np.all(host(a) == 0) for a in out)
