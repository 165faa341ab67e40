"""ecsim_move_moments_noalloc: the fused pass on the library's static device
scratch, against ecsim_move_moments with a caller's workspace.

Two calls in a row on one device, the second with fewer particles on a
smaller grid (the scratch keeps the first call's contents). Each call's moved
particles must equal those of ecsim_move_moments bit for bit (the mover is
the same arithmetic), and J and M must match it and the oracle within the
parity tolerances (the deposit's atomics make their summation order vary).
"""
import numpy as np
import pytest

from tests.gpu_common import dev, host, need_gpu, rel, round32, say, torch

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}


@pytest.fixture(scope="module")
def E():
    need_gpu()
    from paper_2603_16624_amd import ecsim
    return ecsim


@pytest.fixture(scope="module")
def O():
    from oracle import oracle
    return oracle


@pytest.fixture(scope="module")
def I():
    from paper_2603_16624_amd import inputs
    return inputs


def _species(E, I, p, prec):
    if prec == "f64":
        sp = [E.Species.from_f64(s.qom, s.x, s.v, s.q) for s in p.species]
        return sp, [s.x for s in p.species], [s.v for s in p.species], [s.q for s in p.species]
    st = I.to_f32_state(p)
    sp = [E.Species.from_f32(s.qom, f["cell"], f["off"], f["v"], f["q"]) for s, f in zip(p.species, st)]
    return sp, [f["x64"] for f in st], [f["v64"] for f in st], [f["q64"] for f in st]


def _grouped(E, grid, sp):
    out = []
    for s in sp:
        d = s.empty_like()
        E.sort(grid, s, d, torch.empty(grid.nn + 1, dtype=torch.int32, device="cuda"))
        out.append(d)
    return out


def _state(s):
    parts = [host(s.pos), host(s.vel)]
    if s.cell is not None:
        parts.append(host(s.cell).astype(np.float64)[None, :])
    return np.concatenate(parts, axis=0)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_noalloc_matches_workspace_call(E, O, I, prec):
    tdt = torch.float64 if prec == "f64" else torch.float32
    for call, (n, ppc, seed) in enumerate((((10, 8, 6), 20, 61), ((5, 4, 3), 9, 62))):
        say("move_moments_noalloc", prec, "call", call, n, ppc)
        p = I.uniform_plasma(seed, n, ppc)
        rng = np.random.default_rng(seed + 1000)
        En = 1e-2 * rng.standard_normal((3, p.nn))
        BN = np.array([[0.02], [-0.03], [0.2]]) + 0.05 * rng.standard_normal((3, p.nn))
        Bnext = BN + 0.01 * rng.standard_normal(BN.shape)
        for s in p.species:
            s.v = s.v * 8.0   # many particles leave their cell: the stray list is used
        if prec == "f32":
            En, BN, Bnext = round32(En), round32(BN), round32(Bnext)
        grid = E.Grid(p.n, p.h, p.dt)
        sp, xs, vs, qs = _species(E, I, p, prec)
        a = _grouped(E, grid, sp)
        b = [s.clone() for s in a]
        fields = [dev(f, tdt) for f in (En, BN, Bnext)]
        Ja = torch.empty((3, p.nn), dtype=tdt, device="cuda")
        Ma = torch.empty((14, 9, p.nn), dtype=tdt, device="cuda")
        Jb = torch.full((3, p.nn), 7.0, dtype=tdt, device="cuda")
        Mb = torch.full((14, 9, p.nn), 7.0, dtype=tdt, device="cuda")
        kea = torch.zeros(1, dtype=torch.float64, device="cuda")
        keb = torch.zeros(1, dtype=torch.float64, device="cuda")
        E.move_moments(grid, a, *fields, Ja, Ma, kea)
        E.move_moments_noalloc(grid, b, *fields, Jb, Mb, keb)
        torch.cuda.synchronize()
        for sa, sb in zip(a, b):
            assert np.array_equal(_state(sa), _state(sb))
        assert rel(host(Jb), host(Ja)) < TOL[prec]
        assert rel(host(Mb), host(Ma)) < TOL[prec]
        assert abs(host(keb)[0] - host(kea)[0]) <= 1e-12 * abs(host(kea)[0])
        # and the oracle: move, then the moments at the new positions with B_next
        Jo = np.zeros((3, p.nn))
        M27 = np.zeros((27, 9, p.nn))
        for s, x, v, q in zip(p.species, xs, vs, qs):
            x1, v1 = O.move(p.n, p.h, p.dt, x, v, s.qom, En, BN)
            O.moments(p.n, p.h, p.dt, x1, v1, q, s.qom, Bnext, Jo, M27)
        assert rel(host(Jb), Jo) < TOL[prec]
        assert rel(host(Mb), O.m14(p.n, M27)) < TOL[prec]
