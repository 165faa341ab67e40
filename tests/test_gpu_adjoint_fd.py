"""The adjoint of mover -> moments (ecsim_moments_backward through the mover)
at the differentiation workload's full size, against central finite
differences of the FP64 oracle.

Workload: 32^3 cells, 27 particles per cell per species (1,769,472
particles), E ~ N(0, 1e-3), B = B0 + N(0, 1e-3) per component (seeded). Loss
L = <gJ, J> + <gM, M> with seeded N(0, 1) weights, J and M deposited at the
moved positions with the same B. Checked, in the FP64 and the FP32 form:

* dL/dx and dL/dv of 64 seeded particles: a central difference (step 1e-6)
  of each particle's own loss, the oracle moving and depositing it;
* dL/dE and dL/dB at 64 seeded nodes: a central difference of the summed
  loss of every particle that starts within two cells of the node (a node is
  reached only through the stencils before and after a move of far less than
  one cell).

Bound: |adjoint - difference| <= 1e-6 (FP64) or 1e-5 (FP32, the oracle fed the
FP32 values widened) times the largest magnitude among the checked entries.
"""
import numpy as np
import pytest

from tests.gpu_common import dev, host, need_gpu, round32, say, torch

pytestmark = pytest.mark.gpu

EPS = 1e-6
NPART = 64
NNODES = 64
TOL = {"f64": 1e-6, "f32": 1e-5}


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


def near_cells(n, g):
    nx, ny, nz = n
    gx, gy, gz = g % nx, (g // nx) % ny, g // (nx * ny)
    near = np.zeros(nx * ny * nz, dtype=bool)
    for dz in range(-2, 2):
        for dy in range(-2, 2):
            for dx in range(-2, 2):
                near[(gx + dx) % nx + nx * (((gy + dy) % ny) + ny * ((gz + dz) % nz))] = True
    return near


@pytest.mark.timeout(300)
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_adjoint_against_finite_differences(E, O, prec):
    from paper_2603_16624_amd import inputs as I
    p = I.config3()
    say("adjoint vs finite differences", prec, p.name)
    BN = O.centres_to_nodes(p.n, p.B_C)
    En = p.E
    gJ, gM = I.loss_weights(p.nn)
    grid = E.Grid(p.n, p.h, p.dt)
    if prec == "f64":
        tdt = torch.float64
        states = [(s.x, s.v, s.q) for s in p.species]
        sp = [E.Species.from_f64(s.qom, s.x, s.v, s.q) for s in p.species]
    else:
        tdt = torch.float32
        fs = I.to_f32_state(p)
        states = [(f["x64"], f["v64"], f["q64"]) for f in fs]
        sp = [E.Species.from_f32(s.qom, f["cell"], f["off"], f["v"], f["q"]) for s, f in zip(p.species, fs)]
        En, BN, gJ, gM = round32(En), round32(BN), round32(gJ), round32(gM)
    Ed, Bd, gJd, gMd = dev(En, tdt), dev(BN, tdt), dev(gJ, tdt), dev(gM, tdt)
    gE = torch.zeros((3, p.nn), dtype=tdt, device="cuda")
    gB = torch.zeros((3, p.nn), dtype=tdt, device="cuda")
    gxs, gvs = [], []
    for s in sp:
        gx, gv = torch.empty_like(s.pos), torch.empty_like(s.vel)
        E.moments_backward(grid, s, Ed, Bd, gJd, gMd, gx, gv, gE, gB, through_mover=True)
        gxs.append(host(gx).astype(np.float64))
        gvs.append(host(gv).astype(np.float64))
    gE, gB = host(gE).astype(np.float64), host(gB).astype(np.float64)
    tol = TOL[prec]
    rng = np.random.default_rng(3008)   # config 3, purpose 8: the finite-difference sample

    def loss(s, x, v, q, Ef=En, Bf=BN):
        return O.particle_loss(p.n, p.h, p.dt, x, v, q, s.qom, Ef, Bf, gJ, gM)

    # particles: 32 per species
    got, ref = [], []
    for s, (x, v, q), gx, gv in zip(p.species, states, gxs, gvs):
        for i in rng.choice(s.np, size=NPART // 2, replace=False):
            xi, vi, qi = x[:, i:i + 1].copy(), v[:, i:i + 1].copy(), q[i:i + 1]
            for c in range(6):
                up, dn = (xi.copy(), xi.copy()) if c < 3 else (vi.copy(), vi.copy())
                up[c % 3] += EPS
                dn[c % 3] -= EPS
                if c < 3:
                    fd = (loss(s, up, vi, qi)[0] - loss(s, dn, vi, qi)[0]) / (2 * EPS)
                    got.append(gx[c, i])
                else:
                    fd = (loss(s, xi, up, qi)[0] - loss(s, xi, dn, qi)[0]) / (2 * EPS)
                    got.append(gv[c - 3, i])
                ref.append(fd)
    got, ref = np.array(got), np.array(ref)
    assert np.max(np.abs(got - ref)) <= tol * np.max(np.abs(ref))

    # nodes: every particle starting within two cells of the node
    cells = []
    for x, _, _ in states:
        ijk = [np.floor(x[d] / p.h[d]).astype(np.int64) for d in range(3)]
        cells.append(ijk[0] + p.n[0] * (ijk[1] + p.n[1] * ijk[2]))
    got, ref = [], []
    for g in rng.choice(p.nn, size=NNODES, replace=False):
        near = near_cells(p.n, g)
        sel = [(s, x[:, near[c]], v[:, near[c]], q[near[c]]) for s, (x, v, q), c in zip(p.species, states, cells)]
        for f in range(6):
            tot = 0.0
            for sgn in (1.0, -1.0):
                Ef, Bf = En.copy(), BN.copy()
                (Ef if f < 3 else Bf)[f % 3, g] += sgn * EPS
                tot += sgn * sum(loss(s, x, v, q, Ef, Bf).sum() for s, x, v, q in sel)
            ref.append(tot / (2 * EPS))
            got.append(gE[f, g] if f < 3 else gB[f - 3, g])
    got, ref = np.array(got), np.array(ref)
    assert np.max(np.abs(got - ref)) <= tol * np.max(np.abs(ref))
