"""The differentiable mover -> moment gather (paper_2603_16624_amd.autograd)
against the oracle: J and M of the moved species (Eqs. 1, 3 after Eqs. 4, 5,
8), and the gradients of a seeded weighted loss <gJ, J> + <gM, M> with
respect to the pre-move positions and velocities and the grid fields E and B
(the oracle's dual-number derivative). Relative max-norm 1e-12 (FP64) and
1e-5 (FP32, the oracle fed the FP32 values widened; position gradients with
respect to the in-cell offsets, i.e. h times d/dx)."""
import numpy as np
import pytest

from tests.gpu_common import dev, host, need_gpu, rel, round32, say, torch

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}


@pytest.fixture(scope="module")
def A():
    need_gpu()
    from paper_2603_16624_amd import autograd, ecsim
    ecsim.lib()
    return autograd


@pytest.fixture(scope="module")
def O():
    from oracle import oracle
    oracle.lib()
    return oracle


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n,ppc", [((5, 4, 4), 4), ((3, 2, 3), 6)])
def test_autograd_move_moments(A, O, prec, n, ppc):
    from paper_2603_16624_amd import ecsim as E
    from paper_2603_16624_amd import inputs as I
    say("autograd move->moments", prec, n, ppc)
    p = I.uniform_plasma(470, n, ppc)
    rng = np.random.default_rng(471)
    En = 1e-2 * rng.standard_normal((3, p.nn))
    BN = np.array([[0.0], [0.05], [0.2]]) + 0.05 * rng.standard_normal((3, p.nn))
    gJ = rng.standard_normal((3, p.nn))
    gM = rng.standard_normal((14, 9, p.nn))
    grid = E.Grid(p.n, p.h, p.dt)
    s = p.species[0]
    s.v = s.v * 10.0                      # some particles leave their cell
    tol = TOL[prec]
    if prec == "f64":
        tdt = torch.float64
        x, v, q = s.x, s.v, s.q
        Ec, Bc, gJc, gMc = En, BN, gJ, gM
        pos = dev(x, tdt).requires_grad_()
        cell = None
        qarg = dev(q, tdt)                # a per-particle charge tensor
    else:
        tdt = torch.float32
        st = I.to_f32_state(p)[0]
        x, v, q = st["x64"], st["v64"], st["q64"]
        Ec, Bc, gJc, gMc = round32(En), round32(BN), round32(gJ), round32(gM)
        pos = dev(st["off"], tdt).requires_grad_()
        cell = torch.as_tensor(np.ascontiguousarray(st["cell"], dtype=np.int32)).to("cuda")
        qarg = float(q[0])                # one charge for all
    vel = dev(v, tdt).requires_grad_()
    Et = dev(Ec, tdt).requires_grad_()
    Bt = dev(Bc, tdt).requires_grad_()
    pos0 = host(pos).copy()
    J, M = A.move_moments(grid, s.qom, qarg, pos, vel, Et, Bt, cell)
    # forward against the oracle's move then moments (the same B)
    x1, v1 = O.move(p.n, p.h, p.dt, x, v, s.qom, Ec, Bc)
    Jo, M27 = O.moments(p.n, p.h, p.dt, x1, v1, q, s.qom, Bc)
    assert rel(host(J), Jo) < tol
    assert rel(host(M), O.m14(p.n, M27)) < tol
    assert np.array_equal(host(pos), pos0)          # the inputs are not modified
    loss = (J * dev(gJc, tdt)).sum() + (M * dev(gMc, tdt)).sum()
    gpos, gvel, gE, gB = torch.autograd.grad(loss, [pos, vel, Et, Bt])
    gxo, gvo, gEo, gBo = O.grad(p.n, p.h, p.dt, x, v, q, s.qom, Ec, Bc, gJc, gMc)
    if prec == "f32":
        gxo = gxo * np.asarray(p.h)[:, None]
    assert rel(host(gpos), gxo) < tol
    assert rel(host(gvel), gvo) < tol
    assert rel(host(gE), gEo) < tol
    assert rel(host(gB), gBo) < tol


def test_gradcheck_small_grid(A):
    """torch.autograd.gradcheck of the FP64 mover -> moments (3^3 grid, 20
    particles, perturbed fields): the hand-written adjoint's vector-Jacobian
    products against torch's central differences of the library's forward,
    for the positions, the velocities and the grid fields E and B. Particles
    within 1e-4 of a cell face before or after the move are redrawn (the
    weights have kinks there)."""
    from paper_2603_16624_amd import ecsim as E
    say("gradcheck 3^3 x 20 particles")
    n, h, dt = (3, 3, 3), (0.5, 0.5, 0.5), 0.1
    L = np.array([n[d] * h[d] for d in range(3)])
    rng = np.random.default_rng(4800)
    nn = 27
    En = 1e-2 * rng.standard_normal((3, nn))
    BN = np.array([[0.02], [0.05], [0.2]]) + 0.05 * rng.standard_normal((3, nn))
    grid = E.Grid(n, h, dt)
    qom, q = -1.0, 3.7e-4

    def clear_of_faces(x, v):
        from oracle import oracle as O
        x1, _ = O.move(n, h, dt, x, v, qom, En, BN)
        ok = np.ones(x.shape[1], dtype=bool)
        for pos in (x, x1):
            xi = pos / np.asarray(h)[:, None]
            frac = xi - np.floor(xi)
            ok &= np.all((frac > 1e-4) & (frac < 1 - 1e-4), axis=0)
        return ok

    x = np.zeros((3, 0))
    v = np.zeros((3, 0))
    while x.shape[1] < 20:
        xc = rng.random((3, 64)) * L[:, None]
        vc = 0.3 * rng.standard_normal((3, 64))
        keep = clear_of_faces(xc, vc)
        x = np.concatenate([x, xc[:, keep]], axis=1)
        v = np.concatenate([v, vc[:, keep]], axis=1)
    x, v = x[:, :20], v[:, :20]
    pos = dev(x).requires_grad_()
    vel = dev(v).requires_grad_()
    Et = dev(En).requires_grad_()
    Bt = dev(BN).requires_grad_()
    fn = lambda p_, v_, e_, b_: A.move_moments(grid, qom, q, p_, v_, e_, b_)
    assert torch.autograd.gradcheck(fn, (pos, vel, Et, Bt), eps=1e-6, atol=1e-8, rtol=1e-5)
