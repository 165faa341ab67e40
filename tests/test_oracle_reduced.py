"""Pins of the oracle's reduced (1D and 2D) runs: a dimension of one cell is
ignorable and the mover keeps positions along it (the fixPosition step of
Sec. III), while velocities keep all three components."""
import numpy as np
import pytest

H = (0.5, 0.5, 0.5)
DT = 0.1


def _lone(oracle, n, steps, x0, v0, B):
    nn = int(np.prod(n))
    E = np.zeros((3, nn))
    BN = np.tile(np.asarray(B, dtype=float)[:, None], (1, nn))
    x, v = np.array(x0, dtype=float)[:, None], np.array(v0, dtype=float)[:, None]
    xs = [x]
    for _ in range(steps):
        x, v = oracle.move(n, H, DT, x, v, -1.0, E, BN)
        xs.append(x)
    return np.hstack(xs), v


@pytest.mark.parametrize("reduced,fixed", [((16, 16, 1), (2,)), ((16, 1, 1), (1, 2)), ((1, 16, 1), (0, 2))])
def test_reduced_dimensions_keep_position(oracle, reduced, fixed):
    """In uniform fields the velocity history does not depend on position, so a
    reduced run and a full 3D run move alike along the resolved dimensions (to
    rounding: the gathered field is a weighted sum whose weights differ); along
    the single-cell ones the reduced run stays put."""
    x0, v0, B = (3.3, 2.1, 0.27), (0.05, -0.04, 0.06), (0.1, 0.2, 0.3)
    xr, vr = _lone(oracle, reduced, 60, x0, v0, B)
    xf, vf = _lone(oracle, (16, 16, 16), 60, x0, v0, B)
    assert np.max(np.abs(vr - vf)) <= 1e-14
    for d in range(3):
        if d in fixed:
            assert np.all(xr[d] == x0[d])
            assert np.ptp(xf[d]) > 0.1          # the 3D run does move along it
        else:
            assert np.max(np.abs(xr[d] - xf[d])) <= 1e-13


def test_energy_conservation_2d(oracle, inputs):
    """A 2D run (8 x 8 x 1 cells) conserves total energy to the GMRES tolerance."""
    p = inputs.uniform_plasma(90, (8, 8, 1), 27)
    z0 = [s.x[2].copy() for s in p.species]
    state, hist = oracle.run_steps(p, 8, tol=1e-10)
    e0 = hist[0]["total"]
    drift = max(abs(h["total"] - e0) / e0 for h in hist)
    assert drift <= 1e-10
    assert abs(hist[-1]["K"] - hist[0]["K"]) > 1e-7 * e0
    for xs, z in zip(state["x"], z0):
        assert np.array_equal(xs[2], z)
