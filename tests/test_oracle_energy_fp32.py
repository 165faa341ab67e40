"""The FP32 form's one-way energy drift, found and pinned on the CPU.

The scheme conserves the total energy of the particles it integrates
(Secs. I-II: theta = 1/2, the same alpha_p and W_pN in moments and mover). The
FP32 kernels carry beta_s = (q/m)_s dt / 2 as an FP32 constant, so they
integrate particles whose charge-to-mass ratio is 2 beta_s / dt, which differs
from (q/m)_s by the FP32 rounding of beta_s (1.5e-8 relative for q/m = -1 and
dt = 0.1, 4.7e-8 for q/m = 1/25). Energy is still exchanged exactly between
those particles and the fields, but a kinetic energy summed with the masses
q_p / (q/m)_s misstates every exchange by that relative amount, and the
exchange has one sign over many steps, so the total drifts one way. Here the
FP64 oracle runs the scheme on a small double Harris sheet with the FP32
form's charge-to-mass ratios: with the kinetic energy of the masses the
particles actually have, the total is conserved to rounding; with the nominal
masses it drifts one way, about 5e-12 per step here.
"""
import numpy as np
import pytest


def _run(O, p, nsteps, qom_push, qom_energy):
    x = [s.x.copy() for s in p.species]
    v = [s.v.copy() for s in p.species]
    E, BC = p.E.copy(), p.B_C.copy()

    def total(v, E, BC):
        K = sum(O.kinetic(vv, s.q, qe) for s, vv, qe in zip(p.species, v, qom_energy))
        return K + O.field_energy(p.n, p.h, E) + O.field_energy(p.n, p.h, BC)

    e0 = total(v, E, BC)
    drift = []
    for _ in range(nsteps):
        BN = O.centres_to_nodes(p.n, BC)
        J = np.zeros((3, p.nn))
        M27 = np.zeros((27, 9, p.nn))
        for s, xx, vv, qp in zip(p.species, x, v, qom_push):
            O.moments(p.n, p.h, p.dt, xx, vv, s.q, qp, BN, J, M27)
        sol = O.field_solve(p.n, p.h, p.dt, M27, J, E, BC, 1e-10, 30, 1000)
        for i, (s, qp) in enumerate(zip(p.species, qom_push)):
            x[i], v[i] = O.move(p.n, p.h, p.dt, x[i], v[i], qp, sol["E_theta"], BN)
        E, BC = sol["E_next"], sol["BC_next"]
        drift.append((total(v, E, BC) - e0) / e0)
    return np.array(drift)


@pytest.mark.slow
def test_fp32_beta_rounding_is_the_one_way_energy_drift(oracle, inputs):
    O, I = oracle, inputs
    p = I.harris(n=(32, 16, 2), ppc=8)
    qom = [s.qom for s in p.species]
    # the charge-to-mass ratio the FP32 kernels integrate: 2 fp32(beta) / dt
    qom32 = [float(np.float32(q * p.dt / 2.0)) * 2.0 / p.dt for q in qom]
    assert all(0 < abs(a - q) / abs(q) < 6e-8 for a, q in zip(qom32, qom))
    ref = _run(O, p, 10, qom, qom)
    nominal = _run(O, p, 10, qom32, qom)
    consistent = _run(O, p, 10, qom32, qom32)
    # FP64 scheme and FP32 charge-to-mass ratios with matching masses: conserved
    assert np.max(np.abs(ref)) < 1e-13
    assert np.max(np.abs(consistent)) < 1e-13
    # nominal masses: a one-way drift far above rounding, growing every step
    d = np.diff(np.concatenate([[0.0], nominal]))
    assert np.all(np.sign(d) == np.sign(d[-1]))
    assert abs(nominal[-1]) > 1e-11
    # its size is the rounding of beta times the work the field did on each species
    assert abs(nominal[-1]) > 100 * np.max(np.abs(consistent))
