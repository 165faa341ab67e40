"""Shared helpers of the GPU parity tests: device transfer and case printing."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype=dtype, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.max(np.abs(b)) if b.size else 0.0
    if den == 0.0:
        return float(np.max(np.abs(a))) if a.size else 0.0
    return float(np.max(np.abs(a - b)) / den)


def periodic_rel(a, b, L):
    worst = 0.0
    for d in range(3):
        diff = np.asarray(a[d], dtype=np.float64) - np.asarray(b[d], dtype=np.float64)
        diff = diff - L[d] * np.round(diff / L[d])
        if diff.size:
            worst = max(worst, float(np.max(np.abs(diff))) / L[d])
    return worst


def round32(a):
    """FP32 rounding of a host array, returned as FP64 (the values the FP32 kernels see)."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def kinetic0(E, O, p, prec, vs=None, qs=None):
    """Kinetic energy of a plasma's species with the masses the kernels of
    precision prec integrate, m_p = q_p / ecsim_species_qom (in FP32 the
    species' beta is an FP32 constant)."""
    P = E.F64 if prec == "f64" else E.F32
    vs = [s.v for s in p.species] if vs is None else vs
    qs = [s.q for s in p.species] if qs is None else qs
    return sum(O.kinetic(v, q, E.species_qom(P, s.qom, p.dt)) for s, v, q in zip(p.species, vs, qs))


def fp32_drift_bound(p, steps, e0, vs=None, qs=None, nsigma=6.0):
    """Bound on the relative energy drift of the FP32 form over `steps` steps.

    With the masses of kinetic0 the scheme exchanges energy exactly; what the
    FP32 form adds is the rounding of each stored velocity component once per
    step (the update is formed in FP64): an error d with |d| <= u |v_i|,
    u = 2^-24, zero mean and variance at most u^2 v_i^2 / 3, which changes
    the kinetic energy by m_p v . d to first order. Independent over particles
    and steps, the sum has standard deviation at most
    u sqrt(steps * sum_p m_p^2 sum_i v_i^4 / 3); the bound is nsigma of it,
    relative to e0, plus the 1e-10 solver tolerance."""
    u = 2.0 ** -24
    vs = [s.v for s in p.species] if vs is None else vs
    qs = [s.q for s in p.species] if qs is None else qs
    s4 = 0.0
    for s, v, q in zip(p.species, vs, qs):
        m = np.asarray(q, dtype=np.float64) / s.qom * np.ones(v.shape[1])
        s4 += float(np.sum(m * m * np.sum(np.asarray(v, dtype=np.float64) ** 4, axis=0)))
    return nsigma * u * np.sqrt(steps * s4 / 3.0) / e0 + 1e-10
