"""ctypes front end of the FP64 CPU oracle (test infrastructure only).

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may import this module. It builds ``liboracle.so`` from ``ecsim_oracle.cpp``
with g++ (plain loops, -O2, no fast-math, no FMA contraction) and wraps each
exported function with numpy arrays. Array layouts: particle positions and
velocities (3, Np); node fields (3, Nn); M27 (27, 9, Nn); M14 (14, 9, Nn).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ecsim_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")

CXXFLAGS = ["-O2", "-std=c++17", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared"]


def build(force: bool = False) -> str:
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", *CXXFLAGS, SRC, "-o", tmp])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = ctypes.CDLL(LIB)
        _declare(_lib)
    return _lib


_d = ctypes.c_double
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_p = ctypes.c_void_p


def _declare(L):
    L.oracle_weights.argtypes = [_p, _p, _p, _p, _p]
    L.oracle_gather.argtypes = [_p, _p, _i64, _p, _p, _p]
    L.oracle_alpha.argtypes = [_p, _d, _p]
    L.oracle_moments.argtypes = [_p, _p, _d, _i64, _p, _p, _p, _d, _d, _p, _p, _p]
    L.oracle_diagnostics.argtypes = [_p, _p, _i64, _p, _p, _p, _d, _p, _p, _p]
    L.oracle_m14_from_m27.argtypes = [_p, _p, _p]
    L.oracle_canonical14.argtypes = [_p]
    L.oracle_mass_apply27.argtypes = [_p, _p, _p, _p]
    L.oracle_move.argtypes = [_p, _p, _d, _i64, _p, _p, _d, _p, _p]
    L.oracle_move_moments_threads.argtypes = [_p, _p, _d, _i64, _p, _p, _p, _d, _d, _p, _p, _p, _p, _p, _i32]
    L.oracle_move_moments_threads.restype = _i32
    L.oracle_curl_C.argtypes = [_p, _p, _p, _p]
    L.oracle_curl_N.argtypes = [_p, _p, _p, _p]
    L.oracle_centres_to_nodes.argtypes = [_p, _p, _p]
    L.oracle_field_operator.argtypes = [_p, _p, _d, _p, _p, _p]
    L.oracle_field_rhs.argtypes = [_p, _p, _d, _p, _p, _p, _p]
    L.oracle_field_solve.argtypes = [_p, _p, _d, _p, _p, _p, _p, _d, ctypes.c_int, ctypes.c_int,
                                     _p, _p, _p, _p]
    L.oracle_field_solve.restype = ctypes.c_int
    L.oracle_kinetic.argtypes = [_i64, _p, _p, _d, _d]
    L.oracle_kinetic.restype = _d
    L.oracle_field_energy.argtypes = [_p, _p, _p]
    L.oracle_field_energy.restype = _d
    L.oracle_grad.argtypes = [_p, _p, _d, _i64, _p, _p, _p, _d, _d, _p, _p, _p, _p, _p, _p, _p, _p]
    L.oracle_particle_loss.argtypes = [_p, _p, _d, _i64, _p, _p, _p, _d, _d, _p, _p, _p, _p, _p]


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _grid(n, h):
    return np.asarray(n, dtype=np.int32), np.asarray(h, dtype=np.float64)


def _q(q):
    """Per-particle charge array or a scalar -> (array or None, scalar)."""
    if np.isscalar(q):
        return None, float(q)
    return _f64(q), 0.0


def canonical14() -> np.ndarray:
    out = np.zeros((14, 3), dtype=np.int32)
    lib().oracle_canonical14(_ptr(out))
    return out


def weights(n, h, x):
    """Lower node per dimension and the 8 weights W_a (a = ax + 2ay + 4az)."""
    ni, hh = _grid(n, h)
    xx = _f64(x)
    lo = np.zeros(3, dtype=np.int64)
    W = np.zeros(8)
    lib().oracle_weights(_ptr(ni), _ptr(hh), _ptr(xx), _ptr(lo), _ptr(W))
    return lo, W


def gather(n, h, x, F):
    ni, hh = _grid(n, h)
    x = _f64(x)
    F = _f64(F)
    out = np.zeros_like(x)
    lib().oracle_gather(_ptr(ni), _ptr(hh), x.shape[1], _ptr(x), _ptr(F), _ptr(out))
    return out


def alpha(B, beta):
    a = np.zeros(9)
    B = _f64(B)
    lib().oracle_alpha(_ptr(B), float(beta), _ptr(a))
    return a.reshape(3, 3)


def moments(n, h, dt, x, v, q, qom, B_node, J=None, M27=None):
    """Accumulates Eq. 1 into J (3, Nn) and Eq. 3 into M27 (27, 9, Nn)."""
    ni, hh = _grid(n, h)
    nn = int(np.prod(n))
    if J is None:
        J = np.zeros((3, nn))
    if M27 is None:
        M27 = np.zeros((27, 9, nn))
    x = _f64(x)
    v = _f64(v)
    qa, qc = _q(q)
    B_node = _f64(B_node)
    lib().oracle_moments(_ptr(ni), _ptr(hh), float(dt), x.shape[1], _ptr(x), _ptr(v), _ptr(qa), qc,
                         float(qom), _ptr(B_node), _ptr(J), _ptr(M27))
    return J, M27


def diagnostics(n, h, x, v, q, rho=None, Jd=None, P=None):
    """Accumulates the diagnostic moments (Sec. III, diagnostics for I/O): rho (Nn,),
    the unrotated current Jd (3, Nn) and the charge-weighted second velocity
    moment P (6, Nn: xx, xy, xz, yy, yz, zz), each divided by the node volume."""
    ni, hh = _grid(n, h)
    nn = int(np.prod(n))
    rho = np.zeros(nn) if rho is None else rho
    Jd = np.zeros((3, nn)) if Jd is None else Jd
    P = np.zeros((6, nn)) if P is None else P
    x = _f64(x)
    v = _f64(v)
    qa, qc = _q(q)
    lib().oracle_diagnostics(_ptr(ni), _ptr(hh), x.shape[1], _ptr(x), _ptr(v), _ptr(qa), qc, _ptr(rho), _ptr(Jd),
                             _ptr(P))
    return rho, Jd, P


def m14(n, M27):
    M27 = _f64(M27)
    ni = np.asarray(n, dtype=np.int32)
    out = np.zeros((14,) + M27.shape[1:])
    lib().oracle_m14_from_m27(_ptr(ni), _ptr(M27), _ptr(out))
    return out


def mass_apply27(n, M27, E):
    ni = np.asarray(n, dtype=np.int32)
    M27 = _f64(M27)
    E = _f64(E)
    y = np.zeros_like(E)
    lib().oracle_mass_apply27(_ptr(ni), _ptr(M27), _ptr(E), _ptr(y))
    return y


def move(n, h, dt, x, v, qom, E_node, B_node):
    """Returns the moved (x, v); inputs are not modified."""
    ni, hh = _grid(n, h)
    x = _f64(x).copy()
    v = _f64(v).copy()
    lib().oracle_move(_ptr(ni), _ptr(hh), float(dt), x.shape[1], _ptr(x), _ptr(v), float(qom),
                      _ptr(_f64(E_node)), _ptr(_f64(B_node)))
    return x, v


def move_moments_threads(n, h, dt, x, v, q, qom, E_node, B_node, B_next, J=None, M27=None, threads=1):
    """The particle pass of one step on `threads` host threads: the mover (E_node, B_node), then the
    moments at the new positions with B_next accumulated into J and M27 (thread-private grids added
    in thread order). Returns (x', v', J, M27, threads used); x and v are not modified."""
    ni, hh = _grid(n, h)
    nn = int(np.prod(n))
    J = np.zeros((3, nn)) if J is None else J
    M27 = np.zeros((27, 9, nn)) if M27 is None else M27
    x = _f64(x).copy()
    v = _f64(v).copy()
    qa, qc = _q(q)
    used = lib().oracle_move_moments_threads(_ptr(ni), _ptr(hh), float(dt), x.shape[1], _ptr(x), _ptr(v),
                                             _ptr(qa), qc, float(qom), _ptr(_f64(E_node)), _ptr(_f64(B_node)),
                                             _ptr(_f64(B_next)), _ptr(J), _ptr(M27), int(threads))
    return x, v, J, M27, int(used)


def curl_C(n, h, E):
    ni, hh = _grid(n, h)
    E = _f64(E)
    out = np.zeros_like(E)
    lib().oracle_curl_C(_ptr(ni), _ptr(hh), _ptr(E), _ptr(out))
    return out


def curl_N(n, h, B):
    ni, hh = _grid(n, h)
    B = _f64(B)
    out = np.zeros_like(B)
    lib().oracle_curl_N(_ptr(ni), _ptr(hh), _ptr(B), _ptr(out))
    return out


def centres_to_nodes(n, BC):
    ni = np.asarray(n, dtype=np.int32)
    BC = _f64(BC)
    out = np.zeros_like(BC)
    lib().oracle_centres_to_nodes(_ptr(ni), _ptr(BC), _ptr(out))
    return out


def field_operator(n, h, dt, M27, E):
    ni, hh = _grid(n, h)
    E = _f64(E)
    out = np.zeros_like(E)
    lib().oracle_field_operator(_ptr(ni), _ptr(hh), float(dt), _ptr(_f64(M27)), _ptr(E), _ptr(out))
    return out


def field_rhs(n, h, dt, J, E_n, BC_n):
    ni, hh = _grid(n, h)
    b = np.zeros_like(_f64(E_n))
    lib().oracle_field_rhs(_ptr(ni), _ptr(hh), float(dt), _ptr(_f64(J)), _ptr(_f64(E_n)),
                           _ptr(_f64(BC_n)), _ptr(b))
    return b


def field_solve(n, h, dt, M27, J, E_n, BC_n, tol=1e-10, restart=30, maxit=1000):
    """GMRES for E^{n+theta}, then the field advance. Returns a dict."""
    ni, hh = _grid(n, h)
    E_n = _f64(E_n)
    BC_n = _f64(BC_n)
    Et = np.zeros_like(E_n)
    En1 = np.zeros_like(E_n)
    Bn1 = np.zeros_like(BC_n)
    rel = np.zeros(1)
    it = lib().oracle_field_solve(_ptr(ni), _ptr(hh), float(dt), _ptr(_f64(M27)), _ptr(_f64(J)),
                                  _ptr(E_n), _ptr(BC_n), float(tol), int(restart), int(maxit),
                                  _ptr(Et), _ptr(En1), _ptr(Bn1), _ptr(rel))
    return dict(E_theta=Et, E_next=En1, BC_next=Bn1, iters=it, rel_resid=float(rel[0]))


def kinetic(v, q, qom):
    v = _f64(v)
    qa, qc = _q(q)
    return lib().oracle_kinetic(v.shape[1], _ptr(v), _ptr(qa), qc, float(qom))


def field_energy(n, h, F):
    ni, hh = _grid(n, h)
    return lib().oracle_field_energy(_ptr(ni), _ptr(hh), _ptr(_f64(F)))


def grad(n, h, dt, x, v, q, qom, E_node, B_node, gJ, gM, gE=None, gB=None):
    """Reference gradient (dual numbers) of <gJ,J> + <gM,M14> through mover -> moments."""
    ni, hh = _grid(n, h)
    nn = int(np.prod(n))
    x = _f64(x)
    v = _f64(v)
    qa, qc = _q(q)
    gx = np.zeros_like(x)
    gv = np.zeros_like(v)
    if gE is None:
        gE = np.zeros((3, nn))
    if gB is None:
        gB = np.zeros((3, nn))
    lib().oracle_grad(_ptr(ni), _ptr(hh), float(dt), x.shape[1], _ptr(x), _ptr(v), _ptr(qa), qc,
                      float(qom), _ptr(_f64(E_node)), _ptr(_f64(B_node)), _ptr(_f64(gJ)),
                      _ptr(_f64(gM)), _ptr(gx), _ptr(gv), _ptr(gE), _ptr(gB))
    return gx, gv, gE, gB


def particle_loss(n, h, dt, x, v, q, qom, E_node, B_node, gJ, gM):
    ni, hh = _grid(n, h)
    x = _f64(x)
    v = _f64(v)
    qa, qc = _q(q)
    lp = np.zeros(x.shape[1])
    lib().oracle_particle_loss(_ptr(ni), _ptr(hh), float(dt), x.shape[1], _ptr(x), _ptr(v), _ptr(qa),
                               qc, float(qom), _ptr(_f64(E_node)), _ptr(_f64(B_node)),
                               _ptr(_f64(gJ)), _ptr(_f64(gM)), _ptr(lp))
    return lp


# ----------------------------------------------------------------------------
# composite drivers
# ----------------------------------------------------------------------------

def species_moments(plasma, x_list, v_list, B_node):
    """Sum of the moments of every species at the given states."""
    nn = plasma.nn
    J = np.zeros((3, nn))
    M27 = np.zeros((27, 9, nn))
    for s, x, v in zip(plasma.species, x_list, v_list):
        moments(plasma.n, plasma.h, plasma.dt, x, v, s.q, s.qom, B_node, J, M27)
    return J, M27


def total_energy(plasma, v_list, E, BC):
    K = sum(kinetic(v, s.q, s.qom) for s, v in zip(plasma.species, v_list))
    WE = field_energy(plasma.n, plasma.h, E)
    WB = field_energy(plasma.n, plasma.h, BC)
    return K, WE, WB


def run_steps(plasma, nsteps, tol=1e-10, restart=30, maxit=1000, record=None):
    """The scheme's step loop (Sec. II): moments -> field solve -> mover.

    Returns the final state and a per-step list of diagnostics.
    """
    x = [s.x.copy() for s in plasma.species]
    v = [s.v.copy() for s in plasma.species]
    E = plasma.E.copy()
    BC = plasma.B_C.copy()
    hist = []
    K, WE, WB = total_energy(plasma, v, E, BC)
    hist.append(dict(step=0, K=K, WE=WE, WB=WB, total=K + WE + WB, iters=0, rel_resid=0.0))
    for step in range(1, nsteps + 1):
        BN = centres_to_nodes(plasma.n, BC)
        J, M27 = species_moments(plasma, x, v, BN)
        sol = field_solve(plasma.n, plasma.h, plasma.dt, M27, J, E, BC, tol, restart, maxit)
        if record is not None:
            record.append(dict(step=step, x=[a.copy() for a in x], v=[a.copy() for a in v], E=E.copy(),
                               BC=BC.copy(), BN=BN, J=J, M27=M27, E_theta=sol["E_theta"]))
        for i, s in enumerate(plasma.species):
            x[i], v[i] = move(plasma.n, plasma.h, plasma.dt, x[i], v[i], s.qom, sol["E_theta"], BN)
        E, BC = sol["E_next"], sol["BC_next"]
        K, WE, WB = total_energy(plasma, v, E, BC)
        hist.append(dict(step=step, K=K, WE=WE, WB=WB, total=K + WE + WB, iters=sol["iters"],
                         rel_resid=sol["rel_resid"]))
    return dict(x=x, v=v, E=E, BC=BC), hist


def run_steps_threads(plasma, nsteps, threads=1, tol=1e-10, restart=30, maxit=1000):
    """The scheme's step loop with the particle pass on host threads: the moments of the initial
    state, then per step the field solve, and the mover followed by the next step's moments
    (move_moments_threads, with B^n for the mover and B^{n+1} for the moments). The same scheme as
    run_steps (Sec. II), with the mover and the next moments in one pass. Returns the final state,
    the per-step history and the threads used."""
    x = [s.x.copy() for s in plasma.species]
    v = [s.v.copy() for s in plasma.species]
    E = plasma.E.copy()
    BC = plasma.B_C.copy()
    BN = centres_to_nodes(plasma.n, BC)
    J, M27 = species_moments(plasma, x, v, BN)
    hist = []
    used = 1
    for step in range(1, nsteps + 1):
        sol = field_solve(plasma.n, plasma.h, plasma.dt, M27, J, E, BC, tol, restart, maxit)
        BN_next = centres_to_nodes(plasma.n, sol["BC_next"])
        Jn = np.zeros_like(J)
        Mn = np.zeros_like(M27)
        for i, s in enumerate(plasma.species):
            x[i], v[i], Jn, Mn, used = move_moments_threads(plasma.n, plasma.h, plasma.dt, x[i], v[i], s.q, s.qom,
                                                            sol["E_theta"], BN, BN_next, Jn, Mn, threads)
        J, M27, BN = Jn, Mn, BN_next
        E, BC = sol["E_next"], sol["BC_next"]
        K, WE, WB = total_energy(plasma, v, E, BC)
        hist.append(dict(step=step, total=K + WE + WB, iters=sol["iters"], rel_resid=sol["rel_resid"]))
    return dict(x=x, v=v, E=E, BC=BC), hist, used

