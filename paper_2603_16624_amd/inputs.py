"""Seeded synthetic plasmas for the ECsim particle hot path.

This module only draws random numbers and converts between storage layouts.
It holds none of the scheme's arithmetic (no interpolation weights, no
rotation matrix, no deposit), so both the GPU path and the CPU oracle can
consume the same host arrays.

Units follow the normalisation of the paper's field equations (Sec. II,
Eqs. 6-7): Gaussian units with the 4*pi factor, c = 1 and omega_pe = 1.
With omega_ps^2 = 4*pi*rho_s*(q/m)_s, the electron charge density is
rho_e = -1/(4*pi) and the neutralising ion density is rho_i = +1/(4*pi).
A macro-particle carries q_p = rho_s * V_box / N_s and m_p = q_p / (q/m)_s.

Layouts
-------
* particles, FP64 form: absolute positions ``x`` of shape (3, Np) in [0, L),
  velocities ``v`` of shape (3, Np) (structure of arrays, component major);
* particles, FP32 form: ``cell`` int32 (Np,) with ``ix + nx*(iy + ny*iz)``,
  in-cell offsets ``off`` float32 (3, Np) in [0, 1), velocities float32 (3, Np);
* node fields: (3, Nn) with node index ``ix + nx*(iy + ny*iz)``;
* cell-centred fields (B_C): (3, Nc) with the same index for the cell whose
  lower corner is that node.

Seeds: ``numpy.random.default_rng(1000*k + 10*s + purpose)`` for workload k
and species s (electrons 0, ions 1), purpose 0 positions, 1 velocities,
2 rejection draws, 7 loss weights, 8 finite-difference samples,
9 field perturbations.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

FOURPI = 4.0 * math.pi


def rng(k: int, s: int, purpose: int) -> np.random.Generator:
    return np.random.default_rng(1000 * k + 10 * s + purpose)


@dataclasses.dataclass
class Species:
    name: str
    qom: float                 # (q/m)_s
    q: np.ndarray              # per-particle charge, float64 (Np,)
    x: np.ndarray              # float64 (3, Np), absolute position in [0, L)
    v: np.ndarray              # float64 (3, Np)

    @property
    def np(self) -> int:
        return int(self.x.shape[1])

    @property
    def q_uniform(self) -> Optional[float]:
        """The common charge if every particle carries the same one."""
        if self.q.size and np.all(self.q == self.q[0]):
            return float(self.q[0])
        return None


@dataclasses.dataclass
class Plasma:
    n: tuple                   # cells per dimension (nx, ny, nz)
    h: tuple                   # cell size per dimension
    dt: float
    species: List[Species]
    E: np.ndarray              # node field (3, Nn)
    B_C: np.ndarray            # cell-centred field (3, Nc)
    name: str = ""

    @property
    def L(self):
        return tuple(self.n[d] * self.h[d] for d in range(3))

    @property
    def nn(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])

    @property
    def n_particles(self) -> int:
        return sum(s.np for s in self.species)


# ----------------------------------------------------------------------------
# sampling helpers
# ----------------------------------------------------------------------------

def _uniform_per_cell(n, h, ppc, g: np.random.Generator) -> np.ndarray:
    """Exactly ``ppc`` particles per cell, uniform inside each cell, cell order."""
    nx, ny, nz = n
    nc = nx * ny * nz
    cells = np.repeat(np.arange(nc, dtype=np.int64), ppc)
    ix = cells % nx
    iy = (cells // nx) % ny
    iz = cells // (nx * ny)
    u = g.random((3, cells.size))
    x = np.empty((3, cells.size))
    x[0] = (ix + u[0]) * h[0]
    x[1] = (iy + u[1]) * h[1]
    x[2] = (iz + u[2]) * h[2]
    return _clip_box(x, n, h)


def _clip_box(x: np.ndarray, n, h) -> np.ndarray:
    """Keep positions inside [0, L) after float rounding of (i + u) * h."""
    for d in range(3):
        L = n[d] * h[d]
        x[d] = np.where(x[d] >= L, 0.0, x[d])
    return x


def _maxwellian(npart: int, vth: float, g: np.random.Generator) -> np.ndarray:
    return vth * g.standard_normal((3, npart))


def _make_species(name, qom, rho, box_volume, x, v) -> Species:
    npart = x.shape[1]
    q = np.full(npart, rho * box_volume / npart)
    return Species(name=name, qom=qom, q=q, x=x, v=v)


ELECTRON_QOM = -1.0
ION_QOM = 1.0 / 25.0
VTH_E = 0.05
VTH_I = 0.01
B0 = (0.0, 0.0, 0.2)


def uniform_plasma(k: int, n, ppc: int, h=(0.5, 0.5, 0.5), dt=0.1,
                   b0=B0, vth=(VTH_E, VTH_I)) -> Plasma:
    """Two-species Maxwellian plasma with ``ppc`` particles per cell per species."""
    n = tuple(int(a) for a in n)
    h = tuple(float(a) for a in h)
    box_volume = n[0] * h[0] * n[1] * h[1] * n[2] * h[2]
    sp = []
    for s, (name, qom, rho, vt) in enumerate(
            [("electrons", ELECTRON_QOM, -1.0 / FOURPI, vth[0]),
             ("ions", ION_QOM, 1.0 / FOURPI, vth[1])]):
        x = _uniform_per_cell(n, h, ppc, rng(k, s, 0))
        v = _maxwellian(x.shape[1], vt, rng(k, s, 1))
        sp.append(_make_species(name, qom, rho, box_volume, x, v))
    nn = n[0] * n[1] * n[2]
    E = np.zeros((3, nn))
    B_C = np.zeros((3, nn))
    for d in range(3):
        B_C[d] = b0[d]
    return Plasma(n=n, h=h, dt=dt, species=sp, E=E, B_C=B_C, name=f"uniform-{k}")


def config0() -> Plasma:
    """8^3 periodic cells, 27 particles per cell per species (27,648 particles)."""
    p = uniform_plasma(0, (8, 8, 8), 27)
    p.name = "8^3 cells x 27 ppc x 2 species, FP64"
    return p


def config1(ppc: int = 64, n=(64, 64, 64)) -> Plasma:
    """64^3 periodic cells, 64 particles per cell per species (33.5M particles).

    Ions sit uniformly in each cell; electrons are drawn over the whole box with
    density 1 + 0.01 cos(2 pi x / L_x) by rejection sampling.
    """
    k = 1
    n = tuple(int(a) for a in n)
    h = (0.5, 0.5, 0.5)
    L = tuple(n[d] * h[d] for d in range(3))
    box_volume = L[0] * L[1] * L[2]
    nc = n[0] * n[1] * n[2]
    ne = ppc * nc
    # electrons: rejection sampling of x, uniform y, z
    gpos = rng(k, 0, 0)
    grej = rng(k, 0, 2)
    xs = []
    got = 0
    while got < ne:
        m = int((ne - got) * 1.02) + 1024
        xc = gpos.random(m) * L[0]
        u = grej.random(m)
        acc = xc[u < (1.0 + 0.01 * np.cos(2.0 * math.pi * xc / L[0])) / 1.01]
        xs.append(acc[: ne - got])
        got += xs[-1].size
    xe = np.empty((3, ne))
    xe[0] = np.concatenate(xs)
    xe[1] = gpos.random(ne) * L[1]
    xe[2] = gpos.random(ne) * L[2]
    xe = _clip_box(xe, n, h)
    ve = _maxwellian(ne, VTH_E, rng(k, 0, 1))
    xi = _uniform_per_cell(n, h, ppc, rng(k, 1, 0))
    vi = _maxwellian(xi.shape[1], VTH_I, rng(k, 1, 1))
    sp = [_make_species("electrons", ELECTRON_QOM, -1.0 / FOURPI, box_volume, xe, ve),
          _make_species("ions", ION_QOM, 1.0 / FOURPI, box_volume, xi, vi)]
    E = np.zeros((3, nc))
    B_C = np.zeros((3, nc))
    for d in range(3):
        B_C[d] = B0[d]
    return Plasma(n=n, h=h, dt=0.1, species=sp, E=E, B_C=B_C,
                  name=f"{n[0]}x{n[1]}x{n[2]} cells x {ppc} ppc x 2 species, 1% cos electron perturbation")


def config3(n=(32, 32, 32), ppc: int = 27) -> Plasma:
    """Differentiation workload: 32^3 cells, 27 ppc per species, perturbed fields.

    E ~ N(0, 1e-3) and B_C = B0 + N(0, 1e-3) per component, seeded, so that the
    gradient with respect to E and B is not degenerate.
    """
    p = uniform_plasma(3, n, ppc)
    g = rng(3, 0, 9)
    p.E = 1e-3 * g.standard_normal(p.E.shape)
    p.B_C = p.B_C + 1e-3 * g.standard_normal(p.B_C.shape)
    p.name = f"{n[0]}^3 cells x {ppc} ppc x 2 species, perturbed fields"
    return p


def harris(n=(256, 128, 8), ppc: int = 128, k: int = 4) -> Plasma:
    """Double Harris current sheet, periodic, mass ratio 25.

    B_x = B0 [tanh((y - Ly/4)/delta) - tanh((y - 3Ly/4)/delta) - 1] with B0 = 0.1
    and delta = 0.5 d_i = 2.5. Exactly ``ppc`` particles per cell per species,
    uniform inside the cell; each particle belongs to sheet 1, sheet 2 or the
    uniform background (0.1 n0) with probability proportional to the local
    densities, and carries the charge of the total local density. Sheet
    particles drift along z with opposite signs in the two sheets; T_i/T_e = 5.
    """
    n = tuple(int(a) for a in n)
    h = (0.5, 0.5, 0.5)
    L = tuple(n[d] * h[d] for d in range(3))
    b0, delta = 0.1, 2.5
    y1, y2 = L[1] / 4, 3 * L[1] / 4
    # pressure balance n0 (Te + Ti) = B0^2 / (8 pi), Ti = 5 Te, n0 = 1/(4 pi)
    n0 = 1.0 / FOURPI
    te = b0 * b0 / (8 * math.pi) / (6.0 * n0)
    ti = 5.0 * te
    vth_e = math.sqrt(te / 1.0)          # m_e = 1 in units with q/m = -1, |q| = 1
    vth_i = math.sqrt(ti / 25.0)
    # Harris drifts: J_z = -(B0 / (4 pi delta)) sech^2 at sheet 1, split as V_s ~ T_s / q_s
    jz = b0 / (FOURPI * delta)
    # n0 * (-V_e + V_i) = -jz with V_e / V_i = -(Te / Ti)
    vi_drift = -jz / n0 / (1.0 + te / ti)
    ve_drift = -vi_drift * te / ti
    cell_volume = h[0] * h[1] * h[2]
    sp = []
    for s, (name, qom, vth, vdrift) in enumerate(
            [("electrons", ELECTRON_QOM, vth_e, ve_drift), ("ions", ION_QOM, vth_i, vi_drift)]):
        x = _uniform_per_cell(n, h, ppc, rng(k, s, 0))
        npart = x.shape[1]
        y = x[1]
        d1 = 1.0 / np.cosh((y - y1) / delta) ** 2
        d2 = 1.0 / np.cosh((y - y2) / delta) ** 2
        bg = 0.1 * np.ones_like(y)
        tot = d1 + d2 + bg
        u = rng(k, s, 3).random(npart)
        pop = np.where(u < d1 / tot, 1, np.where(u < (d1 + d2) / tot, 2, 0))
        v = _maxwellian(npart, vth, rng(k, s, 1))
        v[2] += np.where(pop == 1, vdrift, np.where(pop == 2, -vdrift, 0.0))
        sign = -1.0 if qom < 0 else 1.0
        q = sign * n0 * tot * cell_volume / ppc
        sp.append(Species(name=name, qom=qom, q=q, x=x, v=v))
    nc = n[0] * n[1] * n[2]
    ycent = (np.arange(nc) // n[0] % n[1] + 0.5) * h[1]
    B_C = np.zeros((3, nc))
    B_C[0] = b0 * (np.tanh((ycent - y1) / delta) - np.tanh((ycent - y2) / delta) - 1.0)
    E = np.zeros((3, nc))
    return Plasma(n=n, h=h, dt=0.1, species=sp, E=E, B_C=B_C,
                  name=f"double Harris {n[0]}x{n[1]}x{n[2]} x {ppc} ppc x 2 species")


def four_species_2d_f32(n=(256, 128, 1), ppc: int = 3600, k: int = 6, dt: float = 0.1):
    """The paper's four-species 2D shape (Sec. IV: 256 x 128 cells, 4 species x
    3600 particles per cell, 471,859,200 particles) as a synthetic stand-in,
    generated directly in the FP32 storage form and already grouped by cell
    (ppc particles of each species per cell, in cell order), one species at a
    time so that no FP64 copy of the state is held. Species: two counter-
    streaming electron beams (drift +-0.1 along x, v_th 0.05) and two ion
    species (q/m 1/25 and 1/50, v_th 0.01) of equal densities, neutral in
    total. Yields per species: name, qom, q (per-particle charge, constant),
    cell int32 (N,), off float32 (3, N), v float32 (3, N), cell_start int32
    (cells + 1,)."""
    n = tuple(int(a) for a in n)
    h = (0.5, 0.5, 0.5)
    nc = n[0] * n[1] * n[2]
    vcell = h[0] * h[1] * h[2]
    specs = [("electrons+x", ELECTRON_QOM, -0.5 / FOURPI, 0.05, 0.1),
             ("electrons-x", ELECTRON_QOM, -0.5 / FOURPI, 0.05, -0.1),
             ("ions", ION_QOM, 0.5 / FOURPI, 0.01, 0.0),
             ("heavy ions", ION_QOM / 2.0, 0.5 / FOURPI, 0.01, 0.0)]
    cell = np.repeat(np.arange(nc, dtype=np.int32), ppc)
    cell_start = (np.arange(nc + 1, dtype=np.int64) * ppc).astype(np.int32)
    for s, (name, qom, rho, vth, drift) in enumerate(specs):
        g = rng(k, s, 0)
        off = g.random((3, nc * ppc), dtype=np.float32)
        v = (vth * rng(k, s, 1).standard_normal((3, nc * ppc), dtype=np.float32)).astype(np.float32)
        v[0] += np.float32(drift)
        yield dict(name=name, qom=qom, q=rho * vcell / ppc, cell=cell, off=off, v=v, cell_start=cell_start,
                   n=n, h=h, dt=dt)


def single_particle(n=(4, 4, 4), h=(0.5, 0.5, 0.5), dt=0.1, x=(1.1, 0.7, 1.3),
                    v=(0.03, -0.02, 0.01), q=-1e-3, qom=-1.0, b=(0.0, 0.0, 0.2),
                    e=(0.0, 0.0, 0.0)) -> Plasma:
    """One particle in uniform node fields (gyration and drift pins)."""
    nn = n[0] * n[1] * n[2]
    sp = [Species(name="lone", qom=qom, q=np.array([q]),
                  x=np.array(x, dtype=np.float64).reshape(3, 1),
                  v=np.array(v, dtype=np.float64).reshape(3, 1))]
    E = np.zeros((3, nn))
    B_C = np.zeros((3, nn))
    for d in range(3):
        E[d] = e[d]
        B_C[d] = b[d]
    return Plasma(n=tuple(n), h=tuple(h), dt=dt, species=sp, E=E, B_C=B_C, name="lone particle")


def random_node_field(nn: int, seed: int, scale: float = 1.0, mean=(0.0, 0.0, 0.0)) -> np.ndarray:
    g = np.random.default_rng(seed)
    f = scale * g.standard_normal((3, nn))
    for d in range(3):
        f[d] += mean[d]
    return f


def loss_weights(nn: int, k: int = 3):
    """Seeded N(0,1) weights for a scalar loss on J-hat (3, Nn) and M (14, 9, Nn)."""
    g = rng(k, 0, 7)
    gJ = g.standard_normal((3, nn))
    gM = g.standard_normal((14, 9, nn))
    return gJ, gM


# ----------------------------------------------------------------------------
# FP32 storage form: int32 cell index + FP32 in-cell offset
# ----------------------------------------------------------------------------

ONE_MINUS_F32 = np.nextafter(np.float32(1.0), np.float32(0.0))


def encode_f32(x: np.ndarray, n, h):
    """Absolute FP64 positions -> (int32 cell, float32 offsets in [0, 1))."""
    u = np.empty_like(x)
    ijk = np.empty(x.shape, dtype=np.int64)
    for d in range(3):
        u[d] = x[d] / h[d]
        ijk[d] = np.floor(u[d]).astype(np.int64) % n[d]
        u[d] = u[d] - np.floor(u[d])
    off = np.minimum(u.astype(np.float32), ONE_MINUS_F32)
    cell = (ijk[0] + n[0] * (ijk[1] + n[1] * ijk[2])).astype(np.int32)
    return cell, np.ascontiguousarray(off)


def decode_f32(cell: np.ndarray, off: np.ndarray, n, h) -> np.ndarray:
    """(cell, float32 offset) -> FP64 absolute position; exact for h = 2^-k."""
    c = cell.astype(np.int64)
    ijk = (c % n[0], (c // n[0]) % n[1], c // (n[0] * n[1]))
    x = np.empty((3, cell.size))
    for d in range(3):
        x[d] = (ijk[d].astype(np.float64) + off[d].astype(np.float64)) * h[d]
    return x


def to_f32_state(p: Plasma):
    """The FP32 form of every species, plus its exact FP64 decoding."""
    out = []
    for s in p.species:
        cell, off = encode_f32(s.x, p.n, p.h)
        v32 = s.v.astype(np.float32)
        x64 = decode_f32(cell, off, p.n, p.h)
        out.append(dict(cell=cell, off=off, v=v32, q=s.q.astype(np.float32),
                        x64=x64, v64=v32.astype(np.float64), q64=s.q.astype(np.float32).astype(np.float64)))
    return out
