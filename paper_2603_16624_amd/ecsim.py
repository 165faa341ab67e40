"""Python binding of libecsim.so (the C ABI in include/ecsim.h).

Argument marshalling only: every step of the hot path runs in the library's
HIP kernels. PyTorch provides device memory and the current HIP stream.
The binding refuses to run without the compiled library: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import List, Optional, Sequence

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libecsim.so")

OK, EINVAL, EHIP, EWORKSPACE, ENONFINITE, ENOCONV = 0, -1, -2, -3, -4, -5
F64, F32 = 0, 1
NOALLOC_SCRATCH_BYTES = 64 << 20   # ECSIM_NOALLOC_SCRATCH_BYTES of include/ecsim.h
ACCUMULATE, SORTED, BWD_THROUGH_MOVER, BWD_OFFSET_GRAD = 1, 2, 8, 16
ENERGY_WS_BYTES = 2048


class EcsimError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"ecsim status {status}: {msg}")
        self.status = status


class _Grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("h", ctypes.c_double * 3), ("dt", ctypes.c_double)]


class _Particles(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_int32), ("np", ctypes.c_int64), ("qom", ctypes.c_double),
                ("pos", ctypes.c_void_p * 3), ("cell", ctypes.c_void_p), ("vel", ctypes.c_void_p * 3),
                ("q", ctypes.c_void_p), ("q_const", ctypes.c_double), ("cell_start", ctypes.c_void_p)]


_lib = None


def lib():
    """Load libecsim.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2603_16624_amd/build.py "
                               "(or __graft_entry__.build()); there is no fallback path")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        st = ctypes.c_int32
        L.ecsim_last_error.restype = ctypes.c_char_p
        L.ecsim_version.restype = ctypes.c_char_p
        sig = {
            "ecsim_workspace_size": [P, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32, P],
            "ecsim_species_qom": [ctypes.c_int32, ctypes.c_double, ctypes.c_double, P],
            "ecsim_move": [P, P, P, P, P, P],
            "ecsim_moments": [P, P, ctypes.c_int32, P, P, P, P, ctypes.c_size_t, ctypes.c_uint32, P],
            "ecsim_move_moments": [P, P, ctypes.c_int32, P, P, P, P, P, P, P, ctypes.c_size_t, ctypes.c_uint32,
                                   P],
            "ecsim_move_moments_noalloc": [P, P, ctypes.c_int32, P, P, P, P, P, P, ctypes.c_uint32, P],
            "ecsim_move_moments_regroup": [P, P, P, ctypes.c_int32, P, P, P, P, P, P, P, ctypes.c_size_t,
                                           ctypes.c_uint32, P],
            "ecsim_diagnostics": [P, P, ctypes.c_int32, P, P, P, P, ctypes.c_size_t, ctypes.c_uint32, P],
            "ecsim_diagnostics_workspace_size": [P, ctypes.c_int32, ctypes.c_uint32, P],
            "ecsim_mass_apply": [P, ctypes.c_int32, P, P, ctypes.c_double, ctypes.c_double, P, P],
            "ecsim_moments_backward": [P, P, P, P, P, P, P, P, P, P, P, ctypes.c_size_t, ctypes.c_uint32, P],
            "ecsim_backward_workspace_size": [P, ctypes.c_int64, ctypes.c_int32, P],
            "ecsim_sort": [P, P, P, P, P, P, ctypes.c_size_t, P],
            "ecsim_centres_to_nodes": [P, P, P, P, P],
            "ecsim_to_f32": [ctypes.c_int64, P, P, P],
            "ecsim_solve_workspace_size": [P, ctypes.c_int32, P],
            "ecsim_field_solve": [P, ctypes.c_int32, P, P, P, P, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                  P, P, P, P, ctypes.c_size_t, P, P, P],
            "ecsim_field_energy": [P, P, P, P, ctypes.c_size_t, P],
            "ecsim_check_finite": [P],
            "ecsim_nonfinite_read": [P, P],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = st
        _lib = L
    return _lib


EXPORTED = ["ecsim_last_error", "ecsim_version", "ecsim_workspace_size", "ecsim_species_qom", "ecsim_move", "ecsim_moments",
            "ecsim_move_moments", "ecsim_move_moments_noalloc", "ecsim_move_moments_regroup", "ecsim_diagnostics",
            "ecsim_diagnostics_workspace_size",
            "ecsim_mass_apply", "ecsim_moments_backward", "ecsim_backward_workspace_size", "ecsim_sort", "ecsim_centres_to_nodes", "ecsim_to_f32",
            "ecsim_solve_workspace_size", "ecsim_field_solve", "ecsim_field_energy", "ecsim_check_finite",
            "ecsim_nonfinite_read"]


def _check(status: int):
    if status != OK:
        raise EcsimError(status, lib().ecsim_last_error().decode())


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


# ----------------------------------------------------------------------------
# data holders
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Grid:
    n: tuple
    h: tuple
    dt: float

    def c(self) -> _Grid:
        g = _Grid()
        for d in range(3):
            g.n[d] = int(self.n[d])
            g.h[d] = float(self.h[d])
        g.dt = float(self.dt)
        return g

    @property
    def nn(self) -> int:
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])


@dataclasses.dataclass
class Species:
    """Device arrays of one species. pos/vel are (3, np) contiguous tensors."""
    prec: int
    qom: float
    pos: torch.Tensor
    vel: torch.Tensor
    cell: Optional[torch.Tensor] = None     # int32 (np,), FP32 form only
    q: Optional[torch.Tensor] = None        # per-particle charge, or None
    q_const: float = 0.0
    cell_start: Optional[torch.Tensor] = None

    @property
    def np(self) -> int:
        return int(self.pos.shape[1])

    @property
    def dtype(self):
        return torch.float64 if self.prec == F64 else torch.float32

    def c(self) -> _Particles:
        p = _Particles()
        p.prec = self.prec
        p.np = self.np
        p.qom = float(self.qom)
        esz = 8 if self.prec == F64 else 4
        n = self.np
        for d in range(3):
            p.pos[d] = self.pos.data_ptr() + d * n * esz if n else None
            p.vel[d] = self.vel.data_ptr() + d * n * esz if n else None
        p.cell = self.cell.data_ptr() if self.cell is not None else None
        p.q = self.q.data_ptr() if self.q is not None else None
        p.q_const = float(self.q_const)
        p.cell_start = self.cell_start.data_ptr() if self.cell_start is not None else None
        return p

    def empty_like(self) -> "Species":
        return Species(self.prec, self.qom, torch.empty_like(self.pos), torch.empty_like(self.vel),
                       None if self.cell is None else torch.empty_like(self.cell),
                       None if self.q is None else torch.empty_like(self.q), self.q_const, None)

    def clone(self) -> "Species":
        return Species(self.prec, self.qom, self.pos.clone(), self.vel.clone(),
                       None if self.cell is None else self.cell.clone(),
                       None if self.q is None else self.q.clone(), self.q_const,
                       None if self.cell_start is None else self.cell_start.clone())

    @staticmethod
    def from_f64(qom, x, v, q, device="cuda") -> "Species":
        """FP64 form from host arrays x, v (3, np) and charges q (np,) or scalar."""
        pos = torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64).to(device)
        vel = torch.as_tensor(np.ascontiguousarray(v), dtype=torch.float64).to(device)
        qa, qc = _charges(q, torch.float64, device)
        return Species(F64, float(qom), pos, vel, None, qa, qc)

    @staticmethod
    def from_f32(qom, cell, off, v, q, device="cuda") -> "Species":
        """FP32 form from host arrays: cell int32 (np,), offsets float32 (3, np), v float32 (3, np)."""
        pos = torch.as_tensor(np.ascontiguousarray(off, dtype=np.float32)).to(device)
        vel = torch.as_tensor(np.ascontiguousarray(v, dtype=np.float32)).to(device)
        cl = torch.as_tensor(np.ascontiguousarray(cell, dtype=np.int32)).to(device)
        qa, qc = _charges(q, torch.float32, device)
        return Species(F32, float(qom), pos, vel, cl, qa, qc)


def _charges(q, dtype, device):
    q = np.asarray(q, dtype=np.float64)
    if q.ndim == 0:
        return None, float(q)
    if q.size and np.all(q == q[0]):
        return None, float(q[0])
    return torch.as_tensor(q).to(dtype=dtype, device=device), 0.0


# ----------------------------------------------------------------------------
# entry points
# ----------------------------------------------------------------------------

def version() -> str:
    return lib().ecsim_version().decode()


def workspace_size(grid: Grid, np_: int, prec: int, flags: int = 0) -> int:
    out = ctypes.c_size_t(0)
    _check(lib().ecsim_workspace_size(ctypes.byref(grid.c()), int(np_), int(prec), int(flags), ctypes.byref(out)))
    return int(out.value)


def species_qom(prec: int, qom: float, dt: float) -> float:
    """The charge-to-mass ratio the kernels of precision prec move a species of ratio qom with
    (the masses of every kinetic energy the library returns are q_p / this)."""
    out = ctypes.c_double(0.0)
    _check(lib().ecsim_species_qom(int(prec), float(qom), float(dt), ctypes.byref(out)))
    return out.value


def move(grid: Grid, sp: Species, E: torch.Tensor, B: torch.Tensor, ke: Optional[torch.Tensor] = None,
         stream=None):
    """Mover (Eqs. 4, 5, 8) in place on sp; ke (device float64 scalar) += kinetic energy."""
    c = sp.c()
    _check(lib().ecsim_move(ctypes.byref(grid.c()), ctypes.byref(c), _ptr(E), _ptr(B), _ptr(ke), _stream(stream)))


def _total(species):
    return sum(s.np for s in species)


def moments(grid: Grid, species: Sequence[Species], B: torch.Tensor, J: torch.Tensor, M: torch.Tensor,
            flags: int = 0, ws: Optional[torch.Tensor] = None, stream=None):
    """Moment gather (Eqs. 1, 3) summed over species into J (3, Nn) and M (14, 9, Nn)."""
    arr = (_Particles * len(species))(*[s.c() for s in species])
    if ws is None and (flags & SORTED):
        ws = torch.empty(workspace_size(grid, _total(species), species[0].prec), dtype=torch.uint8,
                         device=J.device)
    nbytes = 0 if ws is None else ws.numel() * ws.element_size()
    _check(lib().ecsim_moments(ctypes.byref(grid.c()), arr, len(species), _ptr(B), _ptr(J), _ptr(M), _ptr(ws),
                               nbytes, int(flags), _stream(stream)))


def diagnostics_workspace_size(grid: Grid, prec: int, flags: int = 0) -> int:
    out = ctypes.c_size_t(0)
    _check(lib().ecsim_diagnostics_workspace_size(ctypes.byref(grid.c()), int(prec), int(flags), ctypes.byref(out)))
    return int(out.value)


def diagnostics(grid: Grid, species: Sequence[Species], rho: torch.Tensor, J: torch.Tensor, P: torch.Tensor,
                flags: int = 0, ws: Optional[torch.Tensor] = None, stream=None):
    """Diagnostic moments summed over species: rho (Nn,), the current without
    rotation J (3, Nn) and the charge-weighted second velocity moment P (6, Nn)."""
    arr = (_Particles * len(species))(*[s.c() for s in species])
    if ws is None:
        need = diagnostics_workspace_size(grid, species[0].prec if species else F64, flags)
        ws = torch.empty(need, dtype=torch.uint8, device=rho.device) if need else None
    nbytes = 0 if ws is None else ws.numel() * ws.element_size()
    _check(lib().ecsim_diagnostics(ctypes.byref(grid.c()), arr, len(species), _ptr(rho), _ptr(J), _ptr(P), _ptr(ws),
                                   nbytes, int(flags), _stream(stream)))


def move_moments(grid: Grid, species: Sequence[Species], E: torch.Tensor, B: torch.Tensor, B_next: torch.Tensor,
                 J: torch.Tensor, M: torch.Tensor, ke: Optional[torch.Tensor] = None, flags: int = 0,
                 ws: Optional[torch.Tensor] = None, stream=None):
    """Fused mover (E, B) then moment gather at the new positions with B_next; species need cell_start."""
    arr = (_Particles * len(species))(*[s.c() for s in species])
    if ws is None:
        ws = torch.empty(workspace_size(grid, _total(species), species[0].prec), dtype=torch.uint8,
                         device=J.device)
    _check(lib().ecsim_move_moments(ctypes.byref(grid.c()), arr, len(species), _ptr(E), _ptr(B), _ptr(B_next),
                                    _ptr(J), _ptr(M), _ptr(ke), _ptr(ws), ws.numel(), int(flags), _stream(stream)))


def move_moments_noalloc(grid: Grid, species: Sequence[Species], E: torch.Tensor, B: torch.Tensor,
                         B_next: torch.Tensor, J: torch.Tensor, M: torch.Tensor, ke: Optional[torch.Tensor] = None,
                         flags: int = 0, stream=None):
    """move_moments on the library's static device scratch: no workspace, no allocation."""
    arr = (_Particles * len(species))(*[s.c() for s in species])
    _check(lib().ecsim_move_moments_noalloc(ctypes.byref(grid.c()), arr, len(species), _ptr(E), _ptr(B),
                                            _ptr(B_next), _ptr(J), _ptr(M), _ptr(ke), int(flags), _stream(stream)))


def move_moments_regroup(grid: Grid, species: Sequence[Species], dst: Sequence[Species], E: torch.Tensor,
                         B: torch.Tensor, B_next: torch.Tensor, J: torch.Tensor, M: torch.Tensor,
                         ke: Optional[torch.Tensor] = None, flags: int = 0, ws: Optional[torch.Tensor] = None,
                         stream=None):
    """The fused pass of move_moments that also writes each species' moved particles, grouped by cell,
    into dst (same sizes; a cell_start is allocated where dst has none) for the next pass."""
    for d in dst:
        if d.cell_start is None:
            d.cell_start = torch.empty(grid.nn + 1, dtype=torch.int32, device=J.device)
    arr = (_Particles * len(species))(*[s.c() for s in species])
    darr = (_Particles * len(dst))(*[d.c() for d in dst])
    if ws is None:
        ws = torch.empty(workspace_size(grid, _total(species), species[0].prec), dtype=torch.uint8,
                         device=J.device)
    _check(lib().ecsim_move_moments_regroup(ctypes.byref(grid.c()), arr, darr, len(species), _ptr(E), _ptr(B),
                                            _ptr(B_next), _ptr(J), _ptr(M), _ptr(ke), _ptr(ws), ws.numel(),
                                            int(flags), _stream(stream)))


def mass_apply(grid: Grid, M: torch.Tensor, x: torch.Tensor, y: torch.Tensor, a: float = 1.0, b: float = 0.0,
               stream=None):
    """y = a (M x) + b y with M in FP32 or FP64 and x, y FP64 (3, Nn)."""
    prec = F32 if M.dtype == torch.float32 else F64
    _check(lib().ecsim_mass_apply(ctypes.byref(grid.c()), prec, _ptr(M), _ptr(x), float(a), float(b), _ptr(y),
                                  _stream(stream)))


def backward_workspace_size(grid: Grid, np_: int, prec: int) -> int:
    """Workspace bytes of moments_backward for np_ grouped particles (ecsim_backward_workspace_size)."""
    out = ctypes.c_size_t()
    _check(lib().ecsim_backward_workspace_size(ctypes.byref(grid.c()), int(np_), int(prec), ctypes.byref(out)))
    return out.value


def moments_backward(grid: Grid, sp: Species, E: Optional[torch.Tensor], B: torch.Tensor, gJ: torch.Tensor,
                     gM: torch.Tensor, gpos: torch.Tensor, gvel: torch.Tensor, gE: Optional[torch.Tensor],
                     gB: torch.Tensor, through_mover: bool = True, offset_grad: bool = False,
                     ws: Optional[torch.Tensor] = None, stream=None):
    """Adjoint of (mover ->) moments; gpos, gvel (3, np) overwritten, gE, gB (3, Nn) accumulated.
    offset_grad (FP32 particles): gpos with respect to the in-cell offsets instead of the positions.
    A species with cell_start takes the brick-tiled kernel (its workspace is allocated if not given)."""
    esz = gpos.element_size()
    n = sp.np
    gp = (ctypes.c_void_p * 3)(*[gpos.data_ptr() + d * n * esz if n else None for d in range(3)])
    gv = (ctypes.c_void_p * 3)(*[gvel.data_ptr() + d * n * esz if n else None for d in range(3)])
    flags = (BWD_THROUGH_MOVER if through_mover else 0) | (BWD_OFFSET_GRAD if offset_grad else 0)
    if ws is None and sp.cell_start is not None:
        ws = torch.empty(backward_workspace_size(grid, n, sp.prec), dtype=torch.uint8, device=gpos.device)
    nbytes = 0 if ws is None else ws.numel() * ws.element_size()
    c = sp.c()
    _check(lib().ecsim_moments_backward(ctypes.byref(grid.c()), ctypes.byref(c), _ptr(E), _ptr(B), _ptr(gJ),
                                        _ptr(gM), gp, gv, _ptr(gE), _ptr(gB), _ptr(ws), nbytes, flags,
                                        _stream(stream)))


def sort(grid: Grid, src: Species, dst: Species, cell_start: torch.Tensor, perm: Optional[torch.Tensor] = None,
         ws: Optional[torch.Tensor] = None, stream=None):
    """Counting sort by cell from src into dst; cell_start int32 (Nc + 1,)."""
    if ws is None:
        ws = torch.empty(max(workspace_size(grid, src.np, src.prec), 1), dtype=torch.uint8, device=src.pos.device)
    cs, cd = src.c(), dst.c()
    _check(lib().ecsim_sort(ctypes.byref(grid.c()), ctypes.byref(cs), ctypes.byref(cd), _ptr(cell_start), _ptr(perm),
                            _ptr(ws), ws.numel(), _stream(stream)))
    dst.cell_start = cell_start


def centres_to_nodes(grid: Grid, BC: torch.Tensor, BN: Optional[torch.Tensor] = None,
                     BN32: Optional[torch.Tensor] = None, stream=None):
    _check(lib().ecsim_centres_to_nodes(ctypes.byref(grid.c()), _ptr(BC), _ptr(BN), _ptr(BN32), _stream(stream)))


def to_f32(src: torch.Tensor, dst: torch.Tensor, stream=None):
    _check(lib().ecsim_to_f32(src.numel(), _ptr(src), _ptr(dst), _stream(stream)))


def solve_workspace_size(grid: Grid, restart: int = 30) -> int:
    out = ctypes.c_size_t(0)
    _check(lib().ecsim_solve_workspace_size(ctypes.byref(grid.c()), int(restart), ctypes.byref(out)))
    return int(out.value)


def field_solve(grid: Grid, M: torch.Tensor, J: torch.Tensor, E_n: torch.Tensor, BC_n: torch.Tensor,
                E_theta: torch.Tensor, E_next: torch.Tensor, BC_next: torch.Tensor, tol: float = 1e-10,
                restart: int = 30, maxit: int = 1000, ws: Optional[torch.Tensor] = None, stream=None):
    """FP64 GMRES solve of Eqs. 6-7 and the field advance; returns (iterations, relative residual)."""
    if ws is None:
        ws = torch.empty(solve_workspace_size(grid, restart), dtype=torch.uint8, device=J.device)
    prec = F32 if M.dtype == torch.float32 else F64
    it = ctypes.c_int32(0)
    res = ctypes.c_double(0.0)
    _check(lib().ecsim_field_solve(ctypes.byref(grid.c()), prec, _ptr(M), _ptr(J), _ptr(E_n), _ptr(BC_n),
                                   float(tol), int(restart), int(maxit), _ptr(E_theta), _ptr(E_next), _ptr(BC_next),
                                   _ptr(ws), ws.numel(), ctypes.byref(it), ctypes.byref(res), _stream(stream)))
    return int(it.value), float(res.value)


def field_energy(grid: Grid, F: torch.Tensor, out: torch.Tensor, ws: Optional[torch.Tensor] = None, stream=None):
    if ws is None:
        ws = torch.empty(ENERGY_WS_BYTES, dtype=torch.uint8, device=F.device)
    _check(lib().ecsim_field_energy(ctypes.byref(grid.c()), _ptr(F), _ptr(out), _ptr(ws), ws.numel(),
                                    _stream(stream)))


def check_finite(stream=None):
    """Synchronous: raises EcsimError (status ENONFINITE) if a kernel produced a NaN or an
    infinity on this device since the last check; clears the flag."""
    _check(lib().ecsim_check_finite(_stream(stream)))


def nonfinite_read(flag_out: torch.Tensor, stream=None):
    """Asynchronous: the device flag (0 or 1) into the int32 device tensor flag_out, then cleared."""
    _check(lib().ecsim_nonfinite_read(_ptr(flag_out), _stream(stream)))


# ----------------------------------------------------------------------------
# the scheme's step loop on the device
# ----------------------------------------------------------------------------

class Simulation:
    """Per-step loop of the scheme (Sec. II): moments -> field solve -> mover.

    Particles stay on the device in the requested precision; the fields E, B_C,
    the GMRES solve and the energy diagnostic are FP64. With ``sort=True`` the
    particles are re-sorted by cell before each deposit and the tiled deposit
    is used; between re-sorts (every ``sort_every`` steps) the cell ranges
    are a stale grouping that the deposit corrects for. With ``fused=True``
    the mover and the next step's moments run as one pass; with
    ``regroup=True`` as well, every ``sort_every``-th pass also writes the
    particles grouped by cell into a second set of arrays
    (ecsim_move_moments_regroup) in place of a separate re-sort, and the
    passes in between run on that grouping as it goes stale.
    """

    def __init__(self, plasma, prec: int = F64, device="cuda", tol: float = 1e-10, restart: int = 30,
                 sort: bool = True, fused: bool = False, sort_every: int = 4, regroup: bool = False):
        from . import inputs as I
        self.grid = Grid(plasma.n, plasma.h, plasma.dt)
        self.prec = prec
        self.tol = tol
        self.restart = restart
        self.do_sort = sort or fused
        self.fused = fused
        self.regroup = bool(regroup and fused)
        self.sort_every = max(1, int(sort_every))
        self.nstep = 0
        self.primed = False
        self.device = device
        nn = self.grid.nn
        self.species: List[Species] = []
        if prec == F64:
            for s in plasma.species:
                self.species.append(Species.from_f64(s.qom, s.x, s.v, s.q, device))
        else:
            for s, f in zip(plasma.species, I.to_f32_state(plasma)):
                self.species.append(Species.from_f32(s.qom, f["cell"], f["off"], f["v"], f["q"], device))
        dt = torch.float64 if prec == F64 else torch.float32
        self.E = torch.as_tensor(plasma.E, dtype=torch.float64).to(device).contiguous()
        self.BC = torch.as_tensor(plasma.B_C, dtype=torch.float64).to(device).contiguous()
        self.BN = torch.empty((3, nn), dtype=torch.float64, device=device)
        self.BN_p = torch.empty((3, nn), dtype=dt, device=device) if prec == F32 else self.BN
        self.Et_p = torch.empty((3, nn), dtype=dt, device=device) if prec == F32 else None
        self.J = torch.zeros((3, nn), dtype=dt, device=device)
        self.M = torch.zeros((14, 9, nn), dtype=dt, device=device)
        self.E_theta = torch.empty_like(self.E)
        self.E_next = torch.empty_like(self.E)
        self.BC_next = torch.empty_like(self.BC)
        self.solve_ws = torch.empty(solve_workspace_size(self.grid, restart), dtype=torch.uint8, device=device)
        self.scal = torch.zeros(4, dtype=torch.float64, device=device)
        self.energy_ws = torch.empty(ENERGY_WS_BYTES, dtype=torch.uint8, device=device)
        self._spare = [s.empty_like() for s in self.species]
        self._cell_start = [torch.empty(nn + 1, dtype=torch.int32, device=device) for _ in self.species]
        np_max = max(s.np for s in self.species)
        np_tot = sum(s.np for s in self.species)
        self.ws = torch.empty(max(workspace_size(self.grid, max(np_tot, np_max), prec), 1), dtype=torch.uint8,
                              device=device)
        self.sort_ws = self.ws
        self.BN_next = torch.empty((3, nn), dtype=torch.float64, device=device)
        self.BN_next_p = torch.empty((3, nn), dtype=dt, device=device) if prec == F32 else self.BN_next
        self.last_iters = 0
        self.last_resid = 0.0

    def sort_particles(self):
        for i, s in enumerate(self.species):
            dst = self._spare[i]
            sort(self.grid, s, dst, self._cell_start[i], None, self.sort_ws)
            self._spare[i] = s
            s.cell_start = None
            self.species[i] = dst

    def node_B(self):
        centres_to_nodes(self.grid, self.BC, self.BN, self.BN_p if self.prec == F32 else None)

    def deposit(self):
        flags = SORTED if (self.do_sort and all(s.cell_start is not None for s in self.species)) else 0
        moments(self.grid, self.species, self.BN_p, self.J, self.M, flags, ws=self.ws)

    def solve(self):
        it, res = field_solve(self.grid, self.M, self.J, self.E, self.BC, self.E_theta, self.E_next, self.BC_next,
                              self.tol, self.restart, ws=self.solve_ws)
        self.last_iters, self.last_resid = it, res

    def push(self, ke: Optional[torch.Tensor] = None):
        if self.prec == F32:
            to_f32(self.E_theta, self.Et_p)
            Et = self.Et_p
        else:
            Et = self.E_theta
        for s in self.species:
            # the cell ranges stay a valid (stale) grouping: the tiled deposit
            # takes particles that left their range through its stray list
            move(self.grid, s, Et, self.BN_p, ke)

    def advance_fields(self):
        self.E, self.E_next = self.E_next, self.E
        self.BC, self.BC_next = self.BC_next, self.BC

    def prime(self):
        """Fused loop: sort, then the moments of the initial state."""
        self.sort_particles()
        self.node_B()
        self.deposit()
        self.primed = True

    def fused_fields(self):
        """Node fields of the fused pass: B^{n+1} at the nodes, E^{n+theta} in particle precision."""
        centres_to_nodes(self.grid, self.BC_next, self.BN_next, self.BN_next_p if self.prec == F32 else None)
        if self.prec == F32:
            to_f32(self.E_theta, self.Et_p)

    def fused_particles(self, ke: Optional[torch.Tensor] = None):
        """The fused particle pass proper (fused_fields() first)."""
        Et = self.Et_p if self.prec == F32 else self.E_theta
        if self.regroup_now():
            move_moments_regroup(self.grid, self.species, self._spare, Et, self.BN_p, self.BN_next_p, self.J, self.M,
                                 ke, ws=self.ws)
            self.species, self._spare = list(self._spare), list(self.species)
            return
        move_moments(self.grid, self.species, Et, self.BN_p, self.BN_next_p, self.J, self.M, ke, ws=self.ws)

    def regroup_now(self) -> bool:
        """Whether the coming fused pass regroups (the last pass of each period of sort_every)."""
        return self.regroup and (self.nstep + 1) % self.sort_every == 0

    def fused_pass(self, ke: Optional[torch.Tensor] = None):
        """Mover with (E^{n+theta}, B^n), then the moments at x^{n+1/2} with B^{n+1}."""
        self.fused_fields()
        self.fused_particles(ke)

    def advance_fused(self):
        self.advance_fields()
        self.BN, self.BN_next = self.BN_next, self.BN
        if self.prec == F32:
            self.BN_p, self.BN_next_p = self.BN_next_p, self.BN_p
        else:
            self.BN_p, self.BN_next_p = self.BN, self.BN_next
        self.nstep += 1
        if not self.regroup and self.nstep % self.sort_every == 0:
            self.sort_particles()

    def step(self):
        if self.fused:
            if not self.primed:
                self.prime()
            self.solve()
            self.scal[0] = 0.0
            self.fused_pass(self.scal[0:1])
            self.advance_fused()
            return
        if self.do_sort and (self.nstep % self.sort_every == 0 or any(s.cell_start is None for s in self.species)):
            self.sort_particles()
        self.node_B()
        self.deposit()
        self.solve()
        self.scal[0] = 0.0
        self.push(self.scal[0:1])
        self.advance_fields()
        self.nstep += 1

    def energy(self):
        """(W_E, W_B) of the current fields on the host (FP64 device reductions)."""
        field_energy(self.grid, self.E, self.scal[1:2], self.energy_ws)
        field_energy(self.grid, self.BC, self.scal[2:3], self.energy_ws)
        return self.scal[1].item(), self.scal[2].item()
