"""The C-ABI library: loads, exports every declared symbol, validates arguments.

These run without a GPU: argument validation happens on the host before any
HIP call, so invalid calls must return ECSIM_EINVAL / ECSIM_EWORKSPACE.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ecsim.h")


@pytest.fixture(scope="module")
def E():
    from paper_2603_16624_amd import ecsim
    if not os.path.exists(ecsim.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return ecsim


def declared_symbols():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ecsim_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_the_hot_path(E):
    names = declared_symbols()
    for required in ("ecsim_move", "ecsim_moments", "ecsim_mass_apply", "ecsim_moments_backward"):
        assert required in names


def test_library_exports_every_declared_symbol(E):
    L = E.lib()
    for name in declared_symbols():
        assert hasattr(L, name), name
    assert sorted(E.EXPORTED) == declared_symbols()


def test_version(E):
    assert "gfx950" in E.version()


def _grid(E, n=(4, 4, 4), h=(0.5, 0.5, 0.5), dt=0.1):
    return E.Grid(n, h, dt).c()


def test_invalid_grid_rejected(E):
    L = E.lib()
    out = ctypes.c_size_t(0)
    for n, h, dt in [((0, 4, 4), (0.5,) * 3, 0.1), ((4, 4, 4), (0.5, -1.0, 0.5), 0.1),
                     ((4, 4, 4), (0.5,) * 3, 0.0), ((4, 4, 4), (0.5, float("nan"), 0.5), 0.1)]:
        g = E.Grid(n, h, dt).c()
        st = L.ecsim_workspace_size(ctypes.byref(g), 10, E.F64, 0, ctypes.byref(out))
        assert st == E.EINVAL
        assert b"grid" in L.ecsim_last_error()
    assert L.ecsim_workspace_size(None, 10, E.F64, 0, ctypes.byref(out)) == E.EINVAL
    assert L.ecsim_workspace_size(ctypes.byref(_grid(E)), 10, 7, 0, ctypes.byref(out)) == E.EINVAL


def test_workspace_size_positive(E):
    L = E.lib()
    out = ctypes.c_size_t(0)
    assert L.ecsim_workspace_size(ctypes.byref(_grid(E)), 1000, E.F32, 0, ctypes.byref(out)) == E.OK
    assert out.value >= 2 * 4 * 1000 + 4 * 64


def _particles(E, prec=0, np_=8, qom=-1.0, cell=False, ptr=0x1000):
    p = E._Particles()
    p.prec = prec
    p.np = np_
    p.qom = qom
    for d in range(3):
        p.pos[d] = ptr
        p.vel[d] = ptr
    p.cell = ptr if cell else None
    p.q = None
    p.q_const = 1.0
    p.cell_start = None
    return p


def test_move_argument_validation(E):
    L = E.lib()
    g = _grid(E)
    fake = ctypes.c_void_p(0x1000)
    # NULL fields
    p = _particles(E)
    assert L.ecsim_move(ctypes.byref(g), ctypes.byref(p), None, fake, None, None) == E.EINVAL
    # FP32 without a cell array
    p = _particles(E, prec=E.F32)
    assert L.ecsim_move(ctypes.byref(g), ctypes.byref(p), fake, fake, None, None) == E.EINVAL
    assert b"cell" in L.ecsim_last_error()
    # FP64 with a cell array
    p = _particles(E, prec=E.F64, cell=True)
    assert L.ecsim_move(ctypes.byref(g), ctypes.byref(p), fake, fake, None, None) == E.EINVAL
    # zero charge-to-mass ratio, negative np, bad precision
    for kw in (dict(qom=0.0), dict(np_=-1), dict(prec=3)):
        p = _particles(E, **kw)
        assert L.ecsim_move(ctypes.byref(g), ctypes.byref(p), fake, fake, None, None) == E.EINVAL
    # NULL position pointer with np > 0
    p = _particles(E)
    p.pos[1] = None
    assert L.ecsim_move(ctypes.byref(g), ctypes.byref(p), fake, fake, None, None) == E.EINVAL


def test_moments_argument_validation(E):
    L = E.lib()
    g = _grid(E)
    fake = ctypes.c_void_p(0x1000)
    arr = (E._Particles * 2)(_particles(E), _particles(E, prec=E.F32, cell=True))
    # mixed precisions
    assert L.ecsim_moments(ctypes.byref(g), arr, 2, fake, fake, fake, None, 0, 0, None) == E.EINVAL
    arr = (E._Particles * 1)(_particles(E))
    # nspecies out of range, unknown flags, sorted without cell_start, NULL outputs
    assert L.ecsim_moments(ctypes.byref(g), arr, 0, fake, fake, fake, None, 0, 0, None) == E.EINVAL
    assert L.ecsim_moments(ctypes.byref(g), arr, 1, fake, fake, fake, None, 0, 0x80, None) == E.EINVAL
    assert L.ecsim_moments(ctypes.byref(g), arr, 1, fake, fake, fake, None, 0, E.SORTED, None) == E.EINVAL
    assert L.ecsim_moments(ctypes.byref(g), arr, 1, fake, None, fake, None, 0, 0, None) == E.EINVAL


def test_mass_apply_and_solve_validation(E):
    L = E.lib()
    g = _grid(E)
    fake = ctypes.c_void_p(0x1000)
    # aliasing x and y
    assert L.ecsim_mass_apply(ctypes.byref(g), E.F64, fake, fake, 1.0, 0.0, fake, None) == E.EINVAL
    assert L.ecsim_mass_apply(ctypes.byref(g), 5, fake, fake, 1.0, 0.0, ctypes.c_void_p(0x2000), None) == E.EINVAL
    out = ctypes.c_size_t(0)
    assert L.ecsim_solve_workspace_size(ctypes.byref(g), 0, ctypes.byref(out)) == E.EINVAL
    assert L.ecsim_solve_workspace_size(ctypes.byref(g), 30, ctypes.byref(out)) == E.OK
    need = out.value
    it = ctypes.c_int32(0)
    res = ctypes.c_double(0)
    args = [ctypes.byref(g), E.F64, fake, fake, fake, fake, 1e-10, 30, 100, fake, fake, fake]
    # workspace too small
    st = L.ecsim_field_solve(*args, fake, need - 1, ctypes.byref(it), ctypes.byref(res), None)
    assert st == E.EWORKSPACE
    # tolerance out of range
    bad = list(args)
    bad[6] = 0.0
    assert L.ecsim_field_solve(*bad, fake, need, ctypes.byref(it), ctypes.byref(res), None) == E.EINVAL
    # 2^29 cells: beyond the 32-bit byte offsets of the operator kernels
    big = E.Grid((1024, 1024, 512), (1.0, 1.0, 1.0), 0.1).c()
    assert L.ecsim_mass_apply(ctypes.byref(big), E.F64, fake, fake, 1.0, 0.0, ctypes.c_void_p(0x2000), None) == E.EINVAL
    big_args = [ctypes.byref(big)] + args[1:]
    assert L.ecsim_field_solve(*big_args, fake, 1 << 62, ctypes.byref(it), ctypes.byref(res), None) == E.EINVAL
    assert b"2^29" in L.ecsim_last_error()


def test_sort_and_backward_validation(E):
    L = E.lib()
    g = _grid(E)
    fake = ctypes.c_void_p(0x1000)
    src = _particles(E, ptr=0x1000)
    dst = _particles(E, ptr=0x1000)   # aliases src
    assert L.ecsim_sort(ctypes.byref(g), ctypes.byref(src), ctypes.byref(dst), fake, None, fake, 1 << 20, None) == E.EINVAL
    dst = _particles(E, ptr=0x9000)
    assert L.ecsim_sort(ctypes.byref(g), ctypes.byref(src), ctypes.byref(dst), fake, None, fake, 1, None) == E.EWORKSPACE
    p = _particles(E)
    gp = (ctypes.c_void_p * 3)(0x1000, 0x1000, 0x1000)
    # through the mover without E
    st = L.ecsim_moments_backward(ctypes.byref(g), ctypes.byref(p), None, fake, fake, fake, gp, gp, fake, fake,
                                  None, 0, E.BWD_THROUGH_MOVER, None)
    assert st == E.EINVAL
    st = L.ecsim_moments_backward(ctypes.byref(g), ctypes.byref(p), fake, fake, fake, fake, gp, gp, fake, fake,
                                  None, 0, 0x40, None)
    assert st == E.EINVAL
    # grouped particles (cell_start) need the workspace of the tiled kernel:
    # the list count, a list entry per particle and a 268-value table per cell
    need = ctypes.c_size_t(0)
    assert L.ecsim_backward_workspace_size(ctypes.byref(g), p.np, p.prec, ctypes.byref(need)) == E.OK
    assert need.value >= 256 + 4 * p.np + 268 * 8 * 64
    need32 = ctypes.c_size_t(0)
    assert L.ecsim_backward_workspace_size(ctypes.byref(g), p.np, E.F32, ctypes.byref(need32)) == E.OK
    assert 268 * 4 * 64 <= need32.value < need.value
    assert L.ecsim_backward_workspace_size(ctypes.byref(g), -1, p.prec, ctypes.byref(need)) == E.EINVAL
    assert L.ecsim_backward_workspace_size(ctypes.byref(g), p.np, 7, ctypes.byref(need)) == E.EINVAL
    assert L.ecsim_backward_workspace_size(ctypes.byref(g), p.np, p.prec, None) == E.EINVAL
    assert L.ecsim_backward_workspace_size(None, p.np, p.prec, ctypes.byref(need)) == E.EINVAL
    L.ecsim_backward_workspace_size(ctypes.byref(g), p.np, p.prec, ctypes.byref(need))
    p.cell_start = ctypes.c_void_p(0x5000)
    st = L.ecsim_moments_backward(ctypes.byref(g), ctypes.byref(p), fake, fake, fake, fake, gp, gp, fake, fake,
                                  fake, need.value - 1, E.BWD_THROUGH_MOVER, None)
    assert st == E.EWORKSPACE
    st = L.ecsim_moments_backward(ctypes.byref(g), ctypes.byref(p), fake, fake, fake, fake, gp, gp, fake, fake,
                                  None, need.value, E.BWD_THROUGH_MOVER, None)
    assert st == E.EWORKSPACE


def test_diagnostics_argument_validation(E):
    """ecsim_diagnostics validates before launching anything (no GPU needed)."""
    L = E.lib()
    g = _grid(E)
    fake = ctypes.c_void_p(0x1000)
    arr = (E._Particles * 2)(_particles(E), _particles(E, prec=E.F32, cell=True))
    # mixed precisions
    assert L.ecsim_diagnostics(ctypes.byref(g), arr, 2, fake, fake, fake, None, 0, 0, None) == E.EINVAL
    arr = (E._Particles * 1)(_particles(E))
    # no species, unknown flags, sorted without cell_start, NULL outputs
    assert L.ecsim_diagnostics(ctypes.byref(g), arr, 0, fake, fake, fake, None, 0, 0, None) == E.EINVAL
    assert L.ecsim_diagnostics(ctypes.byref(g), arr, 1, fake, fake, fake, None, 0, 0x80, None) == E.EINVAL
    assert L.ecsim_diagnostics(ctypes.byref(g), arr, 1, fake, fake, fake, None, 0, E.SORTED, None) == E.EINVAL
    for outs in ((None, fake, fake), (fake, None, fake), (fake, fake, None)):
        assert L.ecsim_diagnostics(ctypes.byref(g), arr, 1, *outs, None, 0, 0, None) == E.EINVAL
    assert b"ecsim_diagnostics" in L.ecsim_last_error()


def test_diagnostics_workspace_size(E):
    L = E.lib()
    g = _grid(E)   # 4^3 nodes
    out = ctypes.c_size_t(0)
    assert L.ecsim_diagnostics_workspace_size(ctypes.byref(g), E.F32, 0, ctypes.byref(out)) == E.OK
    assert out.value == 8 * 10 * 64
    assert L.ecsim_diagnostics_workspace_size(ctypes.byref(g), E.F64, 0, ctypes.byref(out)) == E.OK
    assert out.value == 0
    assert L.ecsim_diagnostics_workspace_size(ctypes.byref(g), E.F32, E.SORTED, ctypes.byref(out)) == E.OK
    assert out.value == 256
    assert L.ecsim_diagnostics_workspace_size(ctypes.byref(g), 9, 0, ctypes.byref(out)) == E.EINVAL
    assert L.ecsim_diagnostics_workspace_size(ctypes.byref(g), E.F32, 0x40, ctypes.byref(out)) == E.EINVAL
    assert L.ecsim_diagnostics_workspace_size(ctypes.byref(g), E.F32, 0, None) == E.EINVAL
    # FP32 without SORTED needs the workspace
    fake = ctypes.c_void_p(0x1000)
    arr = (E._Particles * 1)(_particles(E, prec=E.F32, cell=True))
    assert L.ecsim_diagnostics(ctypes.byref(g), arr, 1, fake, fake, fake, None, 0, 0, None) == E.EWORKSPACE


def test_move_moments_regroup_validation(E):
    """ecsim_move_moments_regroup rejects mismatched, incomplete or aliasing targets before any launch."""
    L = E.lib()
    g = _grid(E)
    fake = ctypes.c_void_p(0x1000)
    gp = lambda p, cs: (setattr(p, "cell_start", cs), p)[1]
    src = (E._Particles * 1)(gp(_particles(E, prec=E.F32, cell=True, ptr=0x1000), 0x5000))

    def call(dst, ns=1, s=src, ws=fake, wsb=1 << 40):
        return L.ecsim_move_moments_regroup(ctypes.byref(g), s, dst, ns, fake, fake, fake, fake, fake, None, ws, wsb,
                                            0, None)

    good = lambda **kw: gp(_particles(E, prec=E.F32, cell=True, ptr=0x9000, **kw), 0x6000)
    assert call(None) == E.EINVAL
    assert call((E._Particles * 1)(gp(_particles(E, prec=E.F32, cell=True, ptr=0x9000), None))) == E.EINVAL
    assert b"cell_start" in L.ecsim_last_error()
    assert call((E._Particles * 1)(good(np_=9))) == E.EINVAL                  # size differs
    assert call((E._Particles * 1)(gp(_particles(E, prec=E.F64, ptr=0x9000), 0x6000))) == E.EINVAL   # precision
    d = good()
    d.q = ctypes.c_void_p(0x9100)                                             # charge array where the source has none
    assert call((E._Particles * 1)(d)) == E.EINVAL
    d = good()
    d.vel[2] = ctypes.c_void_p(0x1000)                                        # aliases a source array
    assert call((E._Particles * 1)(d)) == E.EINVAL
    assert b"alias" in L.ecsim_last_error()
    d = good()
    d.cell_start = ctypes.c_void_p(0x5000)                                    # aliases the source ranges
    assert call((E._Particles * 1)(d)) == E.EINVAL
    assert call((E._Particles * 1)(good()), ws=None, wsb=0) == E.EWORKSPACE
    # species x cells beyond the int32 ranges
    big = E.Grid((1290, 1290, 1290), (0.5,) * 3, 0.1).c()   # 2,146,689,000 cells, 4 species: > 2^31 entries
    src4 = (E._Particles * 4)(*[gp(_particles(E, prec=E.F32, cell=True, ptr=0x1000 + 0x100 * i), 0x5000 + i)
                                for i in range(4)])
    dst4 = (E._Particles * 4)(*[gp(_particles(E, prec=E.F32, cell=True, ptr=0x9000 + 0x100 * i), 0x6000 + i)
                                for i in range(4)])
    assert L.ecsim_move_moments_regroup(ctypes.byref(big), src4, dst4, 4, fake, fake, fake,
                                        fake, fake, None, fake, 1 << 40, 0, None) == E.EINVAL
    assert b"exceeds" in L.ecsim_last_error()


def test_move_moments_noalloc_validation(E):
    """The static-scratch pass rejects bad arguments and inputs beyond its scratch before any launch."""
    L = E.lib()
    g = _grid(E)
    fake = ctypes.c_void_p(0x1000)
    gp = lambda p, cs: (setattr(p, "cell_start", cs), p)[1]

    def call(parts, ns=1, flags=0, J=fake):
        return L.ecsim_move_moments_noalloc(ctypes.byref(g), parts, ns, fake, fake, fake, J, fake, None, flags,
                                            None)

    small = (E._Particles * 1)(gp(_particles(E, prec=E.F32, cell=True), 0x5000))
    assert call(small, flags=0x100) == E.EINVAL
    assert call(small, J=None) == E.EINVAL
    assert call((E._Particles * 1)(gp(_particles(E, prec=E.F32, cell=True), None))) == E.EINVAL   # no ranges
    need = ctypes.c_size_t(0)
    for prec, np_ in ((E.F32, 2_000_000), (E.F64, 600_000)):
        assert L.ecsim_workspace_size(ctypes.byref(g), np_, prec, 0, ctypes.byref(need)) == E.OK
        assert need.value > E.NOALLOC_SCRATCH_BYTES
        big = (E._Particles * 1)(gp(_particles(E, prec=prec, np_=np_, cell=prec == E.F32), 0x5000))
        assert call(big) == E.EWORKSPACE
        assert b"scratch" in L.ecsim_last_error()


def test_sorted_species_limits_are_errors(E):
    """With ECSIM_SORTED more than 4 species is an error, not a silent switch to the any-order deposit."""
    L = E.lib()
    g = _grid(E)
    fake = ctypes.c_void_p(0x1000)
    sp = []
    for i in range(5):
        p = _particles(E, ptr=0x1000 + 0x100 * i)
        p.cell_start = 0x8000 + 0x100 * i
        sp.append(p)
    arr = (E._Particles * 5)(*sp)
    assert L.ecsim_moments(ctypes.byref(g), arr, 5, fake, fake, fake, fake, 1 << 40, E.SORTED, None) == E.EINVAL
    assert b"at most 4 species" in L.ecsim_last_error()
    assert L.ecsim_diagnostics(ctypes.byref(g), arr, 5, fake, fake, fake, fake, 1 << 40, E.SORTED, None) == E.EINVAL
    assert b"at most 4 species" in L.ecsim_last_error()


def test_nonfinite_api_validation(E):
    """The non-finite status code and the checks' host-side validation."""
    L = E.lib()
    assert E.ENONFINITE == -4
    txt = open(HEADER).read()
    assert "ECSIM_ENONFINITE = -4" in txt
    assert L.ecsim_nonfinite_read(None, None) == E.EINVAL
    assert b"flag_out" in L.ecsim_last_error()


def test_offset_gradient_flag_needs_fp32(E):
    L = E.lib()
    g = _grid(E)
    fake = ctypes.c_void_p(0x1000)
    gp = (ctypes.c_void_p * 3)(0x1000, 0x1000, 0x1000)
    p = _particles(E)   # FP64
    st = L.ecsim_moments_backward(ctypes.byref(g), ctypes.byref(p), fake, fake, fake, fake, gp, gp, fake, fake,
                                  None, 0, E.BWD_THROUGH_MOVER | E.BWD_OFFSET_GRAD, None)
    assert st == E.EINVAL
    assert b"OFFSET_GRAD" in L.ecsim_last_error()
