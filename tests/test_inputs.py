"""Seeded synthetic workloads: sizes, charges and the FP32 storage form."""
import math

import numpy as np


def test_config0_shape_and_charges(inputs):
    p = inputs.config0()
    assert p.n == (8, 8, 8)
    assert [s.np for s in p.species] == [13824, 13824]
    qe = p.species[0].q_uniform
    qi = p.species[1].q_uniform
    assert abs(qe + 0.125 / 27 / (4 * math.pi)) < 1e-18
    assert abs(qi - 0.125 / 27 / (4 * math.pi)) < 1e-18
    # exactly 27 particles per cell, inside the box
    for s in p.species:
        cell = (np.floor(s.x[0] / 0.5) + 8 * (np.floor(s.x[1] / 0.5) + 8 * np.floor(s.x[2] / 0.5))).astype(int)
        assert np.all(np.bincount(cell, minlength=512) == 27)
        assert np.all((s.x >= 0) & (s.x < 4.0))


def test_seeded_reproducible(inputs):
    a = inputs.config0()
    b = inputs.config0()
    for s, t in zip(a.species, b.species):
        assert np.array_equal(s.x, t.x) and np.array_equal(s.v, t.v)


def test_thermal_speeds(inputs):
    p = inputs.uniform_plasma(5, (16, 16, 16), 16)
    assert abs(np.std(p.species[0].v) / 0.05 - 1) < 0.01
    assert abs(np.std(p.species[1].v) / 0.01 - 1) < 0.01


def test_perturbed_electron_density(inputs):
    p = inputs.config1(ppc=8, n=(32, 8, 8))
    xe = p.species[0].x[0]
    assert xe.size == 8 * 32 * 8 * 8
    L = 16.0
    # first Fourier coefficient of the density: 0.01/2 relative amplitude (1.01 normalisation)
    c = np.mean(np.cos(2 * math.pi * xe / L))
    assert abs(c - 0.005 / 1.0) < 4.0 / math.sqrt(xe.size)


def test_f32_encoding_is_exact_on_decode(inputs):
    p = inputs.config0()
    st = inputs.to_f32_state(p)
    for s, f in zip(p.species, st):
        assert f["cell"].dtype == np.int32 and f["off"].dtype == np.float32
        assert np.all((f["off"] >= 0) & (f["off"] < 1))
        # decode then encode again is the identity
        c2, o2 = inputs.encode_f32(f["x64"], p.n, p.h)
        assert np.array_equal(c2, f["cell"]) and np.array_equal(o2, f["off"])
        assert np.max(np.abs(f["x64"] - s.x)) < 0.5 * 2 ** -24


def test_harris_structure(inputs):
    p = inputs.harris(n=(8, 128, 2), ppc=4)
    # B_x = -B0 outside the two sheets and +B0 between them
    bx = p.B_C[0].reshape(2, 128, 8)[0, :, 0]
    assert bx.min() < -0.09 and bx.max() > 0.09
    # both species sample the same density profile: near neutrality
    qe = p.species[0].q.sum()
    qi = p.species[1].q.sum()
    assert abs(qe + qi) < 1e-2 * abs(qi)


def test_four_species_2d_structure(inputs):
    """The four-species 2D stand-in, at a reduced size: grouped by cell (ppc of
    each species per cell, in cell order, ranges as cell_start), offsets in
    [0, 1), total charge zero, the electron beams drifting +-0.1 along x."""
    import numpy as np
    n, ppc = (8, 6, 1), 50
    sp = list(inputs.four_species_2d_f32(n=n, ppc=ppc))
    assert len(sp) == 4
    nc = n[0] * n[1]
    total = 0.0
    for d in sp:
        assert d["cell"].dtype == np.int32 and d["off"].dtype == np.float32 and d["v"].dtype == np.float32
        assert np.array_equal(d["cell"], np.repeat(np.arange(nc), ppc))
        assert np.array_equal(d["cell_start"], np.arange(nc + 1) * ppc)
        assert d["off"].min() >= 0.0 and d["off"].max() < 1.0
        total += d["q"] * d["cell"].size
    assert abs(total) < 1e-12 * sum(abs(d["q"]) * d["cell"].size for d in sp)
    assert abs(sp[0]["v"][0].mean() - 0.1) < 0.01 and abs(sp[1]["v"][0].mean() + 0.1) < 0.01
    assert abs(sp[0]["v"][1].std() - 0.05) < 0.005 and abs(sp[2]["v"][1].std() - 0.01) < 0.001
