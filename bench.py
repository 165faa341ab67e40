#!/usr/bin/env python3
"""Benchmark of the ECsim per-step particle hot path on one MI355X.

Workload (synthetic, seeded): 64^3 periodic cells, cell size 0.5 d_e, dt = 0.1,
two species (electrons q/m = -1, ions q/m = 1/25) with 64 particles per cell
each (33,554,432 particles), Maxwellian velocities (v_th 0.05 / 0.01),
electron density perturbed by 1% cos(2 pi x / L_x), B0 = (0, 0, 0.2), E = 0.

One step is the scheme's step: FP64 GMRES field solve (tol 1e-10) for
E^{n+theta}, then one fused particle pass -- mover with (E^{n+theta}, B^n) and
the moment gather (J-hat, M) at the new positions with B^{n+1}, i.e. the next
step's moments -- on the cell grouping that every --sort-every-th pass
rewrites (ecsim_move_moments_regroup: that pass also writes the particles
regrouped by cell; with --no-regroup a counting re-sort every --sort-every
steps keeps the grouping instead). The metric is particles per second
through mover + moments (the fused pass, with the regrouping pass's extra
cost or the re-sort amortised over the period), in the FP32 storage form
(headline) and the FP64 form;
the field solve runs in every step and is reported separately. Times are HIP
events on the stream the kernels run on, inside a region bracketed by device
synchronisation.

Prints one JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM bytes of one FP32 ecsim_move_moments call on the 64^3 workload, from the
# FETCH_SIZE and WRITE_SIZE passes summarised in the profile named below
# (scaled by a 1 GiB device copy). Valid only for the kernel sources whose
# hash is recorded; any change to them makes the figure stale (reported null).
TRAFFIC = {"sources_sha256": "a44d262f9708bbb83ff74759b2dc4f7b8b5da6625910ad36ad87e42da61d9c81",
           "plain_call": 3799674858,     # a fused call on the grouping the last regrouping left
           "regroup_call": 5397404139,   # a regrouping call after three plain ones
           "profile": "profiles/move_moments_64cubed_fp32.md"}


def kernel_sources_sha256():
    import glob
    import hashlib
    h = hashlib.sha256()
    # every source the fused pass is built from (the adjoint's is not)
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2603_16624_amd", "csrc", "*"))):
        if os.path.basename(f) == "adjoint.hip":
            continue
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--ppc", type=int, default=64)
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 form")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=8, help="oracle runs on 1/cpu-sample of the particles")
    ap.add_argument("--sort-every", type=int, default=4)
    ap.add_argument("--regroup", dest="regroup", action="store_true", default=True,
                    help="fused path: every --sort-every-th pass regroups the particles by cell (default)")
    ap.add_argument("--no-regroup", dest="regroup", action="store_false",
                    help="fused path: re-sort with a counting sort every --sort-every steps instead")
    ap.add_argument("--no-error", action="store_true", help="skip the FP32-vs-FP64 error measurement")
    ap.add_argument("--calib-copy", action="store_true", help="end with a 1 GiB device copy (byte-counter reference)")
    ap.add_argument("--no-extras", action="store_true", help="skip the apply and adjoint timings")
    ap.add_argument("--path", choices=("fused", "split"), default="fused",
                    help="fused: one mover+moments kernel; split: mover, then the tiled deposit")
    return ap.parse_args()


def algorithmic_bytes(prec, nparticles, nn, q_read=0):
    """Bytes the fused mover + moments pass must move per step.

    Per particle: the state (positions + velocities [+ cell]) read once and
    written once, and a per-particle charge read (``q_read`` particles, none
    when every particle of a species has the same charge); per node:
    E^{n+theta}, B^n and B^{n+1} read, J-hat and the 14 x 9 mass-matrix
    entries written once.
    """
    part, fld = (28, 4) if prec == "f32" else (48, 8)
    return 2 * part * nparticles + fld * q_read + fld * (9 + 3 + 126) * nn


def _median(a):
    a = sorted(a)
    n = len(a)
    return 0.5 * (a[(n - 1) // 2] + a[n // 2]) if n else 0.0


def run_form(prec, args, plasma):
    import torch
    from paper_2603_16624_amd import ecsim as E
    P = E.F32 if prec == "f32" else E.F64
    fused = args.path == "fused"
    sim = E.Simulation(plasma, prec=P, tol=1e-10, fused=fused, sort=True, sort_every=args.sort_every,
                       regroup=fused and args.regroup)
    st = torch.cuda.current_stream()
    ev = lambda: torch.cuda.Event(enable_timing=True)
    if fused:
        sim.prime()
    else:
        sim.sort_particles()
        sim.node_B()
        sim.deposit()

    # events: 0 solve 1 | 2 field prep 3 particle kernels 4 | re-sort 5 | 6 (split: moments) 7
    def one_step(record):
        e = [ev() for _ in range(8)]
        e[0].record(st)
        sim.solve()
        e[1].record(st)
        sim.scal[0] = 0.0
        e[2].record(st)
        rg = fused and sim.regroup_now()
        if fused:
            sim.fused_fields()
            e[3].record(st)
            sim.fused_particles(sim.scal[0:1])
        else:
            if sim.prec == E.F32:
                E.to_f32(sim.E_theta, sim.Et_p)
            e[3].record(st)
            sim.push(sim.scal[0:1])
        e[4].record(st)
        sim.advance_fields()
        if fused:
            sim.BN, sim.BN_next = sim.BN_next, sim.BN
            if sim.prec == E.F32:
                sim.BN_p, sim.BN_next_p = sim.BN_next_p, sim.BN_p
            else:
                sim.BN_p, sim.BN_next_p = sim.BN, sim.BN_next
        sim.nstep += 1
        sorted_now = not sim.regroup and sim.nstep % sim.sort_every == 0
        if sorted_now:
            sim.sort_particles()
        e[5].record(st)
        e[6].record(st)
        if not fused:
            sim.node_B()
            sim.deposit()
        e[7].record(st)
        if record is not None:
            record.append((e, sorted_now, rg))

    for _ in range(args.warmup):
        one_step(None)
    torch.cuda.synchronize()
    rec = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        one_step(rec)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    el = lambda i, j: [e[i].elapsed_time(e[j]) for e, *_ in rec]
    solve_ms = _median(el(0, 1))
    fields_ms = _median(el(2, 3))
    kernel_ms = _median(el(3, 4))            # fused: the ecsim_move_moments call; split: the mover
    plain_call_ms = regroup_call_ms = None
    if fused and sim.regroup:
        # every sort_every-th pass regroups: its cost is amortised over the
        # period as a re-sort's would be (a regrouping pass is timed after the
        # K steps if none fell inside them)
        rg_t = [e[3].elapsed_time(e[4]) for e, _, r in rec if r]
        pl_t = [e[3].elapsed_time(e[4]) for e, _, r in rec if not r]
        while not rg_t:
            extra = []
            one_step(extra)
            torch.cuda.synchronize()
            if extra[0][2]:
                rg_t.append(extra[0][0][3].elapsed_time(extra[0][0][4]))
        regroup_call_ms = _median(rg_t)
        plain_call_ms = _median(pl_t) if pl_t else regroup_call_ms
        kernel_ms = plain_call_ms + (regroup_call_ms - plain_call_ms) / sim.sort_every
    moments_ms = 0.0 if fused else _median(el(6, 7))
    resort = [e[4].elapsed_time(e[5]) for e, s_, _ in rec if s_]
    sort_ms = _median(resort) if resort else 0.0
    full_ms = _median(el(0, 7))
    pass_ms = fields_ms + kernel_ms + moments_ms + sort_ms / args.sort_every
    npart = plasma.n_particles
    q_read = sum(sp.np for sp in plasma.species if sp.q_uniform is None)
    nbytes = algorithmic_bytes(prec, npart, plasma.nn, q_read)
    out = dict(prec=prec, path=args.path, particles=npart, pass_ms=pass_ms, fields_ms=fields_ms, kernel_ms=kernel_ms,
               plain_call_ms=plain_call_ms, regroup_call_ms=regroup_call_ms,
               moments_ms=moments_ms, sort_ms=sort_ms, sort_every=args.sort_every, solve_ms=solve_ms,
               full_step_ms=full_ms, wall_s=wall, gmres_iters=sim.last_iters, gmres_resid=sim.last_resid,
               particles_per_s=npart / (pass_ms * 1e-3),
               # the grouping renewed every step: by the regrouping pass, or by the re-sort
               particles_per_s_with_sort_every_step=(
                   npart / ((fields_ms + regroup_call_ms) * 1e-3) if regroup_call_ms is not None
                   else npart / ((pass_ms - sort_ms / args.sort_every + sort_ms) * 1e-3) if sort_ms else None),
               bytes_per_step=nbytes, hbm_frac_pass=nbytes / (pass_ms * 1e-3) / (HBM_PEAK_GBS * 1e9),
               kernel_gbs=nbytes / (kernel_ms * 1e-3) / 1e9 if fused else None)
    del sim
    torch.cuda.empty_cache()
    return out


def fixed_error(plasma, steps=5):
    """FP32-form error against the FP64 path on the full workload, step by step.

    Both forms start from the same state (the FP32 form is the FP64 state
    encoded as cell + offset) and run `steps` steps of the loop side by side
    (field solve, fused pass with the regrouping every 4 steps). After each
    step the relative max-norm differences of J-hat and M (the next step's
    moments) and of E^{n+1} are recorded; the FP64 path itself agrees with the
    FP64 oracle to 1e-12 (the oracle is too slow for 33.5M particles a step).
    """
    import torch
    from paper_2603_16624_amd import ecsim as E
    sims = {P: E.Simulation(plasma, prec=P, tol=1e-10, fused=True, regroup=True) for P in (E.F64, E.F32)}
    rel = lambda a, b: float((a.double() - b.double()).abs().max() / b.double().abs().max())
    per_step = []
    for _ in range(steps):
        for sim in sims.values():
            sim.step()
        torch.cuda.synchronize()
        s64, s32 = sims[E.F64], sims[E.F32]
        per_step.append({"J": rel(s32.J, s64.J), "M": rel(s32.M, s64.M), "E": rel(s32.E, s64.E)})
    del sims
    torch.cuda.empty_cache()
    worst = {k: max(d[k] for d in per_step) for k in ("J", "M", "E")}
    return {**worst, "per_step": per_step, "bound": 1e-5,
            "against": f"FP64 path from the same initial state, after each of {steps} steps"}


def calibrate_copy():
    """A plain device-to-device copy of 1 GiB, three times: the reference for the HBM byte counters."""
    import torch
    x = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    x.fill_(1.0)
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    del x, y
    torch.cuda.empty_cache()


def cpu_baseline(plasma, sample):
    """The FP64 oracle's mover + moments on 1/sample of the particles, on the host."""
    import numpy as np
    from oracle import oracle as O
    rng = np.random.default_rng(12345)
    BN = O.centres_to_nodes(plasma.n, plasma.B_C)
    En = 1e-4 * rng.standard_normal((3, plasma.nn))
    nn = plasma.nn
    J = np.zeros((3, nn))
    M27 = np.zeros((27, 9, nn))
    count = 0
    t0 = time.perf_counter()
    for s in plasma.species:
        k = max(1, s.np // sample)
        x = np.ascontiguousarray(s.x[:, :k])
        v = np.ascontiguousarray(s.v[:, :k])
        x1, v1 = O.move(plasma.n, plasma.h, plasma.dt, x, v, s.qom, En, BN)
        O.moments(plasma.n, plasma.h, plasma.dt, x1, v1, s.q[:k], s.qom, BN, J, M27)
        count += k
    dt = time.perf_counter() - t0
    return dict(value=count / dt, unit="particles/s", cores=1, kind="oracle",
                sample=f"FP64 oracle mover+moments on {count} particles (1/{sample} of each species) "
                       f"of the 64^3 workload, single thread, {dt:.1f} s")


def _time_events(fn, reps, warmup=2):
    """Median of per-call durations, HIP events on the current stream."""
    import torch
    for _ in range(warmup):
        fn()
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    return _median(ts)


def mass_apply_rate(n):
    """The 14-block apply inside GMRES, timed alone at n^3 nodes: y = M x with M
    in FP32 and in FP64 (x, y FP64). Algorithmic bytes per node: M (126 values),
    x read and y written (3 FP64 each)."""
    import torch
    from paper_2603_16624_amd import ecsim as E
    nn = n ** 3
    grid = E.Grid((n, n, n), (0.5, 0.5, 0.5), 0.1)
    g = torch.Generator(device="cuda").manual_seed(5)
    x = torch.randn((3, nn), dtype=torch.float64, device="cuda", generator=g)
    y = torch.empty_like(x)
    out = {}
    for name, dt in (("f32_M", torch.float32), ("f64_M", torch.float64)):
        M = torch.randn((14, 9, nn), dtype=torch.float64, device="cuda", generator=g).to(dt)
        ms = _time_events(lambda: E.mass_apply(grid, M, x, y, 1.0, 0.0), 20)
        nbytes = nn * (126 * M.element_size() + 24 + 24)
        out[name] = {"us_per_call": ms * 1e3, "algorithmic_bytes": nbytes, "GB_per_s": nbytes / (ms * 1e-3) / 1e9,
                     "hbm_frac": nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        del M
    return out


def diagnostics_rate(plasma):
    """Diagnostic moments (charge density, current, pressure tensor) of the 64^3
    workload after a sort, FP32 and FP64, tiled path. Algorithmic bytes: the
    particle state read once (FP32 offsets, cell, velocity: 28 B; FP64: 48 B)
    and the 10 output values per node written once."""
    import torch
    from paper_2603_16624_amd import ecsim as E
    from paper_2603_16624_amd import inputs as I
    p = plasma
    grid = E.Grid(p.n, p.h, p.dt)
    out = {}
    for prec in ("f32", "f64"):
        if prec == "f64":
            sp = [E.Species.from_f64(s.qom, s.x, s.v, s.q) for s in p.species]
            tdt, pb = torch.float64, 48
        else:
            sp = [E.Species.from_f32(s.qom, f["cell"], f["off"], f["v"], f["q"])
                  for s, f in zip(p.species, I.to_f32_state(p))]
            tdt, pb = torch.float32, 28
        grp = []
        for s in sp:
            d = s.empty_like()
            E.sort(grid, s, d, torch.empty(grid.nn + 1, dtype=torch.int32, device="cuda"))
            grp.append(d)
        del sp
        rho = torch.empty(p.nn, dtype=tdt, device="cuda")
        Jd = torch.empty((3, p.nn), dtype=tdt, device="cuda")
        P = torch.empty((6, p.nn), dtype=tdt, device="cuda")
        ws = torch.empty(E.diagnostics_workspace_size(grid, grp[0].prec, E.SORTED), dtype=torch.uint8, device="cuda")
        ms = _time_events(lambda: E.diagnostics(grid, grp, rho, Jd, P, flags=E.SORTED, ws=ws), 5)
        nbytes = p.n_particles * pb + 10 * p.nn * (8 if prec == "f64" else 4)
        out[prec] = {"ms": ms, "particles_per_s": p.n_particles / (ms * 1e-3), "GB_per_s": nbytes / (ms * 1e-3) / 1e9,
                     "hbm_frac": nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        del grp, rho, Jd, P
        torch.cuda.empty_cache()
    return out


def two_d_rate(args):
    """The paper's 2D shape (Sec. IV, GPU generations: 128 x 128 cells, 6400
    particles per cell) as a reduced run: 128 x 128 x 1 cells, 3200 particles
    per cell per species, 2 species (104,857,600 particles), FP32 form, fused
    pass, same protocol as the headline line."""
    from paper_2603_16624_amd import inputs as I
    import torch
    t0 = time.perf_counter()
    p = I.uniform_plasma(2000, (128, 128, 1), 3200)
    p.name = "128x128x1 cells x 3200 ppc x 2 species (2D)"
    r = run_form("f32", args, p)
    keys = ("pass_ms", "kernel_ms", "sort_ms", "solve_ms", "particles_per_s", "particles_per_s_with_sort_every_step",
            "hbm_frac_pass", "kernel_gbs")
    out = {k: r[k] for k in keys}
    out.update(workload=p.name, particles=p.n_particles, wall_s=time.perf_counter() - t0)
    del p
    torch.cuda.empty_cache()
    return out


def harris_rate(args):
    """The double Harris current sheet, 256 x 128 x 8 cells x 128 ppc x 2 species
    (67,108,864 particles, each with its own charge), FP32 form, fused pass,
    same protocol as the headline line."""
    from paper_2603_16624_amd import inputs as I
    import torch
    t0 = time.perf_counter()
    p = I.harris()
    r = run_form("f32", args, p)
    keys = ("pass_ms", "kernel_ms", "sort_ms", "solve_ms", "gmres_iters", "particles_per_s",
            "particles_per_s_with_sort_every_step", "bytes_per_step", "hbm_frac_pass", "kernel_gbs")
    out = {k: r[k] for k in keys}
    out.update(workload=p.name, particles=p.n_particles, wall_s=time.perf_counter() - t0)
    del p
    torch.cuda.empty_cache()
    return out


def four_species_2d_rate(steps=5):
    """The paper's four-species 2D shape, 256 x 128 x 1 cells x 4 species x
    3600 particles per cell (471,859,200 particles), FP32 form: the
    regrouping fused pass (ecsim_move_moments_regroup) with fixed fields
    (E small noise, B0 = (0, 0, 0.2) with noise), one untimed pass, then
    `steps` timed with HIP events on the pass's stream. The field solve is
    not run (it is outside the metric)."""
    import numpy as np
    import torch
    from paper_2603_16624_amd import ecsim as E
    from paper_2603_16624_amd import inputs as I
    t0 = time.perf_counter()
    sp, grid, nn, npart = [], None, 0, 0
    for d in I.four_species_2d_f32():
        if grid is None:
            grid = E.Grid(d["n"], d["h"], d["dt"])
            nn = grid.nn
        s = E.Species.from_f32(d["qom"], d["cell"], d["off"], d["v"], d["q"])
        s.cell_start = torch.as_tensor(d["cell_start"]).to("cuda")
        npart += s.np
        sp.append(s)
        del d
    gen_s = time.perf_counter() - t0
    rng = np.random.default_rng(5008)
    Ed = torch.as_tensor(1e-3 * rng.standard_normal((3, nn)), dtype=torch.float32).to("cuda")
    Bd = torch.as_tensor(np.array([[0.0], [0.0], [0.2]]) + 0.02 * rng.standard_normal((3, nn)),
                         dtype=torch.float32).to("cuda")
    dst = [s.empty_like() for s in sp]
    J = torch.empty((3, nn), dtype=torch.float32, device="cuda")
    M = torch.empty((14, 9, nn), dtype=torch.float32, device="cuda")
    ws = torch.empty(E.workspace_size(grid, npart, E.F32), dtype=torch.uint8, device="cuda")
    st = torch.cuda.current_stream()
    times = []
    for it in range(steps + 1):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        E.move_moments_regroup(grid, sp, dst, Ed, Bd, Bd, J, M, ws=ws)
        b.record(st)
        torch.cuda.synchronize()
        if it:
            times.append(a.elapsed_time(b))
        sp, dst = dst, sp
    ms = _median(times)
    nbytes = algorithmic_bytes("f32", npart, nn)
    out = {"workload": "256x128x1 cells x 4 species x 3600 ppc (2D), FP32, regrouping pass, fixed fields",
           "particles": npart, "pass_ms": ms, "particles_per_s": npart / (ms * 1e-3),
           "hbm_frac_pass": nbytes / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9), "generation_s": gen_s,
           "wall_s": time.perf_counter() - t0}
    del sp, dst, J, M, ws
    torch.cuda.empty_cache()
    return out


def adjoint_time():
    """Adjoint of mover -> moments (ecsim_moments_backward through the mover) on the
    32^3 x 27 ppc x 2 species workload (1,769,472 particles), FP64 and FP32: time
    of one backward over both species."""
    import numpy as np
    import torch
    from paper_2603_16624_amd import ecsim as E
    from paper_2603_16624_amd import inputs as I
    p = I.config3()
    rng = np.random.default_rng(3009)
    En = 1e-3 * rng.standard_normal((3, p.nn))
    BN = np.array([[0.0], [0.0], [0.2]]) + 1e-3 * rng.standard_normal((3, p.nn))
    gJ = rng.standard_normal((3, p.nn))
    gM = rng.standard_normal((14, 9, p.nn))
    grid = E.Grid(p.n, p.h, p.dt)
    out = {}
    for prec, dt in (("f64", torch.float64), ("f32", torch.float32)):
        if prec == "f64":
            sp = [E.Species.from_f64(s.qom, s.x, s.v, s.q) for s in p.species]
        else:
            sp = [E.Species.from_f32(s.qom, f["cell"], f["off"], f["v"], f["q"])
                  for s, f in zip(p.species, I.to_f32_state(p))]
        dev = lambda a: torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dt)
        Ed, Bd, gJd, gMd = dev(En), dev(BN), dev(gJ), dev(gM)
        gE = torch.zeros((3, p.nn), dtype=dt, device="cuda")
        gB = torch.zeros((3, p.nn), dtype=dt, device="cuda")
        gx = [torch.empty_like(s.pos) for s in sp]
        gv = [torch.empty_like(s.vel) for s in sp]

        def bwd():
            for s, a, b in zip(sp, gx, gv):
                E.moments_backward(grid, s, Ed, Bd, gJd, gMd, a, b, gE, gB, through_mover=True)
        ms = _time_events(bwd, 5)
        out[prec] = {"ms": ms, "particles_per_s": p.n_particles / (ms * 1e-3)}
    out["workload"] = f"{p.n[0]}x{p.n[1]}x{p.n[2]} cells x 27 ppc x 2 species ({p.n_particles} particles)"
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU path is not built",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    from paper_2603_16624_amd import ecsim as E
    from paper_2603_16624_amd import inputs as I
    if not os.path.exists(E.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    t0 = time.perf_counter()
    plasma = I.config1(ppc=args.ppc, n=(args.n, args.n, args.n))
    print(f"[bench] workload generated in {time.perf_counter() - t0:.1f} s: {plasma.name}", file=sys.stderr,
          flush=True)
    r32 = run_form("f32", args, plasma)
    print(f"[bench] f32: {json.dumps(r32)}", file=sys.stderr, flush=True)
    r64 = None
    if not args.no_fp64:
        torch.cuda.empty_cache()
        r64 = run_form("f64", args, plasma)
        print(f"[bench] f64: {json.dumps(r64)}", file=sys.stderr, flush=True)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(plasma, args.cpu_sample)
        print(f"[bench] cpu: {json.dumps(cpu)}", file=sys.stderr, flush=True)
    err = None
    if not args.no_error:
        err = fixed_error(plasma)
        print(f"[bench] fixed error: {json.dumps(err)}", file=sys.stderr, flush=True)
    apply = adjoint = diag = two_d = harris = four_2d = None
    if not args.no_extras:
        apply = mass_apply_rate(args.n)
        print(f"[bench] mass apply: {json.dumps(apply)}", file=sys.stderr, flush=True)
        adjoint = adjoint_time()
        print(f"[bench] adjoint: {json.dumps(adjoint)}", file=sys.stderr, flush=True)
        diag = diagnostics_rate(plasma)
        print(f"[bench] diagnostics: {json.dumps(diag)}", file=sys.stderr, flush=True)
        two_d = two_d_rate(args)
        print(f"[bench] 2d: {json.dumps(two_d)}", file=sys.stderr, flush=True)
        harris = harris_rate(args)
        print(f"[bench] harris: {json.dumps(harris)}", file=sys.stderr, flush=True)
        four_2d = four_species_2d_rate()
        print(f"[bench] 2d four species: {json.dumps(four_2d)}", file=sys.stderr, flush=True)
    if args.calib_copy:
        calibrate_copy()
        print("[bench] copy calibration done", file=sys.stderr, flush=True)
    nbytes = r32["bytes_per_step"]
    if args.path == "fused":
        kname = (f"ecsim_move_moments, with ecsim_move_moments_regroup every {args.sort_every}th pass "
                 "(FP32): fused mover + moment gather, incl. its stray passes, amortised per pass" if args.regroup else
                 "ecsim_move_moments (FP32): fused mover + moment gather, incl. its stray passes")
        kms = r32["kernel_ms"]
    else:
        kname = "ecsim_move + ecsim_moments (FP32, tiled, stale grouping)"
        kms = r32["kernel_ms"] + r32["moments_ms"]
    achieved = nbytes / (kms * 1e-3) / 1e9
    traffic = None
    if (args.path == "fused" and args.regroup and TRAFFIC["regroup_call"]
            and TRAFFIC["sources_sha256"] == kernel_sources_sha256()):
        # per call, amortised over the regrouping period as the times are
        traffic = TRAFFIC["plain_call"] + (TRAFFIC["regroup_call"] - TRAFFIC["plain_call"]) / args.sort_every
    keys = ("fields_ms", "kernel_ms", "plain_call_ms", "regroup_call_ms", "moments_ms", "sort_ms", "solve_ms",
            "full_step_ms")
    out = {
        "metric": "particles/s through mover+moments (FP32 vs FP64) at fixed error; % HBM peak",
        "value": r32["particles_per_s"],
        "unit": "particles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r32["pass_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{plasma.name}; FP32 offset+cell storage, FP32 mover and deposit "
                               f"(Kahan-combined MFMA block sums), FP64 GMRES (tol 1e-10), "
                               + (f"{args.path} path, regrouped by cell in the pass every {args.sort_every} steps"
                                  if args.path == "fused" and args.regroup
                                  else f"{args.path} path, re-sort every {args.sort_every} steps"),
                   "cells": list(plasma.n), "particles": plasma.n_particles, "ppc_per_species": args.ppc,
                   "parallelism": "single GPU"},
        "hbm_frac": r32["hbm_frac_pass"],
        "breakdown_ms": {k: r32[k] for k in keys},
        "sort_every": args.sort_every,
        "particles_per_s_with_sort_every_step": r32["particles_per_s_with_sort_every_step"],
        "gmres": {"iters_last": r32["gmres_iters"], "rel_resid_last": r32["gmres_resid"]},
        "fixed_error": err,
        "fp64": None if r64 is None else {
            "value": r64["particles_per_s"], "ms_per_step": r64["pass_ms"], "hbm_frac": r64["hbm_frac_pass"],
            "breakdown_ms": {k: r64[k] for k in keys}},
        "roofline": {"kernel": kname, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes": nbytes, "launch_ms": kms},
        "cpu_baseline": cpu,
        "mass_apply": apply,
        "adjoint_backward": adjoint,
        "diagnostics": diag,
        "reduced_2d": two_d,
        "double_harris": harris,
        "four_species_2d": four_2d,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
