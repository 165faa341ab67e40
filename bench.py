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
TRAFFIC = {"sources_sha256": "bbfba33374831832c03a9fa9ce5accc0d3e41359baf29d8431a50b28fe18e5bb",
           "plain_call": 4154500000,     # a fused call on the grouping the last regrouping left
           "regroup_call": 5600000000,   # a regrouping call after three plain ones
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
    ap.add_argument("--steps", type=int, default=12)
    ap.add_argument("--warmup", type=int, default=2)
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
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only the adjoint timing (32^3 x 27 ppc x 2 species), printed as one JSON line")
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


def fixed_error(plasma, steps=5, record=None):
    """FP32-form error on the full workload, step by step, beside the FP64 path.

    Both forms start from the same state (the FP32 form is the FP64 state
    encoded as cell + offset) and run `steps` steps of the loop side by side
    (field solve, fused pass with the regrouping every 4 steps). After each
    step the relative max-norm differences of J-hat and M (the next step's
    moments) and of E^{n+1} between the two runs are recorded: the free-running
    divergence of the FP32 form from the FP64 one. With `record` (a list), the
    FP32 run's inputs and outputs of every step are also kept on the host, for
    the comparison with the FP64 oracle that the CPU-baseline leg makes.
    """
    import numpy as np
    import torch
    from paper_2603_16624_amd import ecsim as E
    sims = {P: E.Simulation(plasma, prec=P, tol=1e-10, fused=True, regroup=True) for P in (E.F64, E.F32)}
    rel = lambda a, b: float((a.double() - b.double()).abs().max() / b.double().abs().max())
    cpu = lambda t: t.detach().cpu().numpy()
    per_step = []
    for _ in range(steps):
        s32 = sims[E.F32]
        if record is not None and s32.primed:
            pre = dict(species=[dict(cell=cpu(sp.cell), off=cpu(sp.pos), v=cpu(sp.vel),
                                     q=None if sp.q is None else cpu(sp.q), q_const=sp.q_const, qom=sp.qom)
                                for sp in s32.species],
                       J=cpu(s32.J), M=cpu(s32.M), E=cpu(s32.E), BC=cpu(s32.BC))
        for sim in sims.values():
            if record is not None and sim is s32 and not sim.primed:
                sim.prime()
                pre = dict(species=[dict(cell=cpu(sp.cell), off=cpu(sp.pos), v=cpu(sp.vel),
                                         q=None if sp.q is None else cpu(sp.q), q_const=sp.q_const, qom=sp.qom)
                                    for sp in sim.species],
                           J=cpu(sim.J), M=cpu(sim.M), E=cpu(sim.E), BC=cpu(sim.BC))
            sim.step()
        torch.cuda.synchronize()
        s64 = sims[E.F64]
        per_step.append({"J": rel(s32.J, s64.J), "M": rel(s32.M, s64.M), "E": rel(s32.E, s64.E)})
        if record is not None:
            # the pass's fields as the kernels saw them (FP32 copies) and its results
            # after the step the node-field buffers have swapped: BN_next_p holds
            # the mover's B^n, BN_p the deposit's B^{n+1}
            pre.update(Et=cpu(s32.Et_p), Bmove=cpu(s32.BN_next_p), Bdep=cpu(s32.BN_p),
                       J1=cpu(s32.J), M1=cpu(s32.M), E1=cpu(s32.E))
            record.append(pre)
    del sims
    torch.cuda.empty_cache()
    worst = {k: max(d[k] for d in per_step) for k in ("J", "M", "E")}
    return {**worst, "per_step": per_step, "bound": 1e-5,
            "against": f"FP64 GPU path from the same initial state, free-running, after each of {steps} steps"}


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


def host_cpu():
    """CPU model and core counts of the host (lscpu), and the threads this process may use."""
    import subprocess
    info = {"model": None, "physical_cores": None, "logical_cpus": None}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        kv = {}
        for line in out.splitlines():
            if ":" in line:
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        info["model"] = kv.get("Model name")
        sockets = int(kv.get("Socket(s)", "1") or 1)
        cores = int(kv.get("Core(s) per socket", "0") or 0)
        info["physical_cores"] = sockets * cores if cores else None
        info["logical_cpus"] = int(kv.get("CPU(s)", "0") or 0) or None
    except Exception:
        pass
    affinity = len(os.sched_getaffinity(0))
    omp = os.environ.get("OMP_NUM_THREADS")
    threads = affinity
    if omp and omp.isdigit() and int(omp) > 0:
        threads = min(threads, int(omp))
    if info["physical_cores"]:
        threads = min(threads, info["physical_cores"])
    info["cpus_allowed"] = affinity
    info["threads"] = max(1, threads)
    return info


def _m27_from_m14(O, n, M14):
    """The 27 blocks of every node from the 14 stored ones (M_{g,g-o} = block k of node g - o)."""
    import numpy as np
    nx, ny, nz = n
    off = O.canonical14()
    M27 = np.zeros((27, 9, nx * ny * nz))
    for k in range(14):
        ox, oy, oz = (int(a) for a in off[k])
        M27[(ox + 1) + 3 * (oy + 1) + 9 * (oz + 1)] = M14[k]
        if k:
            src = M14[k].reshape(9, nz, ny, nx)
            M27[(-ox + 1) + 3 * (-oy + 1) + 9 * (-oz + 1)] = np.roll(src, (oz, oy, ox), axis=(1, 2, 3)).reshape(9, -1)
    return M27


def oracle_error(O, plasma, rec, threads, nnodes=8):
    """The FP32 form against the FP64 oracle, step by step, from the FP32 run's own state.

    For every recorded step: J-hat and the 14 mass-matrix blocks after the
    fused pass at sampled nodes, against the oracle's mover (with the pass's
    E^{n+theta} and B^n) and moments (with B^{n+1}) of every particle that
    starts within two cells of those nodes, fed the FP32 state widened exactly
    to FP64; and E^{n+1} over the whole grid, against the oracle's GMRES field
    solve (tolerance 1e-10) and field advance from the same moments and fields.
    """
    import numpy as np
    from paper_2603_16624_amd import inputs as I
    p = plasma
    nx, ny, nz = p.n
    rel = lambda a, b: float(np.max(np.abs(a - b)) / np.max(np.abs(b)))
    rng = np.random.default_rng(4711)
    out = []
    t0 = time.perf_counter()
    for r in rec:
        nodes = rng.choice(p.nn, size=nnodes, replace=False)
        near = np.zeros(p.nn, dtype=bool)
        for gnode in nodes:
            gx, gy, gz = gnode % nx, (gnode // nx) % ny, gnode // (nx * ny)
            for dz in range(-3, 3):
                for dy in range(-3, 3):
                    for dx in range(-3, 3):
                        near[(gx + dx) % nx + nx * (((gy + dy) % ny) + ny * ((gz + dz) % nz))] = True
        Et, Bm, Bd = (np.asarray(r[k], dtype=np.float64) for k in ("Et", "Bmove", "Bdep"))
        Jo = np.zeros((3, p.nn))
        M27 = np.zeros((27, 9, p.nn))
        for s in r["species"]:
            idx = np.nonzero(near[s["cell"]])[0]
            x = I.decode_f32(s["cell"][idx], s["off"][:, idx], p.n, p.h)
            v = s["v"][:, idx].astype(np.float64)
            q = s["q"][idx].astype(np.float64) if s["q"] is not None else float(np.float32(s["q_const"]))
            _, _, Jo, M27, _ = O.move_moments_threads(p.n, p.h, p.dt, x, v, q, s["qom"], Et, Bm, Bd, Jo, M27,
                                                       threads)
        Mo = O.m14(p.n, M27)
        del M27
        eJ = rel(r["J1"][:, nodes].astype(np.float64), Jo[:, nodes])
        eM = rel(r["M1"][:, :, nodes].astype(np.float64), Mo[:, :, nodes])
        del Mo
        M27 = _m27_from_m14(O, p.n, r["M"].astype(np.float64))
        sol = O.field_solve(p.n, p.h, p.dt, M27, r["J"].astype(np.float64), r["E"], r["BC"], 1e-10)
        del M27
        eE = rel(r["E1"], sol["E_next"])
        out.append({"J": eJ, "M": eM, "E": eE, "oracle_gmres_iters": sol["iters"]})
    worst = {k: max(d[k] for d in out) for k in ("J", "M", "E")} if out else {}
    return {**worst, "per_step": out, "bound": 1e-5, "nodes_per_step": nnodes, "wall_s": time.perf_counter() - t0,
            "against": "FP64 oracle, one step from the FP32 run's own state (J, M at sampled nodes; "
                       "E^{n+1} over the grid from the same moments)"}


def cpu_baseline(plasma, sample, rec=None):
    """The CPU leg: the FP64 oracle timed on the host, and (with `rec`) the FP32
    form's per-step error against it.

    Timings (std clock around the oracle calls): the oracle's particle pass --
    mover, then the moments at the moved positions -- on all the threads this
    process may use (thread-private grids added in a fixed order) over
    1/`sample` of each species of the 64^3 workload, and on one thread over
    1/(16 `sample`); and the whole scheme on the 8^3 workload (moments, GMRES
    field solve, mover; 10 steps), on all threads and on one.
    """
    import numpy as np
    from oracle import oracle as O
    from paper_2603_16624_amd import inputs as I
    cpu = host_cpu()
    nt = cpu["threads"]
    rng = np.random.default_rng(12345)
    BN = O.centres_to_nodes(plasma.n, plasma.B_C)
    En = 1e-4 * rng.standard_normal((3, plasma.nn))

    def pass_rate(frac, threads):
        J = np.zeros((3, plasma.nn))
        M27 = np.zeros((27, 9, plasma.nn))
        count, dt = 0, 0.0
        for s in plasma.species:
            k = max(1, s.np // frac)
            x = np.ascontiguousarray(s.x[:, :k])
            v = np.ascontiguousarray(s.v[:, :k])
            q = s.q[:k] if np.ndim(s.q) else s.q
            t0 = time.perf_counter()
            _, _, J, M27, used = O.move_moments_threads(plasma.n, plasma.h, plasma.dt, x, v, q, s.qom, En, BN, BN,
                                                         J, M27, threads)
            dt += time.perf_counter() - t0
            count += k
        return count, dt, used

    c_all, t_all, used = pass_rate(sample, nt)
    c_one, t_one, _ = pass_rate(16 * sample, 1)
    p0 = I.config0()
    steps0 = 10
    t0 = time.perf_counter()
    O.run_steps_threads(p0, steps0, threads=nt)
    t0_all = time.perf_counter() - t0
    t0 = time.perf_counter()
    O.run_steps_threads(p0, steps0, threads=1)
    t0_one = time.perf_counter() - t0
    base = dict(value=c_all / t_all, unit="particles/s", cores=used, kind="oracle",
                sample=f"FP64 oracle particle pass (mover, then moments at the moved positions) on {c_all} "
                       f"particles (1/{sample} of each species) of the 64^3 x 64 ppc x 2 species workload, "
                       f"{used} threads, {t_all:.1f} s",
                cpu_model=cpu["model"], physical_cores=cpu["physical_cores"], cpus_allowed=cpu["cpus_allowed"],
                one_core={"value": c_one / t_one, "unit": "particles/s", "cores": 1,
                          "sample": f"{c_one} particles (1/{16 * sample} of each species), {t_one:.1f} s"},
                small_workload_10_steps={
                    "workload": "8^3 cells x 27 ppc x 2 species (27,648 particles), 10 steps of moments, "
                                "GMRES field solve (tol 1e-10) and mover",
                    "all_cores": {"cores": used, "s": t0_all, "particles_steps_per_s": p0.n_particles * steps0 / t0_all},
                    "one_core": {"cores": 1, "s": t0_one, "particles_steps_per_s": p0.n_particles * steps0 / t0_one}})
    err = oracle_error(O, plasma, rec, nt) if rec else None
    return base, err


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


def adjoint_bytes(p, prec):
    """Algorithmic bytes of one backward through the mover over all species: the particle state read
    (position, velocity; FP32 also the cell) and its gradients written, the node fields E, B, gJ and
    the 14 stored blocks of gM read, and gE, gB read and written (accumulated)."""
    esz = 8 if prec == "f64" else 4
    per_particle = 6 * esz + (4 if prec == "f32" else 0) + 6 * esz
    per_node = (3 + 3 + 3 + 126) * esz + 2 * 6 * esz
    return p.n_particles * per_particle + p.nn * per_node


def adjoint_time():
    """Adjoint of mover -> moments (ecsim_moments_backward through the mover) on the
    32^3 x 27 ppc x 2 species workload (1,769,472 particles), FP64 and FP32: time
    of one backward over both species, with the particles grouped by cell (the
    brick-tiled kernel) and in any order (one thread per particle)."""
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
        grouped = []
        for s in sp:
            d = s.empty_like()
            E.sort(grid, s, d, torch.empty(grid.nn + 1, dtype=torch.int32, device="cuda"))
            grouped.append(d)
        ws = [torch.empty(E.backward_workspace_size(grid, s.np, s.prec), dtype=torch.uint8, device="cuda") for s in sp]

        def bwd(species, wss):
            def run():
                for s, a, b, w in zip(species, gx, gv, wss):
                    E.moments_backward(grid, s, Ed, Bd, gJd, gMd, a, b, gE, gB, through_mover=True, ws=w)
            return run
        ms = _time_events(bwd(grouped, ws), 5)
        ms_any = _time_events(bwd(sp, [None] * len(sp)), 5)
        nbytes = adjoint_bytes(p, prec)
        out[prec] = {"ms": ms, "particles_per_s": p.n_particles / (ms * 1e-3), "algorithmic_bytes": nbytes,
                     "GB_per_s": nbytes / (ms * 1e-3) / 1e9, "hbm_frac": nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "any_order": {"ms": ms_any, "particles_per_s": p.n_particles / (ms_any * 1e-3)}}
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
    if args.adjoint_only:
        print(json.dumps({"adjoint": adjoint_time()}), flush=True)
        return
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
    err = None
    rec = None
    if not args.no_error:
        rec = [] if not args.no_cpu_baseline else None
        err = fixed_error(plasma, record=rec)
        print(f"[bench] fixed error (FP32 vs FP64 path): {json.dumps(err)}", file=sys.stderr, flush=True)
    cpu = None
    if not args.no_cpu_baseline:
        cpu, oerr = cpu_baseline(plasma, args.cpu_sample, rec)
        rec = None
        print(f"[bench] cpu: {json.dumps(cpu)}", file=sys.stderr, flush=True)
        if oerr is not None:
            print(f"[bench] fixed error (FP32 vs oracle): {json.dumps(oerr)}", file=sys.stderr, flush=True)
            err = {**oerr, "fp64_path_divergence": err}
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
