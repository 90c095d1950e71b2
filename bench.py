#!/usr/bin/env python3
"""Throughput of the coupled phase-field step on one MI355X.

One "step" is one call-level pass of the whole hot path: the mechanical
equilibrium solve (PCG to the workload's tolerance, preconditioned by a
multigrid V-cycle unless --precond jacobi), the J2 return
map, the elastic / chemical driving forces, the fluxes and reaction, the
explicit update of the five fields and the FP64 ledger.  The default workload
is the 256^3 porous recipe (64 Voronoi grains, 20 % ellipsoidal pores lined
with a 2-cell iron rim, plasticity on, Omega_f 0.2, FP32 arithmetic with FP64
reductions, CG to 1e-6) with the learned warm start: the network is trained
beforehand, untimed, on the plain method's trajectory of the 128^3 core-shell
recipe only, then frozen.

Prints ONE JSON line.  Besides the throughput it reports the dominant
kernel's roofline figures (average launch duration measured with HIP events),
every stencil kernel's fraction of HBM peak, the same steps from the same
state on the plain mixed path and on the plain FP64 GPU path, the field and
increment error of the timed configuration against the FP64 CPU oracle on a
reduced instance of the same recipe, and the oracle's own throughput on a
bounded sample (``cpu_baseline``).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0     # MI355X HBM3E, vendor figure


def algorithmic_bytes_per_cell(kind, dim, es, precond="jacobi"):
    """Bytes a kernel must move per cell (reads + writes of the arrays the
    method needs), by kernel class; es = element size of the state."""
    nc = 4 if dim == 2 else 6
    if kind == "apply":        # read z, p_old (dim each), K, G; write p_new, q (dim each)
        return (4 * dim + 2) * es
    if kind == "update":
        if dim == 3 and precond == "mg":   # read r, q, write r; after odd iterations also read u, p, p_prev, write u
            return 5 * dim * es
        if precond == "mg":    # 2D: read u, p, r, q; write u, r
            return 6 * dim * es
        if dim == 3:           # read r, q, D^-1, write r, z; after odd iterations also read u, p, p_prev, write u
            return 7 * dim * es
        return 8 * dim * es    # read u, p, r, q, D^-1; write u, r, z (dim each)
    if kind == "step":         # read 5 fields, mu, u, eps_p, eps_P; write 5 fields, eps_p, eps_P
        nf = 10 if es == 4 else 5  # FP32 state: each field is an FP32 pair (hi, lo)
        return (nf + 1 + dim + nc + 1 + nf + nc + 1) * es
    if kind == "mu":           # read phi_f, phi_w, x_O; write mu
        return 4 * es
    if kind == "smooth":
        # multigrid sweeps on the solve's grid, four per cycle: the two-sweep pass from zero (read b, D^-1, K,
        # G; write x), the residual sweep (read x, b, K, G; write r) and two post-smoothing sweeps (read x, b,
        # D^-1, K, G; write x); the 3D FP32 sweeps read D^-1, K and G as bf16 copies (2 bytes each)
        lo = 2 if (dim == 3 and es == 4) else es
        return ((2 * dim * es + (dim + 2) * lo) + (3 * dim * es + 2 * lo) + 2 * (3 * dim * es + (dim + 2) * lo)) / 4.0
    if kind == "solve_setup":
        if dim == 3:           # average of the set-up pass (phi_f, phi_w, eps_p -> K, G, b, D^-1), the residual
            # pass (u, K, G, b, D^-1 -> r, z) and the true residual (u, K, G, b -> q)
            return ((2 + nc + 2 + 2 * dim) + (dim + 2 + 2 * dim + 2 * dim) + (dim + 2 + dim + dim)) * es / 3.0
        # 2D: average of ||b|| (K, G, phi_f, eps_p), residual (+u, r, z, D^-1), true residual
        return ((2 + 1 + nc) + (dim + 2 + 1 + nc + 3 * dim) + (dim + 2 + 1 + nc)) * es / 3.0
    return 0.0


NN_FLOP_PER_VOXEL = 2 * 27 * (6 * 32 + 32 * 32 + 32 * 32 + 32 * 3)   # one inference, algorithmic
BF16_PEAK_TFLOPS = 2500.0  # MI355X dense bf16 matrix peak, vendor figure


KERNEL_NAMES = {("update", 3, 4): "k_cg_update<float, 3>", ("apply", 3, 4): "k_apply3<float, 8, 0>",
                ("step", 3, 4): "k_step3<float>", ("mu", 3, 4): "k_mu<float, 3>",
                ("update", 3, 8): "k_cg_update<double, 3>", ("apply", 3, 8): "k_apply3<double, 8, 0>",
                ("update", 2, 4): "k_cg_update<float, 2>", ("apply", 2, 4): "k_apply2<float>",
                ("step", 2, 4): "k_step<float, 2>", ("mu", 2, 4): "k_mu<float, 2>",
                ("smooth", 3, 4): ("k_apply3<float, 8, 4> @fine", "k_apply3<float, 8, 3> @fine"),
                ("smooth", 2, 4): ("k_apply2s<float, 4> @fine", "k_apply2s<float, 3> @fine")}
# launches per cycle of each kernel of a kind made of several (weights of their traffic)
KERNEL_WEIGHTS = {"smooth": (1, 3)}


def source_sha():
    """sha256[:16] over the kernel sources, as recorded in profiles/*_traffic.json."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2111_11538_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profiled_traffic(tag, kind, dim, es, name=None):
    """HBM bytes per launch of a kernel from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE summary, or None if it is missing or the kernels changed since."""
    path = os.path.join(ROOT, "profiles", f"{tag}_traffic.json")
    name = name or KERNEL_NAMES.get((kind, dim, es))
    if not name or not os.path.exists(path):
        return None, None
    with open(path) as fh:
        d = json.load(fh)
    names = name if isinstance(name, tuple) else (name,)
    weights = KERNEL_WEIGHTS.get(kind, (1,)) if isinstance(name, tuple) else (1,)
    if d.get("kernel_source_sha") != source_sha() or any(n not in d.get("kernels", {}) for n in names):
        return None, None
    tot = sum(w * (d["kernels"][n]["fetch_bytes"] + d["kernels"][n]["write_bytes"]) for n, w in zip(names, weights))
    return tot / sum(weights), os.path.relpath(path, ROOT)


def pf_kinds():
    from paper_2111_11538_amd import pf
    return pf.KERNEL_KINDS


def run_gpu(wl, precision, steps, warmup, timing, rtol, fields=None, net=None, every=1, precond="jacobi"):
    """timing: None (no events), or the kernel kinds to bracket with events
    (the CG kernels on every `every`-th iteration of each solve)."""
    import torch
    from paper_2111_11538_amd import pf
    ctx = pf.Context(wl.dim, wl.shape, wl.h, wl.dt, wl.params, device=0, precision=precision,
                     plasticity=wl.plasticity, cg_rtol=rtol, warm="learned" if net is not None else "prev",
                     cg_precond=precond)
    ctx.set_fields(fields if fields is not None else wl.fields)
    if net is not None:
        net.attach(ctx)
    tag = precision + (" learned" if net is not None else "")
    print(f"[bench] {tag}: warmup {warmup} steps", file=sys.stderr, flush=True)
    st0 = ctx.step(warmup) if warmup > 0 else ctx.step(0)
    it0 = st0["cg_iters_total"]
    if timing:
        ctx.timing(True, kinds=timing, every=every)
    torch.cuda.synchronize()
    print(f"[bench] {tag}: timing {steps} steps", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    st = ctx.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rep = ctx.timing_report() if timing else None
    if timing:
        ctx.timing(False)
    ctx.close()
    return {"seconds": t1 - t0, "stats": st, "cg_iters": st["cg_iters_total"] - it0, "kernels": rep}


INCR_TOL = {"phi_f": 1e-3, "phi_w": 1e-3, "xO": 1e-4, "xH": 1e-4, "xW": 1e-3}
FIELD_TOL = 1e-4


def accuracy_sample(name, n, steps=10, params=None, settle=0, precond="jacobi"):
    """The timed configuration (mixed GPU path, CG 1e-6, with the learned start
    when trained parameters are given) against the FP64 oracle solved to 1e-10
    on an n^3 (or n^2) instance of the same recipe: per-field relative error
    and the error of the increment over the run (absolute RMS where the
    increment's RMS is below 1e-12, i.e. rounding noise)."""
    import numpy as np
    from paper_2111_11538_amd import inputs as I
    from paper_2111_11538_amd import pf
    from oracle import oracle as O
    wl = I.workload(name, n=n)
    learned = params is not None and wl.dim == 3
    g = pf.Context(wl.dim, wl.shape, wl.h, wl.dt, wl.params, precision=wl.precision, plasticity=wl.plasticity,
                   cg_rtol=wl.cg_rtol, warm="learned" if learned else "prev", cg_precond=precond)
    g.set_fields(wl.fields)
    net = None
    if learned:
        net = pf.Net(max_voxels=int(np.prod(wl.shape)))
        net.set_params(params)
        net.attach(g)
    o = O.OracleSim(wl.dim, wl.shape, wl.h, wl.dt, wl.params, wl.fields, plasticity=wl.plasticity, cg_rtol=1e-10)
    iters, used = [], []
    for _ in range(steps):
        st = g.step()
        o.step()
        iters.append(st["cg_iters"])
        used.append(st["warm_used"])
    out = g.fields()
    g.close()
    if net is not None:
        net.close()
    fe, ie, ok = {}, {}, True
    for k in ("phi_f", "phi_w", "xO", "xH", "xW"):
        b, a, b0 = o.f[k], out[k], wl.fields[k]
        rms = float(np.sqrt(np.mean(b * b)))
        fe[k] = float(np.linalg.norm(a - b) / np.linalg.norm(b)) if rms >= 1e-6 else float(np.sqrt(np.mean((a - b) ** 2)))
        db, da = b - b0, a - b0
        if float(np.sqrt(np.mean(db * db))) < 1e-12:
            ie[k] = {"abs_rms": float(np.sqrt(np.mean((da - db) ** 2)))}
            ok &= ie[k]["abs_rms"] < 1e-15
        else:
            ie[k] = float(np.linalg.norm(da - db) / np.linalg.norm(db))
            ok &= ie[k] < INCR_TOL[k]
        ok &= fe[k] < FIELD_TOL
    ue = float(np.linalg.norm(out["ux"] - o.ux) / np.linalg.norm(o.ux))
    return {"sample": f"{name} {n}^{wl.dim} (reduced instance of the timed recipe), {steps} steps, mixed GPU, "
                      f"{'MG-' if precond == 'mg' else 'Jacobi-'}PCG 1e-6"
                      f"{', learned start' if learned else ''} vs FP64 oracle, Jacobi-PCG 1e-10",
            "max_field_rel_err": max(v for v in fe.values()), "field_err": fe, "incr_rel_err": ie, "u_rel_err": ue,
            "gates": {"field": FIELD_TOL, "increment": INCR_TOL}, "within_gates": bool(ok),
            "cg_iters": iters, "learned_used_steps": int(sum(1 for u in used if u == 2))}


def cpu_baseline(name, n, budget_s=15.0, max_steps=12):
    """The FP64 oracle on a bounded sample: an n^3 (or n^2) instance of the
    timed recipe, one untimed cold-start step, then warm-started steps until
    about `budget_s` seconds have passed."""
    from paper_2111_11538_amd import inputs as I
    from oracle import oracle as O
    wl = I.workload(name, n=n)
    o = O.OracleSim(wl.dim, wl.shape, wl.h, wl.dt, wl.params, wl.fields, plasticity=wl.plasticity, cg_rtol=wl.cg_rtol)
    o.step()
    t0 = time.perf_counter()
    steps, iters = 0, 0
    while steps < max_steps and (time.perf_counter() - t0 < budget_s or steps < 2):
        st = o.step()
        steps += 1
        iters += st["cg_iters"]
    dt = time.perf_counter() - t0
    ncell = 1
    for d in wl.shape:
        ncell *= d
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    return {"value": ncell * steps / dt, "unit": "voxel-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"FP64 C oracle (OpenMP over cell loops; CG dot products serial), {name} "
                      f"{'x'.join(str(x) for x in reversed(wl.shape))} (reduced instance of the timed recipe), "
                      f"steps 2-{steps + 1} (warm-started, {iters / steps:.0f} CG iterations/step at rtol "
                      f"{wl.cg_rtol:g}), {dt:.1f} s",
            "cg_iters_per_step": iters / steps}


BATCH_TRANSIENT_STEPS = 24


def run_batch(args):
    """The 64-instance batch (2D core-shell template, sides U{64..512}),
    autotuned, one persistent graph launch per step."""
    import torch
    from paper_2111_11538_amd import inputs as I
    from paper_2111_11538_amd import pf, autotune
    inst = I.batch_instances()
    shapes = [s for s, _ in inst]
    p = I.Params()
    h = I.H_DEFAULT
    dt = I.stable_dt(p, h, 2)
    prec = "mixed"
    b = pf.Batch(shapes, h, dt, p, precision=prec, plasticity=True, cg_rtol=1e-6)
    for k, (_, f) in enumerate(inst):
        b.set_fields(k, f)
    cells = sum(ny * nx for ny, nx in shapes)
    print(f"[bench] batch of {len(shapes)}, {cells} cells: warmup {args.warmup}", file=sys.stderr, flush=True)
    # the first steps of the recipe are a start-up transient (their solves
    # take about twice the CG iterations of later ones): like the 3D learned
    # runs, which follow 24 recorded solves, the timed steps follow 24 steps
    b.step(args.warmup + BATCH_TRANSIENT_STEPS)
    # the whole state after the warm-up (fields, displacements, plastic
    # strains), restored after tuning: the timed steps then do the same work
    # whatever number of trial steps the tuner took
    saved = [b.fields(k) for k in range(len(shapes))]
    tuned = autotune.tune(b, prec, cache_path=None, log=lambda m: print(m, file=sys.stderr, flush=True))
    for k, f in enumerate(saved):
        b.set_fields(k, f)
    del saved
    b.step(1)
    trace_marker(args.copy_probe)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = b.step(args.steps)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    trace_marker(args.copy_probe)
    iters = [s["cg_iters"] for s in st]
    es = 4
    bytes_step = sum((s["cg_iters"] * (algorithmic_bytes_per_cell("apply", 2, es) + algorithmic_bytes_per_cell("update", 2, es))
                      + algorithmic_bytes_per_cell("step", 2, es) + algorithmic_bytes_per_cell("mu", 2, es)) * ny * nx
                     for s, (ny, nx) in zip(st, shapes))
    achieved = bytes_step / (sec / args.steps) / 1e9
    traffic, traffic_src = profiled_traffic(f"batch_{len(shapes)}_core_shell_2d", None, 2, es, name="k_batch_step<float>")
    b.close()
    line = {
        "metric": "voxel-steps/s at <=1e-4 rel err vs FP64 oracle; % of HBM peak; CG iters/step",
        "value": cells * args.steps / sec, "unit": "voxel-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * sec / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 arithmetic, f32-pair state, f64 reductions", "data": "synthetic",
        "config": {"workload": f"batch of {len(shapes)} 2D core-shell instances, sides U{{64..512}}, plasticity on, "
                               f"CG rtol 1e-06, one persistent graph launch per step, timed after "
                               f"{BATCH_TRANSIENT_STEPS + args.warmup + 1} untimed steps", "cells": cells},
        "cg_iters_per_step": {"mean": sum(iters) / len(iters), "max": max(iters)},
        "roofline": {"bound": "hbm", "kernel": "k_batch_step (whole step, algorithmic bytes of apply+update per "
                     "iteration per instance + step)", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "traffic_source": traffic_src, "timed_with": "wall clock of the timed steps (one launch per step)"},
        "tiles": {k: v for k, v in tuned.items() if k != "trials"},
    }
    print(json.dumps(line), flush=True)


def run_trends(args):
    """The core-shell study of Sec. 4.2 over minutes of model time: a 2D
    wuestite core (radius 24 cells, 1.9 um) in a 4-cell ferrite shell inside a
    5 um gas box, advanced with the implicit species update and the reaction
    solved exactly per cell (dt = 10 ms), for Omega_f in 0 ... 0.4 (elastic)
    and 0.1, 0.4 (elasto-plastic), with the small-strain mechanics of the step
    or (--kinematics finite) the finite-strain solver attached; records the
    reduction degree (Eq. 39), the largest von Mises stress and plastic strain
    over time."""
    import torch
    from paper_2111_11538_amd import inputs as I
    from paper_2111_11538_amd import pf
    n, dt = 64, 1e-2
    T = args.trend_seconds
    every = max(1, int(round(T / dt / 24)))
    steps = every * 24
    f0 = I.ic_core_shell((n, n), r_core=24.0, r_shell=28.0, noise_seed=I.SEED_BASE + 6)
    cases = [(om, False) for om in (0.0, 0.1, 0.2, 0.25, 0.3, 0.4)] + [(0.1, True), (0.4, True)]
    if args.trend_cases:                 # e.g. "0.1e,0.4p": Omega_f and e(lastic) / p(lastic)
        cases = [(float(c[:-1]), c[-1] == "p") for c in args.trend_cases.split(",")]
    out = {}
    t0 = time.perf_counter()
    finite = args.kinematics == "finite"
    for om, plastic in cases:
        p = I.Params(Omega_f=om)
        c = pf.Context(2, (n, n), I.H_DEFAULT, dt, p, precision="fp64", plasticity=plastic, cg_rtol=1e-8,
                       species_implicit=2, species_rtol=1e-10, mechanics=not finite)
        fs = None
        if finite:
            fs = pf.FiniteStrain(2, (n, n), I.H_DEFAULT, p, plasticity=plastic, newton_rtol=1e-8, cg_rtol=1e-3)
            c.attach_fs(fs)
        c.set_fields(f0)
        rec = {"t_s": [], "red_degree": [], "max_vm_GPa": [], "max_epsP": [], "mean_phi_f": []}
        vm_max = 0.0
        for k in range(steps // every):
            st = c.step(every)
            vm_max = max(vm_max, st["max_vm"])
            rec["t_s"].append(round((k + 1) * every * dt, 3))
            rec["red_degree"].append(round(st["red_degree"], 5))
            rec["max_vm_GPa"].append(round(st["max_vm"] / 1e9, 4))
            rec["max_epsP"].append(round(st["max_epsP"], 5))
            rec["mean_phi_f"].append(round(float(c.get("phi_f").mean()), 5))
            print(f"[trends]   Omega_f={om:g} {'p' if plastic else 'e'} t={rec['t_s'][-1]:g} s f={rec['red_degree'][-1]:.4f} "
                  f"vm={rec['max_vm_GPa'][-1]:.3f} GPa cg/step(last)={st['cg_iters']} ({time.perf_counter() - t0:.0f} s)",
                  file=sys.stderr, flush=True)
        rec["peak_vm_GPa_sampled"] = round(vm_max / 1e9, 4)
        rec["O_drift"] = st["O_drift"]
        c.close()
        if fs is not None:
            fs.close()
        key = f"Omega_f={om:g} {'elasto-plastic' if plastic else 'elastic'}"
        out[key] = rec
        print(f"[trends] {key}: reduction degree {rec['red_degree'][-1]:.4f} at {T:g} s, largest sampled "
              f"sigma_vm {rec['peak_vm_GPa_sampled']:.3f} GPa ({time.perf_counter() - t0:.0f} s)", file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    line = {"metric": "core-shell trends (Sec. 4.2): reduction degree and largest von Mises stress over time",
            "workload": f"2D core-shell {n}x{n}, h {I.H_DEFAULT:g} m, core r 24, shell to r 28, gas box; "
                        f"dt {dt:g} s, {steps} steps, species implicit with the reaction solved exactly; "
                        f"{'finite-strain' if finite else 'small-strain'} mechanics",
            "cases": out}
    print(json.dumps(line), flush=True)


FP64_VECTOR_PEAK_TFLOPS = 78.6   # MI355X FP64 vector (non-matrix) peak, vendor figure
# FP64 operations per cell of the 3D tangent kernel (dual numbers, 8 Gauss
# points, F_P = I): SQ_INSTS_VALU_FLOPS_FP64 x 64 lanes per launch at 128^3,
# divided by the cells (24.48 GFLOP / 2097152)
FS_TANGENT_FLOP_PER_CELL = 11672
FS_KERNEL_BYTES_PER_CELL = {
    # tangent J v and residual R(u), per cell: nodal u (and v) 8 B per component
    # per node (one node per cell), phi_f, phi_w, the element forces written
    # (2^d d doubles) and F_P read (2^d 9 doubles) unless it is the identity
    "tangent": lambda d, fpi: 8 * (2 * d + 2 + (1 << d) * d + (0 if fpi else (1 << d) * 9)),
    "residual": lambda d, fpi: 8 * (d + 2 + (1 << d) * d + (0 if fpi else (1 << d) * 9)),
    # gather: element forces read, nodal vector written, the dot partner read
    "gather": lambda d, fpi: 8 * ((1 << d) * d + 2 * d),
}


def run_finite_strain(args):
    """Finite-strain mechanics (Sec. 2.2): one solve (Newton from u = 0, then
    the return map and the driving forces) of the 128^3 core-shell recipe at
    Omega_f 0.4, elasto-plastic, with HIP events on every launch; the largest
    von Mises stress of the 2D core-shell of the trend study (core r 24, shell
    to 28) under small and finite strain for Omega_f 0.1 ... 0.4; and the FE
    oracle timed on a 12^3 instance of the same recipe."""
    import numpy as np
    import torch
    from paper_2111_11538_amd import inputs as I
    from paper_2111_11538_amd import pf
    n = args.n or 128
    wl = I.workload("core_shell_3d", n=n)
    p = wl.params
    shape = wl.shape
    cells = int(np.prod(shape))
    # warm-up on a small instance (first launches, event pool)
    wz = I.workload("core_shell_3d", n=16)
    fz = pf.FiniteStrain(3, wz.shape, wz.h, p, plasticity=True, newton_rtol=1e-8)
    fz.set("phi_f", wz.fields["phi_f"])
    fz.set("phi_w", wz.fields["phi_w"])
    fz.timing(True)
    fz.solve()
    fz.close()
    fs = pf.FiniteStrain(3, shape, wl.h, p, plasticity=True, newton_rtol=1e-8, cg_rtol=1e-3)
    fs.set("phi_f", wl.fields["phi_f"])
    fs.set("phi_w", wl.fields["phi_w"])
    fs.timing(True)
    trace_marker(args.copy_probe)
    torch.cuda.synchronize()
    print(f"[bench] finite strain {shape}: solve", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    st = fs.solve()
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    trace_marker(args.copy_probe)
    rep = fs.timing_report()
    fs.close()
    kernels = {}
    for k, (ms, cnt) in rep.items():
        kernels[k] = {"total_ms": round(ms, 3), "launches": cnt, "avg_us": round(1e3 * ms / cnt, 2) if cnt else None}
    # the tangent kernel ran cg_iters times with work (launches queued past a
    # CG solve's convergence exit at entry): its time per real launch
    tan_ms = rep["tangent"][0]
    tan_us = 1e3 * tan_ms / max(st["cg_iters"], 1)
    bpc = FS_KERNEL_BYTES_PER_CELL["tangent"](3, True)
    gbs = bpc * cells / (tan_us * 1e-6) / 1e9
    tflops = FS_TANGENT_FLOP_PER_CELL * cells / (tan_us * 1e-6) / 1e12
    dom = max(rep, key=lambda k: rep[k][0])
    fs_traffic, fs_traffic_src = profiled_traffic(f"finite_strain_3d_{n}", None, 3, 8, name="k_fs_elem<3, true>")
    # small vs finite strain, 2D core-shell of the trend study
    sweep = {}
    f0 = I.ic_core_shell((64, 64), r_core=24.0, r_shell=28.0, noise_seed=I.SEED_BASE + 6)
    for om in (0.1, 0.2, 0.3, 0.4):
        for plastic in (False, True):
            if plastic and om not in (0.1, 0.4):
                continue
            q = I.Params(Omega_f=om)
            c = pf.Context(2, (64, 64), I.H_DEFAULT, 1e-12, q, precision="fp64", plasticity=plastic, cg_rtol=1e-10)
            c.set_fields(f0)
            small = c.step(1)["max_vm"]
            c.close()
            g2 = pf.FiniteStrain(2, (64, 64), I.H_DEFAULT, q, plasticity=plastic, newton_rtol=1e-10)
            g2.set("phi_f", f0["phi_f"])
            g2.set("phi_w", f0["phi_w"])
            fin = g2.solve()["max_vm"]
            g2.close()
            sweep[f"Omega_f={om:g} {'elasto-plastic' if plastic else 'elastic'}"] = {
                "small_strain_GPa": round(small / 1e9, 3), "finite_strain_GPa": round(fin / 1e9, 3)}
    line = {
        "metric": "finite-strain mechanics: voxel-solves/s (Newton to 1e-8 of ||R(0)||, then the return map)",
        "value": cells / sec, "unit": "voxel-solves/s", "n_gpus": 1, "higher_is_better": True, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"core_shell_3d {n}x{n}x{n} (sphere r {48 * n // 128}, ferrite shell to {52 * n // 128}), "
                               "Omega_f 0.4, elasto-plastic, from u = 0 and F_P = I; trilinear cells, 8 Gauss points",
                   "cells": cells},
        "solve_s": sec, "newton_iters": st["newton_iters"], "cg_iters": st["cg_iters"],
        "line_search_cuts": st["line_search_cuts"], "rel_resid": st["rel_resid"], "yielded_gauss_points": st["yielded"],
        "max_vm_GPa": st["max_vm"] / 1e9, "max_epsP": st["max_epsP"],
        "roofline": {"bound": "alu", "kernel": "tangent (k_fs_elem on dual numbers, one per CG iteration)",
                     "achieved": round(tflops, 2), "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(tflops / FP64_VECTOR_PEAK_TFLOPS, 4), "traffic": fs_traffic,
                     "traffic_source": fs_traffic_src,
                     "flop_per_launch": FS_TANGENT_FLOP_PER_CELL * cells, "avg_launch_us": round(tan_us, 2),
                     "hbm_GBps_algorithmic": round(gbs, 1), "hbm_frac_of_8TBps": round(gbs / HBM_PEAK_GBS, 4),
                     "note": ("FP64 operations of the dual-number stress evaluation per cell (8 Gauss points), "
                              "counted once with rocprofv3 SQ_INSTS_VALU_FLOPS_FP64 (x 64 lanes); time per CG "
                              "iteration that did work (launches queued past convergence excluded)")},
        "dominant_kernel": dom,
        "kernels": kernels,
        "small_vs_finite_strain_max_vm": {"workload": "2D core-shell 64x64 (core r 24, shell to 28), first solve",
                                          "cases": sweep},
    }
    if not args.no_cpu_baseline:
        from oracle import fs_fe_oracle as FE
        m = 12
        wc = I.workload("core_shell_3d", n=m)
        g = FE.FEGrid(3, wc.shape, wc.h, p, wc.fields["phi_f"], wc.fields["phi_w"])
        Fp, eP = FE.identity_plastic(wc.shape, 3)
        t0 = time.perf_counter()
        u, it, rr = g.solve(np.zeros((3,) + g.nodes), Fp, rtol=1e-8)
        g.return_map(u, Fp, eP)
        csec = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": m ** 3 / csec, "unit": "voxel-solves/s", "cores": 1, "kind": "oracle",
                                "sample": f"numpy FE oracle (sparse direct Newton), core_shell_3d {m}^3, "
                                          f"{it} Newton steps, {csec:.1f} s"}
    print(json.dumps(line), flush=True)


def measure_copy_peak(mib=1024, reps=20):
    """Device-to-device copy bandwidth (read + write bytes per second) of a
    plain 1 GiB copy: the practical HBM ceiling on this machine."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3 / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2 * n * 4 / sec / 1e9


def time_train_iters(tn, recs, wl, args, n=20):
    """Device time of one training iteration (forward, loss, backward-data,
    backward-weight, Adam) on one packed batch of crops, averaged over `n`
    iterations between HIP events on the network's stream; priced in the
    algorithmic MFMA flops of the three convolution passes."""
    import torch
    from paper_2111_11538_amd import learned as LR
    LR.train(tn, recs, 1, wl.params.Omega_f, wl.h, crop=(64, 64, 64), batch=args.train_batch, lr=args.train_lr,
             t_min=5)                       # packs one batch of crops into the network's input slots
    cz, cy, cx = (min(64, d) for d in recs[0]["phi_f"].shape)
    vox = args.train_batch * cz * cy * cx
    fwd = NN_FLOP_PER_VOXEL * vox
    bwd_data = 2 * 27 * (32 * 32 + 32 * 32 + 32 * 3) * vox     # input gradients of layers 2-4
    flop = 2 * fwd + bwd_data                                  # forward, backward-weight, backward-data
    total = 0.0
    for _ in range(n):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(tn.stream)
        tn.forward(None, None, args.train_batch, cz, cy, cx)
        tn.loss()
        tn.backward()
        tn.adam(args.train_lr)
        e1.record(tn.stream)
        e1.synchronize()
        total += e0.elapsed_time(e1) / 1e3
    avg = total / n
    tf = flop / avg / 1e12
    return {"bound": "mfma", "kernel": f"one training iteration on {args.train_batch} crops of {cz}x{cy}x{cx} "
            "(4 forward, 3 backward-data and 4 backward-weight convolutions, loss, Adam)",
            "achieved": round(tf, 1), "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(tf / BF16_PEAK_TFLOPS, 4),
            "traffic": None, "flop_per_iter": flop, "avg_iter_us": round(avg * 1e6, 1),
            "timed_with": f"HIP events on the network's stream around {n} iterations after training"}


def train_learned(args):
    """Record the plain method's first solves of the training recipe (the
    128^3 core-shell workload by default), train the network on random 64^3
    crops of them (offline, untimed) and return the trained (then frozen)
    parameters and a summary."""
    import numpy as np
    import torch
    from paper_2111_11538_amd import inputs as I
    from paper_2111_11538_amd import pf, learned as LR
    log = lambda m: print(m, file=sys.stderr, flush=True)
    twl = I.workload(args.train_workload, n=args.train_n)
    c = pf.Context(twl.dim, twl.shape, twl.h, twl.dt, twl.params, precision=twl.precision, plasticity=twl.plasticity,
                   cg_rtol=twl.cg_rtol, warm="prev")
    c.set_fields(twl.fields)
    t0 = time.perf_counter()
    recs = LR.record_trajectory(c, args.train_steps)
    c.close()
    t1 = time.perf_counter()
    ncell = int(np.prod(twl.shape))
    tn = pf.Net(max_voxels=max(args.train_batch * 64 ** 3, ncell), training=True, seed=1)
    LR.init_extrapolation(tn)
    held = recs[-4:]                 # the last 2 recorded solves are held out (2 more give their history)
    v0 = float(np.mean(LR.evaluate(tn, held, twl.params.Omega_f, twl.h)))
    losses = LR.train(tn, recs[:-2], args.train_iters, twl.params.Omega_f, twl.h, crop=(64, 64, 64),
                      batch=args.train_batch, lr=args.train_lr, t_min=5, log=log, log_every=500, val_recs=held,
                      eval_every=25)
    v1 = float(np.mean(LR.evaluate(tn, held, twl.params.Omega_f, twl.h)))
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    params = tn.params()
    train_roof = time_train_iters(tn, recs[:-2], twl, args)   # the training net's weights are not used after this
    tn.close()
    del recs
    torch.cuda.empty_cache()
    info = {"trained_on": f"{twl.name} {'x'.join(str(x) for x in reversed(twl.shape))} (plain method, previous-step "
                          f"start), solves 0-{args.train_steps - 1}; frozen before the timed workload",
            "record_s": round(t1 - t0, 2), "iters": args.train_iters,
            "batch": f"{args.train_batch} crops of 64^3", "train_s": round(t2 - t1, 2),
            "loss_first_last_50": [float(np.mean(losses[:50])), float(np.mean(losses[-50:]))],
            "held_out_full_grid_loss_extrapolation_init": v0, "held_out_full_grid_loss_trained": v1,
            "early_stopping": "best held-out full-grid loss (last 2 recorded solves) over checkpoints every 25 iterations",
            "roofline": train_roof}
    return params, info


def settle(wl, steps, precond="jacobi"):
    """The common starting state of every timed leg: the recipe's initial
    condition advanced `steps` untimed steps by the plain mixed path with the
    previous-step start (past the cold first solves)."""
    from paper_2111_11538_amd import pf
    c = pf.Context(wl.dim, wl.shape, wl.h, wl.dt, wl.params, precision=wl.precision, plasticity=wl.plasticity,
                   cg_rtol=wl.cg_rtol, warm="prev", cg_precond=precond)
    c.set_fields(wl.fields)
    st = c.step(steps) if steps > 0 else c.step(0)
    state = c.fields()
    c.close()
    return state, st


def copy_probe(mib, times):
    """Counter calibration under a profiler: `times` plain device copies of
    `mib` MiB between two trace markers (nothing when mib is 0)."""
    if mib <= 0:
        return
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    trace_marker(mib)
    for _ in range(times):
        dst.copy_(src)
    trace_marker(mib)
    torch.cuda.synchronize()
    del src, dst


def trace_marker(mib):
    """A kernel no other part of the run launches (a flip of four numbers):
    brackets the calibration copies and the timed legs in a profiler's trace
    (nothing when mib is 0)."""
    if mib <= 0:
        return
    import torch
    torch.flip(torch.arange(4, device="cuda"), dims=(0,))
    torch.cuda.synchronize()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="porous_3d")
    ap.add_argument("--n", type=int, default=None, help="grid side override (reduced runs)")
    ap.add_argument("--settle", type=int, default=10,
                    help="untimed steps from the initial condition (previous-step start) before every timed leg")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 GPU run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--acc-n", type=int, default=None, help="side of the accuracy sample (default 48 in 3D, 256 in 2D)")
    ap.add_argument("--cpu-n", type=int, default=None, help="side of the CPU baseline sample (default 64 in 3D, 512 in 2D)")
    ap.add_argument("--precond", default="mg", choices=("mg", "jacobi"),
                    help="preconditioner of the equilibrium CG (the batch workload always uses Jacobi)")
    ap.add_argument("--warm", default="learned", choices=("learned", "prev"),
                    help="CG start of the timed run (learned: network trained first, on the training recipe)")
    ap.add_argument("--train-workload", default="core_shell_3d", help="recipe whose trajectory trains the network")
    ap.add_argument("--train-n", type=int, default=128, help="grid side of the training recipe")
    ap.add_argument("--train-steps", type=int, default=24, help="recorded solves for training")
    ap.add_argument("--train-iters", type=int, default=3000,
                    help="Adam iterations of the network's training (early stopping keeps the best held-out checkpoint)")
    ap.add_argument("--train-lr", type=float, default=1e-4, help="Adam learning rate of the network's training")
    ap.add_argument("--train-batch", type=int, default=4, help="64^3 crops per training minibatch")
    ap.add_argument("--trend-seconds", type=float, default=120.0, help="model time of the core-shell trend runs")
    ap.add_argument("--trend-cases", default="", help="comma list of Omega_f with e (elastic) or p (plastic), e.g. 0.1e,0.4p")
    ap.add_argument("--kinematics", default="small", choices=("small", "finite"),
                    help="mechanics of the trend runs: small strain (in the step) or the finite-strain solver")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="copy this many MiB with a plain device copy first (counter calibration under a profiler) "
                         "and mark the calibration copies and the timed legs with a flip kernel in the trace")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    copy_probe(args.copy_probe, 3)

    if args.workload == "batch":
        run_batch(args)
        return
    if args.workload == "trends":
        run_trends(args)
        return
    if args.workload == "finite_strain":
        run_finite_strain(args)
        return
    copy_peak = measure_copy_peak()

    from paper_2111_11538_amd import inputs as I
    from paper_2111_11538_amd import pf
    wl = I.workload(args.workload, n=args.n)
    ncell = 1
    for d in wl.shape:
        ncell *= d
    es = 4 if wl.precision == "mixed" else 8

    learned = args.warm == "learned" and wl.dim == 3
    params, train_info, net = None, None, None
    if learned:
        print(f"[bench] training on {args.train_workload} at {args.train_n}", file=sys.stderr, flush=True)
        params, train_info = train_learned(args)
    precond = args.precond
    print(f"[bench] settling {wl.name} {wl.shape}: {args.settle} steps", file=sys.stderr, flush=True)
    start, st_settle = settle(wl, args.settle, precond)
    if learned:
        net = pf.Net(max_voxels=ncell)
        net.set_params(params)
    # per-kernel times: a replay of the same steps from the same state with
    # HIP events attached to every dispatch (each timed dispatch then follows
    # a timed one, which keeps the events' own overhead out of the kernel's
    # interval); the throughput run below carries no events
    trace_marker(args.copy_probe)
    brk = run_gpu(wl, wl.precision, args.steps, args.warmup, pf_kinds(), wl.cg_rtol, fields=start, net=net,
                  precond=precond)
    kern = brk["kernels"]
    # the dominant kernel by time ("precond", the coarse half of the multigrid cycle, is a group of short
    # kernels of many shapes, not one kernel: it is reported in the kernel table, not as the roofline)
    dom = max((k for k in ("apply", "update", "step", "mu", "solve_setup", "nn", "smooth")),
              key=lambda k: kern[k][0])
    res = run_gpu(wl, wl.precision, args.steps, args.warmup, None, wl.cg_rtol, fields=start, net=net,
                  precond=precond)
    trace_marker(args.copy_probe)
    ms = 1e3 * res["seconds"] / args.steps
    value = ncell * args.steps / res["seconds"]

    # dominant kernel and its roofline, from the replay's events
    tot_ms, nl = kern[dom]
    avg_s = tot_ms / 1e3 / max(nl, 1)
    bytes_per_launch = algorithmic_bytes_per_cell(dom, wl.dim, es, precond) * ncell
    achieved = bytes_per_launch / avg_s / 1e9
    tag = f"{wl.name}_{wl.shape[0]}_{'learned' if learned else 'prev'}"
    traffic, traffic_src = profiled_traffic(tag, dom, wl.dim, es)
    kernels = {}
    for k, v in kern.items():
        b = algorithmic_bytes_per_cell(k, wl.dim, es, precond) * ncell
        gbs = b / (v[0] / 1e3 / v[1]) / 1e9 if v[1] and b > 0 else None
        kernels[k] = {"total_ms": round(v[0], 3), "launches": v[1],
                      "avg_us": round(1e3 * v[0] / v[1], 2) if v[1] else None,
                      "bytes_per_launch": b or None,
                      "GBps_algorithmic": round(gbs, 1) if gbs else None,
                      "frac_of_8TBps": round(gbs / HBM_PEAK_GBS, 4) if gbs else None,
                      "frac_of_copy": round(gbs / copy_peak, 4) if gbs else None}
    stencils = {k: kernels[k]["frac_of_8TBps"] for k in ("apply", "step", "mu", "solve_setup", "smooth")
                if kernels[k]["frac_of_8TBps"]}

    warm_txt = "previous step"
    if learned:
        warm_txt = (f"learned (network trained only on {args.train_workload} at {args.train_n}^3, solves "
                    f"0-{args.train_steps - 1}, then frozen; judged against the previous step)")
    line = {
        "metric": "voxel-steps/s at <=1e-4 rel err vs FP64 oracle; % of HBM peak; CG iters/step",
        "value": value, "unit": "voxel-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 arithmetic, f32-pair state, f64 reductions" if wl.precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": f"{wl.name} {'x'.join(str(x) for x in reversed(wl.shape))}, "
                               f"plasticity {'on' if wl.plasticity else 'off'}, Omega_f {wl.params.Omega_f:g}, "
                               f"CG rtol {wl.cg_rtol:g}, preconditioner = "
                               f"{'multigrid V-cycle' if precond == 'mg' else 'Jacobi'}, warm start = {warm_txt}; "
                               f"timed after {args.settle} + "
                               f"{args.warmup} untimed steps",
                   "cells": ncell, "dt_s": wl.dt, "h_m": wl.h},
        "cg_iters_per_step": res["cg_iters"] / args.steps,
        "cg_rel_resid_last": res["stats"]["cg_rel_resid"],
        "cg_resid_note": ("CG stops on the recursive residual at rtol; cg_rel_resid_last is the true "
                          "||b - A u|| / ||b|| of the last solve, recomputed after it (in FP32 arithmetic the "
                          "true residual of the FP32 iterate levels off near 1e-5)"),
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "timed_with": ("HIP events attached to every dispatch (hipExtLaunchKernel) in a replay of "
                                    "the timed steps from the same state; the throughput run carries no events"),
                     "launches_timed": nl, "replay_cg_iters_per_step": brk["cg_iters"] / args.steps,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "traffic_source": traffic_src,
                     "torch_copy_GBps": round(copy_peak, 1), "frac_of_copy": round(achieved / copy_peak, 4),
                     "bytes_per_launch": bytes_per_launch, "avg_launch_us": round(avg_s * 1e6, 2)},
        "stencil_kernels_frac_of_8TBps": stencils,
        "kernels": kernels,
        "kernels_note": "HIP events attached to every dispatch, in a replay of the timed steps from the same state",
    }
    if learned:
        nn_ms, nn_n = kern["nn"]
        if nn_n:
            avg = nn_ms / 1e3 / nn_n
            tf = NN_FLOP_PER_VOXEL * ncell / avg / 1e12
            line["roofline_nn"] = {"bound": "mfma", "kernel": "k_conv x4 (one inference)", "achieved": round(tf, 1),
                                   "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(tf / BF16_PEAK_TFLOPS, 4),
                                   "traffic": None, "flop_per_launch": NN_FLOP_PER_VOXEL * ncell,
                                   "avg_launch_us": round(avg * 1e6, 2)}
        line["training"] = train_info
        line["learned_last_step"] = {"warm_used": res["stats"].get("warm_used"), "r0_learned": res["stats"]["r0_learned"],
                                     "r0_prev": res["stats"]["r0_prev"]}
        net.close()
        rp = run_gpu(wl, wl.precision, args.steps, args.warmup, False, wl.cg_rtol, fields=start, precond=precond)
        line["plain_mixed_gpu"] = {"value": ncell * args.steps / rp["seconds"], "ms_per_step": 1e3 * rp["seconds"] / args.steps,
                                   "cg_iters_per_step": rp["cg_iters"] / args.steps,
                                   "note": "same state, steps and preconditioner, previous-step start"}
        line["learned_speedup_vs_plain_mixed"] = value / line["plain_mixed_gpu"]["value"]
    if precond == "mg":
        net_j = None
        if learned:
            net_j = pf.Net(max_voxels=ncell)
            net_j.set_params(params)
        rj = run_gpu(wl, wl.precision, args.steps, args.warmup, False, wl.cg_rtol, fields=start, net=net_j,
                     precond="jacobi")
        if net_j is not None:
            net_j.close()
        line["jacobi_pcg_gpu"] = {"value": ncell * args.steps / rj["seconds"], "ms_per_step": 1e3 * rj["seconds"] / args.steps,
                                  "cg_iters_per_step": rj["cg_iters"] / args.steps,
                                  "note": "same state, steps and warm start, Jacobi-preconditioned CG"}
        line["mg_speedup_vs_jacobi"] = value / line["jacobi_pcg_gpu"]["value"]
    if not args.no_fp64:
        s64 = max(4, args.steps // 2)
        r64 = run_gpu(wl, "fp64", s64, args.warmup, False, wl.cg_rtol, fields=start, precond=precond)
        line["fp64_gpu"] = {"value": ncell * s64 / r64["seconds"], "ms_per_step": 1e3 * r64["seconds"] / s64,
                            "cg_iters_per_step": r64["cg_iters"] / s64,
                            "note": f"plain FP64 GPU path, previous-step start, same state and preconditioner, "
                                    f"{s64} steps"}
        line["speedup_vs_fp64_gpu"] = value / line["fp64_gpu"]["value"]
    if not args.no_accuracy:
        print("[bench] accuracy sample", file=sys.stderr, flush=True)
        acc_n = args.acc_n or (48 if wl.dim == 3 else 256)
        line["accuracy"] = accuracy_sample(wl.name, acc_n, params=params, precond=precond)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(wl.name, args.cpu_n or (64 if wl.dim == 3 else 512))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
