"""Benchmark of the pressure-CG hot path on one MI355X.

Workload (default): 2D periodic unit square, 256 x 256 main cells, degree N = 6 (3,211,264
pressure DoFs), seeded random low-pass velocity (|k| <= 8, max |v| = 0.1), dt = 5e-4, nu = 1e-3,
theta = 0.6. One "step" is one full semi-implicit fractional step (L2 projections, TVD-RK3
convection, implicit viscous solves, divergence RHS, null-space projection, pressure CG to
relative residual 1e-10, velocity update) on device-resident data.

value = pressure DoFs x pressure-CG iterations / wall time of the timed steps (FP64 CG).
The FP32-inner / FP64-refinement path is timed the same way on the same state and reported
under "fp32_refine64". The roofline object covers the fused CG operator-apply kernel: its
duration is measured with HIP events around every launch inside the timed pressure solves.
The CPU baseline is the oracle's assembled-CSR CG timed in a 1-thread subprocess.

Workload batch2d_64 (separate invocation): 64 independent 2D periodic pressure problems, sides
and degrees drawn uniformly from 32..256 and 2..8 (seed 4), each with a standard-normal RHS scaled
to unit norm. One "step" is one batched solve of all problems to relative residual 1e-10 (FP32
iterations with FP64 residual replacement; FP64 CG timed beside it). value = sum over problems of
DoFs x iterations / wall time of the solve.

Workload adjoint3d_48_N3 (separate invocation): 3D periodic 48^3 cells, N = 3, 20 steps (dt 1e-3,
nu 1e-2, theta 0.6) from a seeded smoothed random velocity; one "step" is one gradient of the final
kinetic energy with respect to the initial velocity (checkpoints every 5 steps, solves to 1e-13),
followed by the central finite-difference check on 16 directions. value = pressure DoFs x
pressure-CG iterations (forward, recomputed and adjoint solves) / wall time of the gradients.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
                       [--workload rand2d_256_N6|rand3d_64_N4|batch2d_64|adjoint3d_48_N3]
"""
import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# the sources of the fused operator-apply kernels (the kernel itself and the device helpers it
# inlines); a counter summary is used only while they hash to the value recorded in it
KERNEL_SOURCES = ["paper_1602_05806_amd/csrc/pd_apply_kernels.h",
                  "paper_1602_05806_amd/csrc/pd_apply2d.h", "paper_1602_05806_amd/csrc/pd_device.h"]
# every TIMING_STRIDE-th operator launch of the timed solves carries dispatch events (events on
# every launch would add a few microseconds to each iteration of the measured solve)
TIMING_STRIDE = 16


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(workload, prec):
    """HBM bytes per launch of the fused apply kernel from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by the plain-copy calibration), or None when the
    summary is missing or was taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", f"apply_{prec}_{workload}_pmc.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_hash") != kernel_source_hash():
        return None
    try:
        return 1024.0 * (float(kv["fetch_kib_per_dispatch"]) * float(kv["copy_fetch_factor"]) +
                         float(kv["write_kib_per_dispatch"]) * float(kv["copy_write_factor"]))
    except (KeyError, ValueError):
        return None


METRIC = "pressure-CG DoF-iterations/s + HBM GB/s, FP64 vs FP32+FP64-refine at 1e-10"


def initial_state(pd, ctx, cfg, torch):
    import synthetic
    xi, _ = pd.pd_nodes(ctx)
    coords = synthetic.staggered_coords(cfg["cells"], cfg["lengths"], xi)
    field = synthetic.FourierField(cfg["seed"], len(cfg["cells"]), cfg["kmax"], cfg["lengths"])
    field.normalise(cfg["vmax"])
    U = field.eval(coords)
    n = cfg["N"] + 1
    return [torch.tensor(synthetic.tensor_to_blocked(u, cfg["cells"], n), dtype=torch.float64,
                         device="cuda") for u in U]


def run_steps(pd, ctx, u, p, nsteps, torch):
    iters, solves = 0, []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(nsteps):
        info = pd.pd_step(ctx, u, p)
        if info[3]["status"] != pd.PD_OK:
            raise RuntimeError(f"pressure solve failed: {info[3]}")
        iters += info[3]["iters"]
        solves.append(info)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, iters, solves


def device_copy_gbs(torch, mib=512, reps=10):
    """Measured HBM bandwidth of a plain device copy (torch copy_ of `mib` MiB, twice the size of
    the 256 MB Infinity Cache): read + write bytes / time, best of `reps`."""
    n = mib * 1024 * 1024 // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = float("inf")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(reps):
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3)
    del src, dst
    return 2.0 * n * 8 / best / 1e9


def cpu_baseline(cfg, iters=40):
    """Time the oracle (assembled CSR + plain CG loop) at the full workload size for a fixed number
    of iterations in a subprocess limited to one thread."""
    code = f"""
import time, json, os, sys
sys.path.insert(0, {ROOT!r})
import numpy as np
from oracle.operators import Grid, pressure_operator
from oracle.solvers import cg
g = Grid({tuple(cfg['cells'])!r}, {tuple(cfg['lengths'])!r}, {cfg['N']})
A = pressure_operator(g, {cfg['dt']})
b = np.random.default_rng(0).standard_normal(g.ndof)
t = time.perf_counter()
cg(A, b, 1e-300, {iters})
dt = time.perf_counter() - t
print(json.dumps(dict(value=g.ndof * {iters} / dt, seconds=dt, cores=len(os.sched_getaffinity(0)))))
"""
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                         timeout=600)
    if out.returncode != 0:
        return {"value": None, "unit": "DoF-iterations/s", "cores": 1, "kind": "oracle",
                "sample": f"failed: {out.stderr[-300:]}"}
    r = json.loads(out.stdout.strip().splitlines()[-1])
    return {"value": r["value"], "unit": "DoF-iterations/s", "cores": 1, "kind": "oracle",
            "sample": f"{iters} CG iterations of the assembled FP64 pressure matrix at the full "
                      f"workload size ({cfg['cells']} cells, N={cfg['N']}), scipy CSR matvec + "
                      f"numpy vector updates, 1 thread ({r['seconds']:.1f} s; host has "
                      f"{r['cores']} cores available)"}


def bench_batch(args, pd, torch):
    """Batched workload: one step = one pd_batch_cg_solve of every problem from x = 0."""
    import numpy as np
    import synthetic
    cfg = dict(synthetic.CONFIGS[args.workload])
    specs = synthetic.batch_problems(seed=cfg["seed"], count=cfg["count"],
                                     side_range=cfg["side_range"], N_range=cfg["N_range"])
    B = pd.pd_batch_setup([(p["side"], p["side"]) for p in specs], [(1.0, 1.0)] * len(specs),
                          [p["N"] for p in specs], cfg["dt"],
                          pd.PD_BATCH_AUTOTUNE if args.autotune else 0)
    parts = []
    for p in specs:
        r = synthetic.random_rhs(p["seed"], p["side"] ** 2 * (p["N"] + 1) ** 2)
        parts.append(r / np.linalg.norm(r))
    b = torch.tensor(np.concatenate(parts), dtype=torch.float64, device="cuda")
    del parts
    ndofs = [B.offsets[j + 1] - B.offsets[j] for j in range(B.count)]
    res = {}
    runs = (("fp32_refine64", pd.PD_FP32_REFINE64, 0), ("fp64", pd.PD_FP64, 0),
            ("pcg_fp32_refine64", pd.PD_FP32_REFINE64, 1), ("pcg_fp64", pd.PD_FP64, 1))
    for name, prec, pc in runs:
        pd.pd_batch_configure(B, pd.PD_BCFG_PRECOND, pc)
        x = torch.zeros(B.total, dtype=torch.float64, device="cuda")
        for _ in range(args.warmup):
            pd.pd_batch_cg_solve(B, prec, b, x, cfg["rtol"], cfg["maxit"])
            print(f"bench.py: batch {name} warm-up solve done", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        work, infos = 0, None
        for step in range(args.steps):
            rc, infos = pd.pd_batch_cg_solve(B, prec, b, x, cfg["rtol"], cfg["maxit"])
            if rc != pd.PD_OK:
                raise RuntimeError(f"batched solve failed ({name}): rc {rc}")
            work += sum(n * i["iters"] for n, i in zip(ndofs, infos))
            print(f"bench.py: batch {name} step {step + 1}/{args.steps} done", file=sys.stderr,
                  flush=True)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        bytes_it = 36.0 if prec == pd.PD_FP32_REFINE64 else 72.0   # 9 vector words per DoF
        res[name] = dict(seconds=secs, work=work, infos=infos, bytes_it=bytes_it)
        del x
    r32, r64 = res["fp32_refine64"], res["fp64"]
    p32, p64 = res["pcg_fp32_refine64"], res["pcg_fp64"]
    value = r32["work"] / r32["seconds"]
    falls = [j for j, i in enumerate(r32["infos"]) if i["fallback_iter"] >= 0]
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "DoF-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * r32["seconds"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "problems": B.count, "total_dofs": B.total,
                   "sides": [p["side"] for p in specs], "N": [p["N"] for p in specs],
                   "rtol": cfg["rtol"], "dt": cfg["dt"], "autotune": bool(args.autotune)},
        "solve_ms": 1e3 * r32["seconds"] / args.steps,
        "max_iters": max(i["iters"] for i in r32["infos"]),
        "fp64_fallback_problems": falls,
        "algorithmic_gbs_cg": r32["work"] * r32["bytes_it"] / r32["seconds"] / 1e9,
        "rel_res_true_max": max(i["rel_res_true"] for i in r32["infos"]),
        "fp64": {"value": r64["work"] / r64["seconds"], "unit": "DoF-iterations/s",
                 "solve_ms": 1e3 * r64["seconds"] / args.steps,
                 "max_iters": max(i["iters"] for i in r64["infos"]),
                 "algorithmic_gbs_cg": r64["work"] * r64["bytes_it"] / r64["seconds"] / 1e9,
                 "rel_res_true_max": max(i["rel_res_true"] for i in r64["infos"])},
        "speedup_solve_vs_fp64": r64["seconds"] / r32["seconds"],
        # the same solves with the cell-block Jacobi preconditioner (PD_BCFG_PRECOND)
        "preconditioned": {
            "fp64": {"solve_ms": 1e3 * p64["seconds"] / args.steps,
                     "max_iters": max(i["iters"] for i in p64["infos"]),
                     "rel_res_true_max": max(i["rel_res_true"] for i in p64["infos"])},
            "fp32_refine64": {"solve_ms": 1e3 * p32["seconds"] / args.steps,
                              "max_iters": max(i["iters"] for i in p32["infos"]),
                              "rel_res_true_max": max(i["rel_res_true"] for i in p32["infos"])},
            "speedup_fp64_vs_plain_fp64": r64["seconds"] / p64["seconds"],
            "speedup_fp32_refine64_vs_plain_fp64": r64["seconds"] / p32["seconds"],
            "speedup_fp32_refine64_vs_fp64": p64["seconds"] / p32["seconds"],
            "iters_per_problem_fp64": [i["iters"] for i in p64["infos"]]},
        "per_problem": [{"side": p["side"], "N": p["N"], "iters_refine": i["iters"],
                         "fp64_from": i["fallback_iter"], "iters_fp64": k["iters"]}
                        for p, i, k in zip(specs, r32["infos"], r64["infos"])],
    }
    B.close()
    print(json.dumps(line))


def next_rows(pd, torch):
    """Measurements of the extensions beyond the paper's semi-implicit periodic step, on the
    benchmark's grids: homogeneous Dirichlet pressure walls on every side (64^3 N = 4 pressure
    solve against the periodic one, with the fused apply's live rate), the explicit-viscosity
    step and the space-time step (M = 1, 2; explicit viscous flux) of 256^2 N = 6 against the
    semi-implicit step at the same viscosity (nu = 4e-5, inside the explicit CFL bound)."""
    import synthetic
    out = {}
    # walls: 64^3 N = 4, white right-hand side, FP64 to 1e-10
    cells, N, dt = (64, 64, 64), 4, 1e-3
    for name, mask in (("periodic", 7), ("walls", 0)):
        ctx = pd.pd_setup(3, cells, (1.0, 1.0, 1.0), N, dt, 0.6, 1e-3, periodic_mask=mask)
        b = torch.tensor(synthetic.random_rhs(17, ctx.ndof), dtype=torch.float64, device="cuda")
        x = torch.zeros_like(b)
        pd.pd_cg_solve(ctx, pd.PD_OP_PRESSURE, pd.PD_FP64, b, x, 1e-10, 400000)   # warm-up
        pd.pd_configure(ctx, pd.PD_CFG_TIMING, TIMING_STRIDE)
        pd.pd_timing(ctx, pd.PD_FP64, reset=True)
        x.zero_()
        info = pd.pd_cg_solve(ctx, pd.PD_OP_PRESSURE, pd.PD_FP64, b, x, 1e-10, 400000)
        kt = pd.pd_timing(ctx, pd.PD_FP64, reset=True)
        avg_ms, gbs = kernel_rate(kt)
        out[f"{name}_rand3d_64_N4_solve"] = dict(
            iters=info["iters"], solve_ms=info["ms"], rel_res_true=info["rel_res_true"],
            apply_us=1e3 * avg_ms, apply_gbs=gbs, apply_frac=gbs / HBM_PEAK_GBS if gbs else None)
        ctx.close()
        del b, x
    # explicit viscosity and the space-time step on 256^2 N = 6
    cfg = dict(synthetic.CONFIGS["rand2d_256_N6"])
    cfg["nu"] = 4e-5
    for name, theta, evisc, M in (("semi_implicit", 1.0, 0, None), ("explicit_viscosity", 1.0, 1, None),
                                  ("space_time_M1", 1.0, 1, 1), ("space_time_M2", 1.0, 1, 2)):
        ctx = pd.pd_setup(2, cfg["cells"], cfg["lengths"], cfg["N"], cfg["dt"], theta, cfg["nu"])
        pd.pd_configure(ctx, pd.PD_CFG_P_RTOL, cfg["rtol"])
        pd.pd_configure(ctx, pd.PD_CFG_EXPLICIT_VISC, evisc)
        u = initial_state(pd, ctx, cfg, torch)
        steps, iters, solves = 3, 0, 0
        if M is None:
            p = torch.zeros(ctx.ndof, dtype=torch.float64, device="cuda")
            pd.pd_step(ctx, u, p)                                          # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                info = pd.pd_step(ctx, u, p)
                iters += info[3]["iters"]
                solves += 1
        else:
            p = torch.zeros((M + 1) * ctx.ndof, dtype=torch.float64, device="cuda")
            pd.pd_step_st(ctx, M, u, p)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                info = pd.pd_step_st(ctx, M, u, p)
                for i in info[3:]:
                    iters += i["iters"]
                    solves += 1
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        out[f"{name}_rand2d_256_N6"] = dict(ms_per_step=1e3 * secs / steps,
                                            pressure_solves_per_step=solves / steps,
                                            pressure_iters_per_step=iters / steps, nu=cfg["nu"])
        ctx.close()
        del u, p
    return out


def bench_adjoint(args, pd, torch):
    """Adjoint workload: one step = one gradient of the final kinetic energy with respect to the
    initial velocity (forward rollout with checkpoints, backward with segment recomputation and
    pd_step_adjoint), solves to 1e-13; then the central finite-difference check."""
    import synthetic
    from paper_1602_05806_amd import autograd as ag
    cfg = dict(synthetic.CONFIGS[args.workload])
    cells, N = cfg["cells"], cfg["N"]
    ctx = pd.pd_setup(3, cells, cfg["lengths"], N, cfg["dt"], cfg["theta"], cfg["nu"])
    pd.pd_configure(ctx, pd.PD_CFG_P_RTOL, 1e-13)
    pd.pd_configure(ctx, pd.PD_CFG_V_RTOL, 1e-13)
    xi, _ = pd.pd_nodes(ctx)
    field = synthetic.FourierField(cfg["seed"], 3, cfg["kmax"], cfg["lengths"])
    field.normalise(cfg["vmax"])
    U = field.eval(synthetic.staggered_coords(cells, cfg["lengths"], xi))
    u0 = [torch.tensor(synthetic.tensor_to_blocked(x, cells, N + 1), device="cuda") for x in U]
    steps, every = cfg["steps"], cfg["checkpoint"]

    def gradient():
        ur = [x.clone().requires_grad_(True) for x in u0]
        loss = ag.kinetic_energy(ctx, ag.Rollout.apply(ctx, steps, every, *ur))
        loss.backward()
        return float(loss.detach()), [x.grad for x in ur]

    for _ in range(args.warmup):
        gradient()
    for k in ag.stats:
        ag.stats[k] = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        loss, grad = gradient()
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    st = dict(ag.stats)
    fd = []
    unorm = float(torch.sqrt(sum((x * x).sum() for x in u0)))
    coords = synthetic.staggered_coords(cells, cfg["lengths"], xi)
    for k in range(args.fd_dirs):
        fk = synthetic.FourierField(5000 + k, 3, cfg["kmax"], cfg["lengths"])
        fk.normalise(1.0)
        v = [torch.tensor(synthetic.tensor_to_blocked(x, cells, N + 1), device="cuda")
             for x in fk.eval(coords)]
        eps = 1e-6 * unorm / float(torch.sqrt(sum((x * x).sum() for x in v)))
        with torch.no_grad():
            fp = float(ag.kinetic_energy(ctx, ag.Rollout.apply(
                ctx, steps, every, *[a + eps * b for a, b in zip(u0, v)])))
            fm = float(ag.kinetic_energy(ctx, ag.Rollout.apply(
                ctx, steps, every, *[a - eps * b for a, b in zip(u0, v)])))
        f = (fp - fm) / (2 * eps)
        gv = float(sum((a * b).sum() for a, b in zip(grad, v)))
        fd.append(abs(gv - f) / abs(f))
    ndof = ctx.ndof
    value = ndof * st["pressure_iters"] / secs
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "DoF-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * secs / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "cells": list(cells), "N": N,
                   "dofs_per_component": ndof, "time_steps": steps, "checkpoint_every": every,
                   "dt": cfg["dt"], "nu": cfg["nu"], "theta": cfg["theta"], "rtol": 1e-13,
                   "step": "gradient of the final kinetic energy (forward + adjoint)"},
        "loss": loss,
        "forward_steps_per_gradient": st["steps"] / args.steps,
        "adjoint_steps_per_gradient": st["adjoint_steps"] / args.steps,
        "pressure_iters_per_gradient": st["pressure_iters"] / args.steps,
        "viscous_iters_per_gradient": st["viscous_iters"] / args.steps,
        "fd_check": {"directions": args.fd_dirs, "max_rel_err": max(fd) if fd else None,
                     "rel_errs": fd, "eps": "1e-6 ||U0|| / ||v||",
                     "direction_kind": "smooth random Fourier fields, wavenumbers <= 6",
                     "seeds": "5000 + k"},
    }
    ctx.close()
    print(json.dumps(line))


# Workloads timed by the default invocation: the metric's workload (2D, whose FP64 CG working set
# of about 128 MB sits in the 256 MB Infinity Cache) and the 3D workload whose 1.3 GB working set
# streams from HBM (the roofline workload).
DEFAULT_WORKLOADS = ("rand2d_256_N6", "rand3d_64_N4")
# tolerances at which each path reaches the 1e-10 relative L2 error target, with a margin, on a
# white-noise right-hand side (every mode present), measured against the exact minimum-norm
# solution (errors 3.2e-11 / 1.8e-11 in 2D, 4.7e-11 / 2.0e-11 in 3D)
MATCHED_WHITE_RTOL = {"rand2d_256_N6": {"fp64": 2e-11, "fp32_refine64": 2e-12},
                      "rand3d_64_N4": {"fp64": 5e-12, "fp32_refine64": 2e-12}}


def make_ctx(pd, cfg):
    dim = len(cfg["cells"])
    ctx = pd.pd_setup(dim, cfg["cells"], cfg["lengths"], cfg["N"], cfg["dt"], cfg["theta"],
                      cfg["nu"])
    pd.pd_configure(ctx, pd.PD_CFG_P_RTOL, cfg["rtol"])
    return ctx


def time_steps(pd, torch, ctx, cfg, u, p, steps, warmup):
    """Warm-up steps, then `steps` timed fractional steps per precision on copies of (u, p);
    the fused operator kernel of the pressure solves is timed by dispatch events."""
    dim = len(cfg["cells"])
    results = {}
    for prec_name, prec in (("fp64", pd.PD_FP64), ("fp32_refine64", pd.PD_FP32_REFINE64)):
        pd.pd_configure(ctx, pd.PD_CFG_STEP_PREC, prec)
        u_run = [x.clone() for x in u]
        p_run = p.clone()
        pd.pd_configure(ctx, pd.PD_CFG_TIMING, 0)
        run_steps(pd, ctx, u_run, p_run, warmup, torch)
        pd.pd_configure(ctx, pd.PD_CFG_TIMING, TIMING_STRIDE)
        pd.pd_timing(ctx, pd.PD_FP64, reset=True)
        pd.pd_timing(ctx, pd.PD_FP32, reset=True)
        secs, iters, solves = run_steps(pd, ctx, u_run, p_run, steps, torch)
        pd.pd_configure(ctx, pd.PD_CFG_TIMING, 0)
        kt = pd.pd_timing(ctx, pd.PD_FP64 if prec == pd.PD_FP64 else pd.PD_FP32, reset=True)
        results[prec_name] = dict(
            seconds=secs, iters=iters, psolve_ms=sum(s[3]["ms"] for s in solves),
            outer=[s[3]["outer_iters"] for s in solves],
            rel_res_true=max(s[3]["rel_res_true"] for s in solves),
            visc_iters=[[s[d]["iters"] for d in range(dim)] for s in solves], kernel=kt)
        del u_run, p_run
    pd.pd_configure(ctx, pd.PD_CFG_STEP_PREC, pd.PD_FP64)
    return results


def kernel_rate(kt):
    avg_ms = kt["total_ms"] / max(kt["launches"], 1)
    gbs = kt["bytes_per_launch"] / (avg_ms * 1e-3) / 1e9 if kt["launches"] else None
    return avg_ms, gbs


def error_solves(pd, torch, ctx, cfg, u0, wl, outdir):
    """Pressure solves whose results the oracle checks after the timed region: the workload's
    own kind of right-hand side, b = sum_d B_d U0_d of its seeded initial velocity, at the timed
    rtol, and a white-noise right-hand side (seed 17) at the tolerance each path needs for the
    1e-10 error target. Solutions go to .npy files; returns the solve reports."""
    import numpy as np
    b = torch.empty(ctx.ndof, dtype=torch.float64, device="cuda")
    pd.pd_rhs_div(ctx, u0, b)
    import synthetic
    white = torch.tensor(synthetic.random_rhs(17, ctx.ndof), dtype=torch.float64, device="cuda")
    reports = {}
    for rhs_name, rhs in (("workload_rhs", b), ("white_rhs", white), ("workload_rhs_pcg", b)):
        pd.pd_configure(ctx, pd.PD_CFG_PRECOND, 1 if rhs_name.endswith("pcg") else 0)
        for prec_name, prec in (("fp64", pd.PD_FP64), ("fp32_refine64", pd.PD_FP32_REFINE64)):
            rtol = MATCHED_WHITE_RTOL[wl][prec_name] if rhs_name == "white_rhs" else cfg["rtol"]
            x = torch.zeros_like(rhs)
            pd.pd_cg_solve(ctx, pd.PD_OP_PRESSURE, prec, rhs, x, rtol, 400000)   # warm-up
            x.zero_()
            info = pd.pd_cg_solve(ctx, pd.PD_OP_PRESSURE, prec, rhs, x, rtol, 400000)
            if info["status"] != pd.PD_OK:
                raise RuntimeError(f"{wl} {rhs_name} {prec_name}: solve failed {info}")
            path = os.path.join(outdir, f"{wl}_{rhs_name}_{prec_name}.npy")
            np.save(path, x.cpu().numpy())
            reports[(rhs_name, prec_name)] = dict(rtol=rtol, iters=info["iters"], ms=info["ms"],
                                                  rel_res_true=info["rel_res_true"], path=path)
            del x
    pd.pd_configure(ctx, pd.PD_CFG_PRECOND, 0)
    del b, white
    return reports


ERROR_CHECK = r"""
import json, sys, time
import numpy as np
from oracle.operators import Grid, div_rhs_apply
from oracle.solvers import FastDiag
from oracle import layout
import synthetic


def errors(cfg, paths):
    cells, N, L = tuple(cfg["cells"]), cfg["N"], tuple(cfg["lengths"])
    g = Grid(cells, L, N)
    field = synthetic.FourierField(cfg["seed"], len(cells), cfg["kmax"], L).normalise(cfg["vmax"])
    U = field.eval(synthetic.staggered_coords(cells, L, g.tab.xi))
    rhs = {"workload_rhs": div_rhs_apply(g, U),
           "white_rhs": layout.blocked_to_tensor(synthetic.random_rhs(17, g.ndof), cells, N + 1)}
    del U
    fd = FastDiag(g)
    W = np.ones(g.shape())
    for d in range(g.dim):
        shp = [1] * g.dim
        shp[g.dim - 1 - d] = -1
        W = W * np.tile(g.tab.w, cells[d]).reshape(shp)
    out = {}
    for kind in ("workload_rhs", "white_rhs"):
        ref = fd.solve(rhs[kind], 0.0, cfg["dt"])
        nref = np.sqrt(np.sum(W * ref ** 2))
        for sol in (kind, kind + "_pcg"):
            for prec in ("fp64", "fp32_refine64"):
                if sol + "|" + prec not in paths:
                    continue
                X = layout.blocked_to_tensor(np.load(paths[sol + "|" + prec]), cells, N + 1)
                out[sol + "|" + prec] = float(np.sqrt(np.sum(W * (X - ref) ** 2)) / nref)
    return out
"""


def cpu_leg(main_cfg, checks, timeout=1200):
    """The oracle's legs, after the timed GPU work, in subprocesses: its CG timed at the main
    workload's size on one thread (cpu_baseline), and its check of the saved GPU solutions
    (its own right-hand sides: the matrix-free divergence of the same seeded velocity field and
    the same seeded white noise; its fast-diagonalisation minimum-norm solutions; mass-weighted
    relative L2 errors). checks: list of (cfg, workload, reports)."""
    base = cpu_baseline(main_cfg)
    errs = {}
    for cfg, wl, reports in checks:
        code = ("import json, sys\nsys.path.insert(0, %r)\n" % ROOT) + ERROR_CHECK + (
            "\nt0 = time.perf_counter()\nres = errors(%r, %r)\n"
            "print(json.dumps(dict(errors=res, seconds=time.perf_counter() - t0)))\n"
            % ({k: cfg[k] for k in ("cells", "N", "lengths", "seed", "kmax", "vmax", "dt")},
               {f"{k[0]}|{k[1]}": v["path"] for k, v in reports.items()}))
        out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                             timeout=timeout)
        if out.returncode != 0:
            errs[wl] = (None, "oracle check failed: " + out.stderr[-400:])
        else:
            errs[wl] = (json.loads(out.stdout.strip().splitlines()[-1]), None)
    return base, errs


def workload_line(pd, torch, wl, args, steps, warmup, outdir):
    """Time one workload; returns (summary dict, error-solve reports, ctx sizes)."""
    import synthetic
    cfg = dict(synthetic.CONFIGS[wl])
    ctx = make_ctx(pd, cfg)
    if wl.startswith("rand3d"):
        pd.pd_configure(ctx, pd.PD_CFG_CONVECTION, 0)    # one pressure + viscous solve per step
    u = initial_state(pd, ctx, cfg, torch)
    p = torch.zeros(ctx.ndof, dtype=torch.float64, device="cuda")
    res = time_steps(pd, torch, ctx, cfg, u, p, steps, warmup)
    reports = {} if args.no_check else error_solves(pd, torch, ctx, cfg, u, wl, outdir)
    ndof = ctx.ndof
    ctx.close()
    del u, p
    r64, r32 = res["fp64"], res["fp32_refine64"]
    avg64, gbs64 = kernel_rate(r64["kernel"])
    avg32, gbs32 = kernel_rate(r32["kernel"])
    apply_words = r64["kernel"]["bytes_per_launch"] / (8.0 * ndof) if r64["kernel"]["launches"] else 6.0
    cg_words = 8.0 if apply_words > 7.0 else apply_words + 3.0
    summary = {
        "workload": wl, "cells": list(cfg["cells"]), "N": cfg["N"], "pressure_dofs": ndof,
        "rtol": cfg["rtol"], "steps": steps,
        "fp64": {
            "value": ndof * r64["iters"] / r64["seconds"], "unit": "DoF-iterations/s",
            "ms_per_step": 1e3 * r64["seconds"] / steps,
            "pressure_iters_per_step": r64["iters"] / steps,
            "pressure_solve_ms_per_step": r64["psolve_ms"] / steps,
            "pressure_dof_it_per_s_solve_only": ndof * r64["iters"] / (r64["psolve_ms"] * 1e-3),
            "cg_words_per_dof_it": cg_words,
            "algorithmic_gbs_cg": ndof * r64["iters"] * 8.0 * cg_words / (r64["psolve_ms"] * 1e-3) / 1e9,
            "rel_res_true_max": r64["rel_res_true"],
            "viscous_iters": r64["visc_iters"][0] if r64["visc_iters"] else None,
            "apply_kernel": {"avg_launch_us": 1e3 * avg64, "achieved_gbs": gbs64,
                             "frac": gbs64 / HBM_PEAK_GBS if gbs64 else None,
                             "launches": r64["kernel"]["launches"],
                             "bytes_per_launch": r64["kernel"]["bytes_per_launch"],
                             "traffic": measured_traffic(wl, "fp64")}},
        "fp32_refine64": {
            "value": ndof * r32["iters"] / r32["seconds"], "unit": "DoF-iterations/s",
            "ms_per_step": 1e3 * r32["seconds"] / steps,
            "pressure_iters_per_step": r32["iters"] / steps,
            "outer_iters": r32["outer"],
            "pressure_solve_ms_per_step": r32["psolve_ms"] / steps,
            "speedup_pressure_solve_vs_fp64": r64["psolve_ms"] / r32["psolve_ms"],
            "rel_res_true_max": r32["rel_res_true"],
            "apply_kernel": {"avg_launch_us": 1e3 * avg32, "achieved_gbs": gbs32,
                             "frac": gbs32 / HBM_PEAK_GBS if gbs32 else None,
                             "launches": r32["kernel"]["launches"],
                             "bytes_per_launch": r32["kernel"]["bytes_per_launch"],
                             "traffic": measured_traffic(wl, "fp32")}},
    }
    return cfg, summary, reports


def attach_errors(summary, reports, checked):
    """Error of every checked solve against the oracle (after the timed region) and the speed-up
    of the refined path at matched error."""
    errs, msg = checked
    block = {}
    for (rhs_name, prec_name), r in reports.items():
        e = errs["errors"].get(f"{rhs_name}|{prec_name}") if errs else None
        block.setdefault(rhs_name, {})[prec_name] = {
            "rtol": r["rtol"], "iters": r["iters"], "solve_ms": r["ms"],
            "rel_res_true": r["rel_res_true"], "error_vs_oracle": e}
    for rhs_name, b in block.items():
        b["speedup_fp32_refine64_vs_fp64"] = b["fp64"]["solve_ms"] / b["fp32_refine64"]["solve_ms"]
        b["target_met"] = (None if not errs else all(
            b[k]["error_vs_oracle"] is not None and b[k]["error_vs_oracle"] <= 1e-10
            for k in ("fp64", "fp32_refine64")))
    block["workload_rhs"]["kind"] = ("b = sum_d B_d U0_d of the workload's seeded initial "
                                     "velocity, both paths at the timed rtol")
    pc, base = block.get("workload_rhs_pcg"), block["workload_rhs"]
    if pc is not None:
        pc["kind"] = ("the workload right-hand side with the cell-block Jacobi preconditioned CG "
                      "(PD_CFG_PRECOND) at the timed rtol")
        for k in ("fp64", "fp32_refine64"):
            pc[k]["speedup_vs_unpreconditioned"] = base[k]["solve_ms"] / pc[k]["solve_ms"]
        pc["speedup_fp32_refine64_pcg_vs_fp64_cg"] = (base["fp64"]["solve_ms"] /
                                                      pc["fp32_refine64"]["solve_ms"])
    block["white_rhs"]["kind"] = ("standard-normal b (seed 17), each path at the tolerance it "
                                  "needs for the 1e-10 error target")
    block["error_measure"] = "mass-weighted relative L2 against the oracle's minimum-norm solution"
    if errs is None:
        block["oracle"] = msg
    else:
        block["oracle_seconds"] = errs["seconds"]
    summary["error_vs_oracle"] = block


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rand2d_256_N6")
    ap.add_argument("--no-cpu", action="store_true",
                    help="skip the oracle legs (CPU baseline and the error check)")
    ap.add_argument("--steps3d", type=int, default=3,
                    help="timed steps of the 3D roofline workload in the default invocation")
    ap.add_argument("--single", action="store_true",
                    help="time only --workload (the default invocation also times the 3D one)")
    ap.add_argument("--no-check", action="store_true",
                    help="skip the error solves and the oracle legs (profiling runs)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain 256 MiB device copy (counter calibration)")
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="batch2d_64: the largest fitting tile everywhere instead of the tile "
                         "shapes the autotuner picks per (degree, size bucket, precision)")
    ap.add_argument("--fd-dirs", type=int, default=16,
                    help="adjoint3d_48_N3: finite-difference directions checked after timing")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (the pressure path is measured on one "
              "GPU's share); --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import tempfile
    import torch
    import paper_1602_05806_amd as pd

    if args.calibrate_copy:
        src = torch.randn(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.workload.startswith("batch"):
        bench_batch(args, pd, torch)
        return
    if args.workload.startswith("adjoint"):
        bench_adjoint(args, pd, torch)
        return
    main_wl = args.workload
    extra = ([w for w in DEFAULT_WORKLOADS if w != main_wl]
             if main_wl == DEFAULT_WORKLOADS[0] and not args.single else [])
    if args.no_check:
        args.no_cpu = True
    with tempfile.TemporaryDirectory(prefix="pd_bench_") as outdir:
        cfg, s_main, rep_main = workload_line(pd, torch, main_wl, args, args.steps, args.warmup,
                                              outdir)
        others = []
        for wl in extra:
            print(f"bench.py: timing {wl}", file=sys.stderr, flush=True)
            others.append((wl,) + workload_line(pd, torch, wl, args, args.steps3d, 1, outdir))
        copy_gbs = device_copy_gbs(torch)
        nxt = None if (args.single or args.no_check) else next_rows(pd, torch)
        checks = [(cfg, main_wl, rep_main)] + [(c, wl, r) for wl, c, s, r in others]
        if args.no_check:
            base, errs = None, None
        elif args.no_cpu:
            base, errs = None, {wl: (None, "skipped (--no-cpu)") for _, wl, _ in checks}
        else:
            print("bench.py: oracle legs", file=sys.stderr, flush=True)
            base, errs = cpu_leg(cfg, checks)
        if errs is not None:
            attach_errors(s_main, rep_main, errs[main_wl])
            for wl, c, s, r in others:
                attach_errors(s, r, errs[wl])
    # roofline: the fused FP64 operator kernel of the workload that streams from HBM (the 3D one
    # when the default invocation times it), else of the timed workload itself
    hbm = next((s for wl, c, s, r in others if wl.startswith("rand3d")), s_main)
    ak = hbm["fp64"]["apply_kernel"]
    roof = {"bound": "hbm", "achieved": ak["achieved_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ak["frac"], "traffic": ak["traffic"],
            "kernel": ("k_apply3d (fused CG form, FP64)" if hbm["workload"].startswith("rand3d")
                       else "k_apply2d (fused CG form, FP64)"),
            "workload": hbm["workload"], "avg_launch_us": ak["avg_launch_us"],
            "launches": ak["launches"], "bytes_per_launch": ak["bytes_per_launch"],
            "copy_gbs": copy_gbs,
            "frac_of_copy": (ak["achieved_gbs"] / copy_gbs) if ak["achieved_gbs"] else None}
    f64 = s_main["fp64"]
    line = {
        "metric": METRIC,
        "value": f64["value"],
        "unit": "DoF-iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": f64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": main_wl, "cells": list(cfg["cells"]), "N": cfg["N"],
                   "pressure_dofs": s_main["pressure_dofs"], "dt": cfg["dt"], "nu": cfg["nu"],
                   "theta": cfg["theta"], "rtol": cfg["rtol"],
                   "step": "full fractional step" if not main_wl.startswith("rand3d")
                   else "fractional step without convection"},
        "roofline": roof,
        "fp64": {k: v for k, v in f64.items() if k not in ("value", "unit", "ms_per_step")},
        "fp32_refine64": s_main["fp32_refine64"],
        "error_vs_oracle": s_main.get("error_vs_oracle"),
        "roofline_2d_infinity_cache_resident": {
            "workload": s_main["workload"], "kernel": "k_apply2d (fused CG form, FP64)",
            "note": "FP64 CG working set ~128 MB, held in the 256 MB Infinity Cache",
            **f64["apply_kernel"]} if hbm is not s_main else None,
        "other_workloads": {wl: s for wl, c, s, r in others},
        # Dirichlet walls, explicit viscosity and the space-time step on the benchmark grids
        "extensions": nxt,
        "kernel_source_hash": kernel_source_hash(),
    }
    if base is not None:
        line["cpu_baseline"] = base
    print(json.dumps(line))


if __name__ == "__main__":
    main()
