"""Benchmark: implicit steps/s of the JFNK + physics-based-preconditioner step on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload stratified_2d] [--gpus 1]

A step is one implicit time step X^n -> X^{n+1} (CFL time step from X^n, Newton to
||R^-1 dX||_inf < 1e-8, FGMRES(30) with CGS2, finite-difference J.v, physics-based
preconditioner with multigrid CG).  Default workload: 2D stratified polytrope 256x256 (x
periodic, walls in y, density contrast 10, constant conductivity, Mach 1e-3 velocity
noise), CFL_hydro = 100, sound + thermal preconditioner, FP64 throughout.  W warm-up steps
run from X^0 and are discarded; then K steps are timed from X^0 (the workload's 10 steps
when K = 10).

Also reported on the same state: residual and J.v cell-updates/s (HIP events around each
kernel launch on the library's stream), the HBM roofline of the dominant kernel, and the
CPU oracle timed on a bounded sample.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "implicit steps/s and J·v cell-updates/s at fixed Newton tol; % HBM peak"
HBM_PEAK_GBS = 8000.0


WORKLOADS = ("acoustic_bump_2d", "stratified_2d", "taylor_green_3d", "stratified_2d_kappa",
             "convective_box_3d", "radiative_2d")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="stratified_2d", choices=sorted(WORKLOADS))
    ap.add_argument("--jv", default=None, choices=["fd", "exact"])
    ap.add_argument("--ell", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tuned", action="store_true",
                    help="skip the second timing with one V-cycle per elliptic solve")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="stratified_2d_kappa: skip the adjoint run (gradient through the steps, FD-checked)")
    ap.add_argument("--no-kernels-3d", dest="kernels_3d", action="store_false",
                    help="skip the kernel rates at the 256^3 production size")
    ap.add_argument("--only-kernels-3d", action="store_true",
                    help="only time the single-launch kernels at 256^3 (for profiling them)")
    ap.add_argument("--compare", action="store_true",
                    help="also time the exact-J.v + FP32-elliptic form on the same steps")
    ap.add_argument("--cpu-budget-s", type=float, default=30.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a device copy of 1 GiB five times (calibrates FETCH_SIZE and "
                         "WRITE_SIZE counters against known bytes)")
    return ap.parse_args()


def copy_calibration():
    import torch
    n = (1 << 30) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read_per_launch": 8 * n, "copy_bytes_written_per_launch": 8 * n,
                      "launches": 5}), flush=True)


def source_sha256(rel):
    import hashlib
    with open(os.path.join(ROOT, rel), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic(workload_name, kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary of this workload
    (FETCH_SIZE and WRITE_SIZE per dispatch, scaled by the copy-kernel calibration), or None
    when there is none for this kernel or its source has changed since the counters were
    taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload_name}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if line.startswith("#") or ":" not in line:
                continue
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    try:
        if kv.get("kernel") != kernel or source_sha256(kv["source"]) != kv["source_sha256"]:
            return None
        return 1024.0 * (float(kv["fetch_kib_per_launch"]) * float(kv["fetch_calibration"])
                         + float(kv["write_kib_per_launch"]) * float(kv["write_calibration"]))
    except (KeyError, ValueError, OSError):
        return None


def workload(name):
    import workloads as W
    w = W.CONFIGS[name]()
    return w


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU domain decomposition is a design, not an implementation.",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1512_03662_amd as J

    dev = torch.device("cuda:0")
    if args.copy_calibration:
        copy_calibration()
        return
    if args.only_kernels_3d:
        import workloads as Wl
        w5 = Wl.convective_box_3d(n=256)
        X5 = torch.tensor(w5["X0"], dtype=torch.float64, device=dev)
        ctx5 = J.Context(w5["problem"], gmres_m=1, precond="none")
        r = kernel_rates(J, ctx5, X5, w5["cfl"], int(np.prod(w5["problem"]["shape"])), 5,
                         args.kernel_reps, prefix="3d256_")
        print(json.dumps({"workload": w5["name"], "kernels": r}), flush=True)
        return
    w = workload(args.workload)
    pd = w["problem"]
    jv = args.jv or w["jv_mode"]
    precond = w["precond"]
    X0 = torch.tensor(w["X0"], dtype=torch.float64, device=dev)
    N = int(np.prod(pd["shape"]))
    nvar = 2 + len(pd["shape"])
    ctx = J.Context(pd, precond=precond, jv_mode=jv, ell_precision=args.ell)
    cfl = w["cfl"]

    def run_steps(k):
        X = X0.clone()
        stats = []
        for _ in range(k):
            dt = ctx.cfl_dt(X, cfl)
            stats.append(ctx.implicit_step(X, dt))
        return X, stats

    print(f"# workload {w['name']}: warm-up {args.warmup} step(s)", file=sys.stderr, flush=True)
    run_steps(args.warmup)
    torch.cuda.synchronize()
    print(f"# timing {args.steps} step(s)", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    Xk, stats = run_steps(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sec = t1 - t0
    steps_per_s = args.steps / sec

    # ---- probe pass: the same K steps with every kernel launch timed by HIP events -------
    print("# probe pass", file=sys.stderr, flush=True)
    from paper_1512_03662_amd import _native as Nat
    Nat.probe_enable(True)
    run_steps(args.steps)
    torch.cuda.synchronize()
    probes = Nat.probe_results()
    Nat.probe_enable(False)
    dom = max(probes.items(), key=lambda kv: kv[1][0])
    dom_name, (dom_ms, dom_n, dom_bytes) = dom
    avg_s = dom_ms * 1e-3 / dom_n
    achieved = dom_bytes / dom_n / avg_s / 1e9
    traffic = measured_traffic(w["name"], dom_name)
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": dom_name,
                "launches": dom_n, "avg_us": avg_s * 1e6,
                "algorithmic_bytes_per_launch": dom_bytes / dom_n,
                "share_of_kernel_time": dom_ms / sum(v[0] for v in probes.values())}

    # ---- kernel rates: residual, exact and FD J.v, vjp on X^0 of this workload -------------
    kernels = kernel_rates(J, ctx, X0, cfl, N, nvar, args.kernel_reps, prefix="")
    # and at the full 3D production size (256^3 convective box, 5 variables)
    if args.kernels_3d:
        import workloads as Wl
        w5 = Wl.convective_box_3d(n=256)
        X5 = torch.tensor(w5["X0"], dtype=torch.float64, device=dev)
        ctx5 = J.Context(w5["problem"], gmres_m=1, precond="none")
        kernels.update(kernel_rates(J, ctx5, X5, w5["cfl"], int(np.prod(w5["problem"]["shape"])), 5,
                                    args.kernel_reps, prefix="3d256_"))
        ctx5.close()
        del X5

    # ---- the same steps with each elliptic solve replaced by its preconditioning V-cycle
    # (cg_maxit = 0: the paper fixes eta' = 1e-4 and leaves looser inner solves to future
    # work; FGMRES needs the same iterations here) ----------------------------------------
    tuned = None
    if not args.no_tuned:
        print("# tuned: one V-cycle per elliptic solve", file=sys.stderr, flush=True)
        ctx_t = J.Context(pd, precond=precond, jv_mode=jv, ell_precision=args.ell, cg_maxit=0)
        ctx_save = ctx
        ctx = ctx_t
        run_steps(args.warmup)
        torch.cuda.synchronize()
        tt = time.perf_counter()
        Xt, stats_t = run_steps(args.steps)
        torch.cuda.synchronize()
        sec_t = time.perf_counter() - tt
        ctx = ctx_save
        Xk_np, Xt_np = Xk.cpu().numpy(), Xt.cpu().numpy()
        rel = [float(np.max(np.abs(Xt_np[v] - Xk_np[v])) / max(np.max(np.abs(Xk_np[v])), 1e-300))
               for v in range(nvar)]
        tuned = {
            "form": "cg_maxit = 0 (each elliptic solve is one symmetric multigrid V-cycle)",
            "value": args.steps / sec_t, "unit": "implicit steps/s", "ms_per_step": 1e3 * sec_t / args.steps,
            "speedup_vs_plain": sec / sec_t,
            "solver": {"newton_its": sum(s["newton_its"] for s in stats_t),
                       "gmres_its": sum(s["gmres_its"] for s in stats_t),
                       "cg_its": sum(s["cg_its"] for s in stats_t),
                       "converged_steps": sum(s["converged"] for s in stats_t)},
            "max_rel_diff_vs_plain_per_var": rel,
        }
        ctx_t.close()

    compare = None
    if args.compare:
        print("# compare: exact J.v + FP32 elliptic solves", file=sys.stderr, flush=True)
        ctx_ai = J.Context(pd, precond=precond, jv_mode="exact", ell_precision="fp32")
        ctx_save = ctx
        ctx = ctx_ai
        run_steps(args.warmup)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        Xa, stats_a = run_steps(args.steps)
        torch.cuda.synchronize()
        sec_a = time.perf_counter() - ta
        ctx = ctx_save
        Xk_np, Xa_np = Xk.cpu().numpy(), Xa.cpu().numpy()
        rel = [float(np.max(np.abs(Xa_np[v] - Xk_np[v])) / max(np.max(np.abs(Xk_np[v])), 1e-300))
               for v in range(nvar)]
        compare = {
            "form": "exact J.v + FP32 elliptic (MG-CG) solves",
            "value": args.steps / sec_a, "unit": "implicit steps/s",
            "ms_per_step": 1e3 * sec_a / args.steps,
            "speedup_vs_plain": sec / sec_a,
            "solver": {"newton_its": sum(s["newton_its"] for s in stats_a),
                       "gmres_its": sum(s["gmres_its"] for s in stats_a),
                       "cg_its": sum(s["cg_its"] for s in stats_a),
                       "converged_steps": sum(s["converged"] for s in stats_a)},
            "max_rel_diff_vs_plain_per_var": rel,
        }
        ctx_ai.close()

    rec = {
        "metric": METRIC,
        "value": steps_per_s,
        "unit": "implicit steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * sec / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.ell == "fp64" else "f64 (fp32 elliptic solves)",
        "data": "synthetic",
        "config": {"workload": w["name"], "grid": list(pd["shape"]), "cfl_hydro": cfl,
                   "jv": jv, "precond": precond, "elliptic": args.ell, "newton_tol": 1e-8,
                   "gmres": "FGMRES(30)+CGS2, eta 1e-4", "cg_eta": 1e-4},
        "solver": {"newton_its": sum(s["newton_its"] for s in stats),
                   "gmres_its": sum(s["gmres_its"] for s in stats),
                   "cg_its": sum(s["cg_its"] for s in stats),
                   "converged_steps": sum(s["converged"] for s in stats)},
        "roofline": roofline,
        "kernels": kernels,
        "compare": compare,
        "tuned": tuned,
        "probe_ms": {k: round(v[0], 3) for k, v in sorted(probes.items(), key=lambda kv: -kv[1][0])},
    }
    if args.workload == "stratified_2d_kappa" and not args.no_adjoint:
        print("# adjoint run", file=sys.stderr, flush=True)
        rec["adjoint"] = adjoint_run(J, w)
    if not args.no_cpu_baseline:
        rec["cpu_baseline"], rec["error_vs_oracle"] = cpu_baseline(w, args, Xk_first=first_step(ctx, X0, cfl))
    print(json.dumps(rec), flush=True)


def kinetic_energy(Xt, pd):
    """Sum over faces of rho_f u_d^2 / 2 (rho_f the mean of the two cells, mirrored at walls)."""
    import torch
    nd = len(pd["shape"])
    tot = 0.0
    for d in range(nd):
        ax = nd - 1 - d
        rho = Xt[0]
        lower = torch.roll(rho, 1, dims=ax)
        if pd["bc"][d] == "wall":
            idx = [slice(None)] * nd
            idx[ax] = 0
            lower[tuple(idx)] = rho[tuple(idx)]
        tot = tot + 0.5 * torch.sum(0.5 * (lower + rho) * Xt[2 + d] ** 2)
    return tot


def adjoint_run(J, w, directions=8):
    """The adjoint form of the workload: the gradient of the total kinetic energy after the
    workload's implicit steps (fixed time step from X^0) w.r.t. the initial temperature,
    through ImplicitSteps (per-step checkpoints; each backward step is a transposed FGMRES
    solve with the hand-written J^T w and transposed preconditioner), checked against central
    differences of the forward steps along seeded directions (T -> T (1 + eps d) at fixed rho,
    eps = 1e-7).  Tight solver tolerances (Newton 1e-13, GMRES 1e-11, CG 1e-8) make the
    converged steps, and so the difference quotients, accurate enough for the check."""
    import numpy as np
    import torch
    import workloads as Wl
    dev = torch.device("cuda:0")
    pd = w["problem"]
    ctx = J.Context(pd, precond="sound_thermal", jv_mode="exact", newton_tol=1e-13, newton_max=30,
                    gmres_eta=1e-11, gmres_maxit=600, cg_eta=1e-8)
    X0 = torch.tensor(w["X0"], dtype=torch.float64, device=dev)
    dt = ctx.cfl_dt(X0, w["cfl"])
    dts = [dt] * int(w["steps"])
    Xg = X0.clone().requires_grad_(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loss = kinetic_energy(J.ImplicitSteps.apply(Xg, ctx, dts), pd)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    loss.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    grad_e = Xg.grad[1]
    errs = []
    eps = 1e-7
    for k in range(directions):
        d = torch.tensor(Wl.random_vector(w["X0"][1:2], 2001 + k)[0], dtype=torch.float64, device=dev)
        an = float(torch.sum(grad_e * X0[1] * d))  # dL/deps for e -> e (1 + eps d)
        vals = []
        for sgn in (1.0, -1.0):
            Xp = X0.clone()
            Xp[1] = X0[1] * (1.0 + sgn * eps * d)
            for dtk in dts:
                ctx.implicit_step(Xp, dtk)
            vals.append(float(kinetic_energy(Xp, pd)))
        fd = (vals[0] - vals[1]) / (2 * eps)
        errs.append(abs(fd - an) / abs(an))
    ctx.close()
    return {"form": "gradient of total kinetic energy w.r.t. the initial temperature",
            "steps": len(dts), "dt": dt, "forward_ms": 1e3 * (t1 - t0),
            "backward_ms": 1e3 * (t2 - t1), "loss": float(loss.detach()),
            "fd_directions": directions, "fd_eps": eps,
            "fd_max_rel_err": float(np.max(errs)), "fd_rel_errs": [float(e) for e in errs],
            "solver": "exact J.v, sound+thermal preconditioner, Newton 1e-13, GMRES 1e-11, CG 1e-8"}


def first_step(ctx, X0, cfl):
    X = X0.clone()
    dt = ctx.cfl_dt(X, cfl)
    ctx.implicit_step(X, dt)
    return X.cpu().numpy()


def kernel_rates(J, ctx, X0, cfl, N, nvar, reps, prefix):
    """Cell-updates/s and achieved GB/s (algorithmic bytes) of single-launch kernels, timed
    with HIP events on the library's stream."""
    import torch
    dt0 = ctx.cfl_dt(X0, cfl)
    ctx.set_state_n(X0, dt0)
    g = torch.Generator(device=X0.device)
    g.manual_seed(7)
    v = torch.rand(X0.shape, dtype=torch.float64, device=X0.device, generator=g) - 0.5
    out = torch.empty_like(X0)

    def time_call(fn):
        s = ctx.stream
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        fn()
        e0.record(s)
        for _ in range(reps):
            fn()
        e1.record(s)
        e1.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3

    t_res = time_call(lambda: ctx.residual(X0, out))
    t_jex = time_call(lambda: ctx.jvp(X0, v, "exact", out))
    t_jfd = time_call(lambda: ctx.jvp(X0, v, "fd", out))
    t_vjp = time_call(lambda: ctx.vjp(X0, v, out))
    # algorithmic bytes per cell: residual reads X and b and writes F (24 nvar); the exact
    # J.v reads X and v and writes J v (24 nvar); the FD call also evaluates F(X) and two
    # scaled norms (4 kernels); the vjp reads X and w and writes J^T w (24 nvar)
    B = 24.0 * nvar * N
    r = {
        prefix + "cells": N,
        prefix + "residual_cell_updates_per_s": N / t_res,
        prefix + "residual_GBps": B / t_res / 1e9,
        prefix + "residual_hbm_frac": B / t_res / 1e9 / HBM_PEAK_GBS,
        prefix + "jv_exact_cell_updates_per_s": N / t_jex,
        prefix + "jv_exact_GBps": B / t_jex / 1e9,
        prefix + "jv_exact_hbm_frac": B / t_jex / 1e9 / HBM_PEAK_GBS,
        prefix + "jv_fd_call_cell_updates_per_s": N / t_jfd,
        prefix + "vjp_cell_updates_per_s": N / t_vjp,
        prefix + "vjp_GBps": B / t_vjp / 1e9,
    }
    return r


def cpu_baseline(w, args, Xk_first):
    """The CPU oracle (NumPy, one thread) on the first implicit steps of the same workload,
    stopped once args.cpu_budget_s/3 of CPU time is spent (at most 3 steps)."""
    import numpy as np
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    from oracle.newton import jfnk_step, Opts, Stats
    from oracle.residual import Problem, cfl_dt
    from oracle.scaling import scaling_LR
    P = Problem.from_dict(w["problem"])
    X = w["X0"].copy()
    t0 = time.perf_counter()
    steps = 0
    err = None
    while steps < 3:
        dt = cfl_dt(P, X, w["cfl"])
        X = jfnk_step(P, X, dt, Opts(precond=w["precond"], jv_mode=w["jv_mode"], elliptic="pcg"), Stats())
        steps += 1
        if steps == 1:
            _, R = scaling_LR(P, X)
            err = float(np.max(np.abs((Xk_first - X) / R)))
        if time.perf_counter() - t0 > args.cpu_budget_s / 3:
            break
    sec = time.perf_counter() - t0
    try:
        cores_avail = len(os.sched_getaffinity(0))
    except AttributeError:
        cores_avail = os.cpu_count()
    base = {"value": steps / sec, "unit": "implicit steps/s", "cores": 1, "kind": "oracle",
            "sample": f"first {steps} implicit step(s) of {w['name']} from X^0 (NumPy FP64, one "
                      f"thread; {cores_avail} host cores available)",
            "seconds": sec}
    return base, {"first_step_max_abs_Rinv_dX": err}


if __name__ == "__main__":
    main()
