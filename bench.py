"""Benchmark: implicit steps/s of the JFNK + physics-based-preconditioner step on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload convective_box_3d] [--gpus 1]

A step is one implicit time step X^n -> X^{n+1} (CFL time step from X^n, Newton to
||R^-1 dX||_inf < 1e-8, FGMRES(30) with delayed CGS2, physics-based preconditioner with multigrid
CG).  Default workload: the 3D convective box, 256^3 cells (x, y periodic, walls in z,
polytrope n = 1.5 with density contrast 20, conductivity ~ T^3, Mach 1e-4 velocity noise),
CFL_hydro = 500, sound + thermal preconditioner.  `value` is the plain method: FP64
throughout with the finite-difference J.v.  W warm-up steps run from X^0 and are discarded;
then K steps are timed from X^0 (the workload's 10 steps when K = 10).

The same line carries (i) `compare`: the same K steps with the exact forward-mode J.v and
FP32 elliptic solves, and the per-variable difference from the plain run; (ii) the roofline
of the dominant kernel (HIP events attached to every launch of a probe pass over the first
steps); (iii) single-kernel cell-update rates of F, exact and FD J.v and J^T w on X^0;
(iv) the CPU oracle timed on a bounded sample (on the 3D boxes: its residual, FD J.v,
preconditioner and Arnoldi costs on the 64^3 instance of the same recipe, extrapolated to
the full grid and to steps/s with the GPU run's own iteration counts); (v) the agreement of
the GPU's first step with the oracle.  Prints one JSON line.
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
    ap.add_argument("--workload", default="convective_box_3d", choices=sorted(WORKLOADS))
    ap.add_argument("--jv", default=None, choices=["fd", "exact"])
    ap.add_argument("--ell", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--probe-steps", type=int, default=2,
                    help="steps of the probe pass (every launch timed by HIP events)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tuned", action="store_true",
                    help="also time the steps with one V-cycle per elliptic solve")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="stratified_2d_kappa: skip the adjoint run (gradient through the steps, FD-checked)")
    ap.add_argument("--no-kernels-3d", dest="kernels_3d", action="store_false",
                    help="2D workloads: skip the kernel rates at the 256^3 production size")
    ap.add_argument("--only-kernels-3d", action="store_true",
                    help="only time the single-launch kernels at 256^3 (for profiling them)")
    ap.add_argument("--no-compare", dest="compare", action="store_false",
                    help="skip the exact-J.v + FP32-elliptic form of the same steps")
    ap.add_argument("--no-oracle-check", dest="oracle_check", action="store_false",
                    help="skip the comparison of the first step with the oracle")
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
    taken.  The summary's machine-readable part holds one block per kernel family, each
    opened by a `kernel:` line."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload_name}.txt")
    if not os.path.exists(path):
        return None
    blocks, cur = {}, None
    with open(path) as f:
        for line in f:
            if line.startswith("#") or ":" not in line:
                continue
            k, v = (t.strip() for t in line.split(":", 1))
            if k == "kernel":
                cur = blocks.setdefault(v, {})
            elif cur is not None:
                cur[k] = v
    kv = blocks.get(kernel)
    if kv is None:
        return None
    try:
        if source_sha256(kv["source"]) != kv["source_sha256"]:
            return None
        return 1024.0 * (float(kv["fetch_kib_per_launch"]) * float(kv["fetch_calibration"])
                         + float(kv["write_kib_per_launch"]) * float(kv["write_calibration"]))
    except (KeyError, ValueError, OSError):
        return None


def workload(name):
    import workloads as W
    w = W.CONFIGS[name]()
    return w


def solver_totals(stats):
    return {"newton_its": sum(s["newton_its"] for s in stats),
            "gmres_its": sum(s["gmres_its"] for s in stats),
            "cg_its": sum(s["cg_its"] for s in stats),
            "converged_steps": sum(s["converged"] for s in stats)}


def rel_diff_per_var(A, B):
    """max |A_v - B_v| / max |B_v| per variable (host arrays)."""
    import numpy as np
    return [float(np.max(np.abs(A[v] - B[v])) / max(float(np.max(np.abs(B[v]))), 1e-300))
            for v in range(A.shape[0])]


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU only (asked for --gpus {args.gpus}); "
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
    large = N > (1 << 20)  # the oracle cannot step these grids within the bench's budget
    cfl = w["cfl"]

    def run_steps(ctx, k, keep_first=False):
        X = X0.clone()
        stats = []
        first = None
        for i in range(k):
            dt = ctx.cfl_dt(X, cfl)
            stats.append(ctx.implicit_step(X, dt))
            if keep_first and i == 0:
                first = (X.clone(), dt)
        return X, stats, first

    def timed_form(ctx, label):
        """W warm-up steps (the first one kept as the form's first step), then K timed steps."""
        print(f"# {label}: warm-up {args.warmup} step(s)", file=sys.stderr, flush=True)
        _, _, first = run_steps(ctx, args.warmup, keep_first=True)
        torch.cuda.synchronize()
        print(f"# {label}: timing {args.steps} step(s)", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        Xk, stats, _ = run_steps(ctx, args.steps)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        if first is None:
            _, _, first = run_steps(ctx, 1, keep_first=True)
        print(f"# {label}: {args.steps / sec:.4g} steps/s", file=sys.stderr, flush=True)
        return Xk, stats, sec, first

    ctx = J.Context(pd, precond=precond, jv_mode=jv, ell_precision=args.ell)
    Xk, stats, sec, first_plain = timed_form(ctx, f"{w['name']} plain ({jv} J.v, {args.ell} elliptic)")
    steps_per_s = args.steps / sec

    # ---- probe pass: the first steps again with every kernel launch timed by HIP events ----
    pk = max(1, min(args.probe_steps, args.steps))
    print(f"# probe pass ({pk} step(s))", file=sys.stderr, flush=True)
    from paper_1512_03662_amd import _native as Nat
    Nat.probe_enable(True)
    ctx.set_opts(phase_timing=1)
    _, stats_probe, _ = run_steps(ctx, pk)
    ctx.set_opts(phase_timing=0)
    torch.cuda.synchronize()
    probes = Nat.probe_results()
    Nat.probe_enable(False)
    phase_ms = {k: sum(s[k] for s in stats_probe) / pk for k in ("t_resid", "t_jv", "t_prec", "t_orth")}
    dom = max(probes.items(), key=lambda kv: kv[1][0])
    dom_name, (dom_ms, dom_n, dom_bytes) = dom
    avg_s = dom_ms * 1e-3 / dom_n
    achieved = dom_bytes / dom_n / avg_s / 1e9
    traffic = measured_traffic(w["name"], dom_name)
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": dom_name,
                "launches": dom_n, "avg_us": avg_s * 1e6, "probe_steps": pk,
                "algorithmic_bytes_per_launch": dom_bytes / dom_n,
                "share_of_kernel_time": dom_ms / sum(v[0] for v in probes.values())}

    # ---- kernel rates: residual, exact and FD J.v, vjp on X^0 of this workload -------------
    print("# single-kernel rates", file=sys.stderr, flush=True)
    kernels = kernel_rates(J, ctx, X0, cfl, N, nvar, args.kernel_reps, prefix="")
    ctx_keep = ctx
    # 2D workloads: also at the full 3D production size (256^3 convective box, 5 variables)
    if args.kernels_3d and len(pd["shape"]) == 2:
        import workloads as Wl
        w5 = Wl.convective_box_3d(n=256)
        X5 = torch.tensor(w5["X0"], dtype=torch.float64, device=dev)
        ctx5 = J.Context(w5["problem"], gmres_m=1, precond="none")
        kernels.update(kernel_rates(J, ctx5, X5, w5["cfl"], int(np.prod(w5["problem"]["shape"])), 5,
                                    args.kernel_reps, prefix="3d256_"))
        ctx5.close()
        del X5

    # ---- the same steps with exact J.v and FP32 elliptic solves ----------------------------
    compare = None
    first_ai = None
    if args.compare:
        ctx_ai = J.Context(pd, precond=precond, jv_mode="exact", ell_precision="fp32")
        Xa, stats_a, sec_a, first_ai = timed_form(ctx_ai, "exact J.v + FP32 elliptic")
        print(f"# exact J.v + FP32 elliptic: probe pass ({pk} step(s))", file=sys.stderr, flush=True)
        Nat.probe_enable(True)
        ctx_ai.set_opts(phase_timing=1)
        _, stats_ap, _ = run_steps(ctx_ai, pk)
        torch.cuda.synchronize()
        probes_a = Nat.probe_results()
        Nat.probe_enable(False)
        dom_a, (dms_a, dn_a, db_a) = max(probes_a.items(), key=lambda kv: kv[1][0])
        compare = {
            "form": "exact J.v + FP32 elliptic (MG-CG) solves",
            "value": args.steps / sec_a, "unit": "implicit steps/s",
            "ms_per_step": 1e3 * sec_a / args.steps,
            "speedup_vs_plain": sec / sec_a,
            "solver": solver_totals(stats_a),
            "max_rel_diff_vs_plain_per_var": rel_diff_per_var(Xa.cpu().numpy(), Xk.cpu().numpy()),
            "first_step_max_rel_diff_vs_plain_per_var": rel_diff_per_var(first_ai[0].cpu().numpy(),
                                                                         first_plain[0].cpu().numpy()),
            "dominant_kernel": {"kernel": dom_a, "launches": dn_a, "avg_us": 1e3 * dms_a / dn_a,
                                "achieved_GBps": db_a / (dms_a * 1e-3) / 1e9,
                                "frac_of_hbm_peak": db_a / (dms_a * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                "share_of_kernel_time": dms_a / sum(v[0] for v in probes_a.values())},
            "probe_ms": {k: round(v[0], 3) for k, v in sorted(probes_a.items(), key=lambda kv: -kv[1][0])},
            "phase_ms_per_step": {k: sum(s[k] for s in stats_ap) / pk for k in ("t_resid", "t_jv", "t_prec", "t_orth")},
        }
        ctx_ai.close()
        del Xa

    # ---- the same steps with each elliptic solve replaced by its preconditioning V-cycle
    # (cg_maxit = 0: the paper fixes eta' = 1e-4 and leaves looser inner solves to future
    # work) ---------------------------------------------------------------------------------
    tuned = None
    if args.tuned:
        ctx_t = J.Context(pd, precond=precond, jv_mode=jv, ell_precision=args.ell, cg_maxit=0)
        Xt, stats_t, sec_t, _ = timed_form(ctx_t, "one V-cycle per elliptic solve")
        tuned = {
            "form": "cg_maxit = 0 (each elliptic solve is one symmetric multigrid V-cycle)",
            "value": args.steps / sec_t, "unit": "implicit steps/s", "ms_per_step": 1e3 * sec_t / args.steps,
            "speedup_vs_plain": sec / sec_t,
            "solver": solver_totals(stats_t),
            "max_rel_diff_vs_plain_per_var": rel_diff_per_var(Xt.cpu().numpy(), Xk.cpu().numpy()),
        }
        ctx_t.close()
        del Xt

    ctx = ctx_keep
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
                   "gmres": "FGMRES(30), delayed CGS2, eta 1e-4", "cg_eta": 1e-4},
        "solver": solver_totals(stats),
        "roofline": roofline,
        "kernels": kernels,
        "compare": compare,
        "tuned": tuned,
        "probe_ms": {k: round(v[0], 3) for k, v in sorted(probes.items(), key=lambda kv: -kv[1][0])},
        "phase_ms_per_step": phase_ms,
    }
    if args.workload == "stratified_2d_kappa" and not args.no_adjoint:
        print("# adjoint run", file=sys.stderr, flush=True)
        rec["adjoint"] = adjoint_run(J, w)
    if args.oracle_check:
        print("# first step against the oracle", file=sys.stderr, flush=True)
        if large:
            chk = {"plain": sampled_root_check(ctx, w, X0, first_plain)}
            if first_ai is not None:
                chk["exact_fp32"] = sampled_root_check(ctx, w, X0, first_ai)
            rec["error_vs_oracle"] = chk
        else:
            rec["error_vs_oracle"] = oracle_first_step(w, first_plain, first_ai)
    if not args.no_cpu_baseline:
        print("# CPU oracle baseline", file=sys.stderr, flush=True)
        if large:
            rec["cpu_baseline"] = cpu_baseline_extrapolated(w, stats, args)
        else:
            rec["cpu_baseline"] = cpu_baseline(w, args)
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
        prefix + "vjp_hbm_frac": B / t_vjp / 1e9 / HBM_PEAK_GBS,
    }
    return r


def _blas_threads():
    from threadpoolctl import threadpool_info
    return sorted({int(i["num_threads"]) for i in threadpool_info()}) or [1]


def _host_cores():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count()


def oracle_opts(w):
    from oracle.newton import Opts
    return Opts(precond=w["precond"], jv_mode=w["jv_mode"], elliptic="pcg")


def cpu_baseline(w, args):
    """The CPU oracle's own implicit steps (NumPy FP64, BLAS held to one thread) on the first
    steps of the same workload, stopped once args.cpu_budget_s/3 of time is spent (at most
    3 steps)."""
    from threadpoolctl import threadpool_limits
    from oracle.newton import jfnk_step, Stats
    from oracle.residual import Problem, cfl_dt
    P = Problem.from_dict(w["problem"])
    with threadpool_limits(1):
        threads = _blas_threads()
        X = w["X0"].copy()
        t0 = time.perf_counter()
        steps = 0
        while steps < 3:
            dt = cfl_dt(P, X, w["cfl"])
            X = jfnk_step(P, X, dt, oracle_opts(w), Stats())
            steps += 1
            if time.perf_counter() - t0 > args.cpu_budget_s / 3:
                break
        sec = time.perf_counter() - t0
    return {"value": steps / sec, "unit": "implicit steps/s", "cores": max(threads), "kind": "oracle",
            "sample": f"first {steps} implicit step(s) of {w['name']} from X^0 (NumPy FP64; BLAS "
                      f"threads {threads}; {_host_cores()} host cores available)",
            "seconds": sec}


def oracle_first_step(w, first_plain, first_ai):
    """The GPU's first step against the oracle's JFNK step from the same X^0 and dt:
    max |R^-1 (X_gpu - X_oracle)| (R at the oracle's state) and per-variable relative
    differences, for the plain form and (if run) the exact-J.v + FP32 form."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle.newton import jfnk_step, Stats
    from oracle.residual import Problem
    from oracle.scaling import scaling_LR
    P = Problem.from_dict(w["problem"])
    X1g, dt = first_plain
    with threadpool_limits(1):
        Xo = jfnk_step(P, w["X0"].copy(), dt, oracle_opts(w), Stats())
    _, R = scaling_LR(P, Xo)
    out = {}
    for name, f in (("plain", first_plain), ("exact_fp32", first_ai)):
        if f is None:
            continue
        Xg = f[0].cpu().numpy()
        out[name] = {"first_step_max_abs_Rinv_dX": float(np.max(np.abs((Xg - Xo) / R))),
                     "max_rel_diff_per_var": rel_diff_per_var(Xg, Xo)}
    return out


def sampled_root_check(ctx, w, X0, first, ncells=4096, seed=77):
    """The first step on a grid too large for the oracle's solver: at seeded cells, the
    oracle's F (U/dt - theta R - b, b from X^0) at the GPU's X^1 against the library's F there
    (operator parity), and its size (how closely X^1 is a root of the oracle's F), both
    divided per variable by S_k = max(|U_k|/dt + |b_k|) + max A_k over the sampled cells
    (A_k: the sum of the absolute values of the terms of R_k)."""
    import numpy as np
    from oracle.residual import Problem, conserved_U, residual_R
    P = Problem.from_dict(w["problem"])
    X1, dt = first
    ctx.set_state_n(X0, dt)
    Fg = ctx.residual(X1).cpu().numpy()
    X1n = X1.cpu().numpy()
    X0n = w["X0"]
    rng = np.random.default_rng(seed)
    cells = tuple(rng.integers(0, n, ncells) for n in P.shape)
    b = conserved_U(P, X0n, cells) / dt
    if P.theta != 1.0:
        b = b + (1.0 - P.theta) * residual_R(P, X0n, cells)
    U1 = conserved_U(P, X1n, cells)
    R1, A1 = residual_R(P, X1n, cells, with_abs=True)
    Fo = U1 / dt - P.theta * R1 - b
    idx = tuple(cells[d] for d in reversed(range(P.nd)))
    Fgs = np.stack([Fg[k][idx] for k in range(P.nvar)])
    S = np.max(np.abs(U1) / dt + np.abs(b), axis=1) + np.max(A1, axis=1)
    return {"cells": ncells,
            "F_gpu_vs_oracle_max_rel": float(np.max(np.max(np.abs(Fgs - Fo), axis=1) / S)),
            "oracle_F_at_gpu_state_max_rel": float(np.max(np.max(np.abs(Fo), axis=1) / S))}


def cpu_baseline_extrapolated(w, stats, args, sample_n=64):
    """The CPU oracle on a grid too large for it to step within the bench: its per-call costs
    on the sample_n^3 instance of the same recipe (NumPy FP64, BLAS held to one thread), each
    timed once, scaled by the cell count to the full grid and combined with the GPU run's own
    iteration counts per step:

        t_step = newton * (t_F + t_pc_setup) + gmres * (t_Jv + t_pc_apply + t_arnoldi),

    t_F the residual with its scalings, t_Jv the finite-difference product, t_pc_setup the
    preconditioner's operators and multigrid hierarchy, t_pc_apply one preconditioner
    application corrected to the GPU's mean CG iterations per GMRES iteration with the
    oracle's own cost per CG iteration, t_arnoldi the oracle FGMRES's cost per iteration at
    the GPU's mean Krylov depth (a cheap diagonal operator, identity preconditioner)."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    import workloads as Wl
    from oracle.jacobian import jvp_fd
    from oracle.krylov import fgmres
    from oracle.mg import PCGSolver, pcg
    from oracle.pbp import PBP
    from oracle.residual import Problem, cfl_dt, residual_F, rhs_b
    from oracle.scaling import scaling_LR

    def tm(f):
        t = time.perf_counter()
        r = f()
        return time.perf_counter() - t, r

    gen = {"convective_box_3d": Wl.convective_box_3d, "taylor_green_3d": Wl.taylor_green_3d}
    name = args.workload
    K = len(stats)
    newton = sum(s["newton_its"] for s in stats) / K
    gmres = sum(s["gmres_its"] for s in stats) / K
    cg = sum(s["cg_its"] for s in stats) / K
    t_all = time.perf_counter()
    with threadpool_limits(1):
        threads = _blas_threads()
        ws = gen[name](n=sample_n)
        P = Problem.from_dict(ws["problem"])
        X = ws["X0"]
        dt = cfl_dt(P, X, ws["cfl"])
        b = rhs_b(P, X, dt)
        tF, (F, (L, R)) = tm(lambda: (residual_F(P, X, b, dt), scaling_LR(P, X)))
        v = Wl.random_vector(X, 7, bc=P.bc)
        tJ, _ = tm(lambda: jvp_fd(P, X, b, dt, v, F0=F) / L)
        comp = {"residual_and_scalings": tF, "fd_jv": tJ}
        if ws["precond"] != "none":
            sols = []

            def fac(op):
                s = PCGSolver(op, 1e-4, 50)
                sols.append(s)
                return s
            tS, pbp = tm(lambda: PBP(P, X, dt, ws["precond"], solver_factory=fac))
            r = Wl.random_vector(X, 8, bc=P.bc) * L
            tA, _ = tm(lambda: pbp.apply(r))
            kA = sum(sum(s.iters) for s in sols)
            rhs = np.random.default_rng(9).uniform(-1.0, 1.0, X[0].shape)
            t1, _ = tm(lambda: pcg(sols[0].op, rhs, eta=0.0, maxit=1, mg=sols[0].mg))
            t4, _ = tm(lambda: pcg(sols[0].op, rhs, eta=0.0, maxit=4, mg=sols[0].mg))
            tcg = max(t4 - t1, 0.0) / 3.0
            cg_per_gmres = cg / max(gmres, 1e-300)
            tA_adj = max(tA + (cg_per_gmres - kA) * tcg, 0.0)
            comp.update({"pc_setup": tS, "pc_apply": tA, "pc_apply_cg_its": kA,
                         "cg_iteration": tcg, "pc_apply_at_gpu_cg_count": tA_adj})
        else:
            tS = tA_adj = 0.0
        jbar = int(min(30, max(1, round(gmres / max(newton, 1e-300)))))
        D = 1.0 + np.random.default_rng(10).uniform(0.0, 1.0, X.shape)
        tO, _ = tm(lambda: fgmres(lambda z: D * z, lambda q: q, F / L, eta=1e-300, m=30, maxit=jbar))
        tO /= jbar
        comp["arnoldi_per_iteration"] = tO
    scale = float(np.prod(w["problem"]["shape"])) / float(np.prod(ws["problem"]["shape"]))
    t_step = scale * (newton * (tF + tS) + gmres * (tJ + tA_adj + tO))
    return {"value": 1.0 / t_step, "unit": "implicit steps/s", "cores": max(threads), "kind": "oracle",
            "extrapolated": True,
            "sample": (f"oracle per-call costs on the {sample_n}^3 instance of the same recipe "
                       f"(NumPy FP64, BLAS threads {threads}, {_host_cores()} host cores available), "
                       f"scaled x{scale:.0f} in cells and combined with the GPU run's counts per step "
                       f"(Newton {newton:.2f}, GMRES {gmres:.1f}, CG {cg:.1f}; Krylov depth {jbar})"),
            "seconds_per_step": t_step, "components_s_at_sample": comp,
            "seconds": time.perf_counter() - t_all}


if __name__ == "__main__":
    main()
