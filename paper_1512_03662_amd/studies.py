"""Iteration-count studies of the paper's test problems, run with this library.

    python -m paper_1512_03662_amd.studies tgv [--steps 10] [--newton-tol 1e-6] [--jv exact]
    python -m paper_1512_03662_amd.studies vortex [--steps 5]
    python -m paper_1512_03662_amd.studies si_vortex [--schemes si_schur,jfnk_be]
    python -m paper_1512_03662_amd.studies eta [--steps 10]

tgv:    the 3D Taylor-Green vortex at 64^3 for the Mach numbers and hydrodynamic CFL numbers
        of the paper's timing table (Results section, Taylor-Green vortex): average Newton
        iterations per time step, GMRES iterations per Newton iteration and elliptic (CG)
        iterations per GMRES iteration, with the paper's figures beside them.
vortex: the 2D isentropic vortex at 64^2 (T_inf = 1, 1e2, 1e6, 1e10, i.e. Mach 1e-1 .. 1e-6)
        over a range of advective CFL numbers, with and without the physics-based
        preconditioner: GMRES iterations per Newton iteration (the paper shows these as a
        figure; no numbers are printed there, so only the trend can be compared).
si_vortex: the semi-implicit stepper's temporal convergence on the same vortex at 64^2
        advected to t = 0.4 (Sect. 3.7): L1, L2 and Linf errors of u against the translated
        initial profile for CFL_adv 0.01 .. 3 and the four Mach numbers, beside the implicit
        JFNK step (backward Euler and Crank-Nicolson) on the same cases.

The paper's runs used its own code (MUSIC with Trilinos), Newton tolerance 1e-6 and an
algebraic-multigrid preconditioned parabolic solver; here Newton tolerance 1e-8, FGMRES(30)
with CGS2, eta = 1e-4, and geometric multigrid CG to 1e-4.  Prints one JSON line per case.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Mach number, CFL_hydro, CFL_adv, Newton/dt, GMRES/Newton, parabolic/GMRES (paper's table)
TGV_TABLE = [
    (1e-1, 7.1e0, 0.5, 3.8, 16.6, 2.4),
    (1e-2, 7.0e1, 0.5, 3.1, 15.4, 2.5),
    (1e-3, 8.2e2, 0.5, 2.7, 16.2, 2.5),
    (1e-4, 1.1e4, 0.5, 2.0, 16.1, 2.8),
    (1e-5, 8.1e4, 0.5, 2.0, 22.2, 2.9),
    (1e-6, 4.9e5, 0.49, 4.5, 291.5, 3.0),
    (1e-6, 5.0e4, 0.05, 2.0, 7.0, 2.8),
]


def _run(ctx, X0, cfl, steps, torch):
    X = X0.clone()
    st = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    err = None
    for _ in range(steps):
        dt = ctx.cfl_dt(X, cfl)
        try:
            st.append(ctx.implicit_step(X, dt, raise_on_noconv=False))
        except Exception as e:  # a failed solve ends the case; it is reported, not hidden
            err = str(e)
            break
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    steps = max(len(st), 1)
    newton = sum(s["newton_its"] for s in st)
    gmres = sum(s["gmres_its"] for s in st)
    cg = sum(s["cg_its"] for s in st)
    return {
        "steps": steps,
        "converged_steps": sum(s["converged"] for s in st),
        "newton_per_step": newton / steps,
        "gmres_per_newton": gmres / max(newton, 1),
        "cg_per_gmres": cg / max(gmres, 1),
        "ms_per_step": 1e3 * sec / steps,
        "error": err,
    }


def tgv(args):
    import torch

    import workloads as W
    import paper_1512_03662_amd as J
    dev = torch.device("cuda:0")
    for mach, cfl, cfl_adv, pn, pg, pp in TGV_TABLE:
        w = W.taylor_green_3d(n=64, mach=mach, noise=0.0)
        X0 = torch.tensor(w["X0"], dtype=torch.float64, device=dev)
        # the hardest row (Mach 1e-6 at CFL_adv 0.49) also with the exact forward-mode J.v:
        # the finite-difference product limits the linear solves there (Sect. 5.1.1)
        forms = ("fd", "exact") if cfl > 1e5 else ("fd",)
        if args.jv != "fd":
            forms = (args.jv,)
        for jv in forms:
            ctx = J.Context(w["problem"], precond="sound", jv_mode=jv, newton_tol=args.newton_tol)
            r = _run(ctx, X0, cfl, args.steps, torch)
            ctx.close()
            r.update({"study": "taylor_green_3d_64^3", "mach": mach, "cfl_hydro": cfl, "jv": jv,
                      "newton_tol": args.newton_tol,
                      "paper": {"cfl_adv": cfl_adv, "newton_per_step": pn, "gmres_per_newton": pg,
                                "parabolic_per_gmres": pp}})
            print(json.dumps(r), flush=True)


def vortex(args):
    import torch

    import workloads as W
    import paper_1512_03662_amd as J
    dev = torch.device("cuda:0")
    for t_inf in (1.0, 1e2, 1e6, 1e10):
        w = W.isentropic_vortex_2d(n=64, t_inf=t_inf)
        pd = w["problem"]
        mach = 0.75 / (2 * math.pi * math.sqrt(1.4 * t_inf))
        h = pd["dx"][0]
        c_inf = math.sqrt(1.4 * t_inf)
        X0 = torch.tensor(w["X0"], dtype=torch.float64, device=dev)
        for cfl_adv in (0.01, 0.05, 0.2, 0.5):
            # CFL_hydro from the advective CFL: dt = cfl_adv dx / u_inf
            cfl = cfl_adv * (1.0 + c_inf + 0.75 / (2 * math.pi))
            for prec in ("sound", "none"):
                ctx = J.Context(pd, precond=prec, jv_mode="fd", gmres_maxit=300,
                                alpha1=1.0 if prec == "none" else 1e-5)
                r = _run(ctx, X0, cfl, args.steps, torch)
                ctx.close()
                r.update({"study": "isentropic_vortex_2d_64^2", "mach": mach, "t_inf": t_inf,
                          "cfl_adv": cfl_adv, "cfl_hydro": cfl, "precond": prec, "dx": h})
                print(json.dumps(r), flush=True)


SI_SCHEMES = {
    # name: (stepper, Context options)
    "si_schur": ("si", dict(precond="sound", pc_schur=1)),
    "si_deltaform": ("si", dict(precond="sound", pc_schur=0)),
    "jfnk_be": ("jfnk", dict(precond="sound", jv_mode="fd")),
    "jfnk_cn": ("jfnk", dict(precond="sound", jv_mode="fd", theta=0.5)),
}


def si_vortex(args):
    """Temporal convergence of the isentropic vortex advected to t = 0.4 (Sect. 3.7): errors of
    u against the translated initial profile for the semi-implicit stepper (both readings of
    its system) and for the implicit JFNK step (backward Euler, Crank-Nicolson)."""
    import numpy as np
    import torch

    import workloads as W
    import paper_1512_03662_amd as J
    dev = torch.device("cuda:0")
    n, t_end = 64, args.t_end
    u_ex = W.isentropic_vortex_u_exact(n=n, t=t_end)
    schemes = args.schemes.split(",")
    for t_inf in (1.0, 1e2, 1e6, 1e10):
        w = W.isentropic_vortex_2d(n=n, t_inf=t_inf)
        mach = 0.75 / (2 * math.pi * math.sqrt(1.4 * t_inf))
        h = w["problem"]["dx"][0]
        for name in schemes:
            kind, kw = SI_SCHEMES[name]
            kw = dict(kw)
            pd = dict(w["problem"], theta=kw.pop("theta", 1.0))
            cfls = tuple(float(c) for c in args.cfls.split(","))
            if kind == "jfnk":
                cfls = tuple(c for c in cfls if c >= 0.05)  # the small steps only repeat the SI's plateau
            for cfl_adv in cfls:
                steps = max(1, int(math.ceil(t_end / (cfl_adv * h) - 1e-9)))
                dt = t_end / steps
                ctx = J.Context(pd, gmres_maxit=300, **kw)
                X = torch.tensor(w["X0"], dtype=torch.float64, device=dev)
                err = None
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                try:
                    for _ in range(steps):
                        if kind == "si":
                            ctx.si_step(X, dt)
                        else:
                            ctx.implicit_step(X, dt)
                except Exception as e:  # an unstable or failed run is reported, not hidden
                    err = str(e)
                torch.cuda.synchronize()
                sec = time.perf_counter() - t0
                ctx.close()
                r = {"study": f"isentropic_vortex_2d_64^2_t{t_end:g}", "scheme": name, "t_inf": t_inf,
                     "mach": mach, "cfl_adv": dt / h, "steps": steps, "ms_per_step": 1e3 * sec / steps,
                     "error": err}
                if err is None:
                    d = X[2].cpu().numpy() - u_ex
                    if np.all(np.isfinite(d)):
                        r.update(L1=float(np.mean(np.abs(d))), L2=float(np.sqrt(np.mean(d * d))),
                                 Linf=float(np.max(np.abs(d))))
                    else:
                        r["error"] = "non-finite state"
                print(json.dumps(r), flush=True)


def eta(args):
    """The parabolic-solve tolerance eta' (the paper fixes 1e-4 and leaves larger values to
    future work): the stratified 2D box 256x256 (bench's default workload, 10 steps at
    CFL_hydro 100, sound + thermal preconditioner, FD J.v) for eta' = 1e-4 .. 1, for one or
    two multigrid-preconditioned CG iterations per elliptic solve, and for the V-cycle alone
    (cg_maxit = 0)."""
    import torch

    import workloads as W
    import paper_1512_03662_amd as J
    dev = torch.device("cuda:0")
    w = W.stratified_2d(n=256)
    X0 = torch.tensor(w["X0"], dtype=torch.float64, device=dev)
    cases = [(1e-4, 50), (1e-3, 50), (1e-2, 50), (1e-1, 50), (1.0, 50), (1e-4, 1), (1e-4, 2), (1e-4, 0)]
    for prec in ("fp64", "fp32"):
        for cg_eta, cg_maxit in cases:
            ctx = J.Context(w["problem"], precond=w["precond"], jv_mode=w["jv_mode"], ell_precision=prec,
                            cg_eta=cg_eta, cg_maxit=cg_maxit)
            r = _run(ctx, X0, w["cfl"], 1, torch)  # warm-up
            r = _run(ctx, X0, w["cfl"], args.steps, torch)
            ctx.close()
            r.update({"study": "stratified_2d_256x256_cg_eta", "ell_precision": prec, "cg_eta": cg_eta,
                      "cg_maxit": cg_maxit, "steps_per_s": 1e3 / r["ms_per_step"]})
            print(json.dumps(r), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("study", choices=["tgv", "vortex", "si_vortex", "eta"])
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--jv", choices=["fd", "exact"], default="fd",
                    help="tgv: J.v form of every row (fd: also the exact form on the hardest row)")
    ap.add_argument("--newton-tol", type=float, default=1e-8,
                    help="tgv: Newton tolerance on ||R^-1 dX||_inf (the paper's runs used 1e-6)")
    ap.add_argument("--schemes", default=",".join(SI_SCHEMES),
                    help="si_vortex: comma-separated subset of " + ",".join(SI_SCHEMES))
    ap.add_argument("--t-end", type=float, default=0.4,
                    help="si_vortex: final time (0.4 in the paper; 8 is one domain crossing)")
    ap.add_argument("--cfls", default="0.01,0.02,0.05,0.1,0.2,0.4,0.8,1.6",
                    help="si_vortex: advective CFL numbers (rounded so that t_end is reached)")
    args = ap.parse_args()
    {"tgv": tgv, "vortex": vortex, "si_vortex": si_vortex, "eta": eta}[args.study](args)


if __name__ == "__main__":
    main()
