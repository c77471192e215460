"""Oracle: the implicit step.

TEST INFRASTRUCTURE ONLY.

Two routes to X^{n+1}, the root of F(X) = 0 (eq. newtimestep):

* ``exact_step`` - the plain definition: Newton with the exact sparse Jacobian (coloured
  complex steps) and a sparse LU solve, iterated until the scaled correction reaches
  roundoff.  This is the reference root for parity of converged steps.
* ``jfnk_step`` - the method of Sect. 4: Newton from X^(0) = X^n (Sect. 4.1), the system
  scaled by L and R (eq. jacobian_system_norm), solved by right-preconditioned flexible
  GMRES to ||L^-1(J dX + F)|| < eta ||L^-1 F|| (eq. forcing_term) with J.v by finite
  differences (eqs. jacobian_free, pert_old) or exactly, the physics-based preconditioner
  (Sect. 4.3), and stopped when ||R^-1 dX||_inf < eps (eq. nr_terminate) with at least two
  iterations (Sect. 4.1).  At most ``newton_max`` iterations (no line search: the paper
  describes none).

Pins (tests/test_oracle_newton_adjoint.py): exact Newton converges quadratically to a residual at
roundoff; linear acoustics through one exact step matches the closed-form amplification of
the discrete wave equation; JFNK reaches the exact root within its tolerance; a uniform state
is a fixed point.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse.linalg as spla

from .jacobian import fd_delta, jacobian_sparse, jvp_cs, H_CS
from .krylov import fgmres
from .mg import PCGSolver
from .pbp import PBP
from .residual import Problem, residual_F, rhs_b
from .scaling import scaling_LR


@dataclass
class Opts:
    newton_tol: float = 1e-8
    newton_max: int = 20
    newton_min: int = 2
    gmres_m: int = 30
    gmres_maxit: int = 300
    gmres_eta: float = 1e-4
    jv_mode: str = "fd"          # 'fd' | 'exact'
    fd_lambda: float = 1e-7
    alpha1: float = 1e-5
    alpha2: float = 1.0
    precond: str = "sound"       # 'none' | 'sound' | 'sound_thermal'
    pc_schur: bool = False       # keep div F_u in the pressure equation (Schur complement)
    elliptic: str = "pcg"        # 'pcg' | 'direct'
    ell_dtype: object = np.float64
    cg_eta: float = 1e-4
    cg_maxit: int = 50
    mg_levels: int = 0           # 0: coarsen as far as the grid allows; L: at most L levels
    mg_smooth: int = 2           # degree of the Chebyshev-Jacobi smoother


@dataclass
class Stats:
    newton_its: int = 0
    gmres_its: list = field(default_factory=list)
    cg_its: list = field(default_factory=list)
    converged: bool = False
    f_norms: list = field(default_factory=list)
    dx_norms: list = field(default_factory=list)


def exact_step(prob: Problem, Xn, dt, tol=1e-14, maxit=12, X0=None):
    """Newton with the exact sparse Jacobian and sparse LU; returns (X, history of
    ||R^-1 dX||_inf)."""
    b = rhs_b(prob, Xn, dt)
    X = (Xn if X0 is None else X0).copy()
    hist = []
    for _ in range(maxit):
        F = residual_F(prob, X, b, dt)
        J = jacobian_sparse(prob, X, b, dt)
        dX = -spla.spsolve(J.tocsc(), F.ravel()).reshape(X.shape)
        _, R = scaling_LR(prob, X)
        X = X + dX
        hist.append(float(np.max(np.abs(dX / R))))
        if hist[-1] < tol:
            break
    return X, hist


def jfnk_step(prob: Problem, Xn, dt, opts: Opts = None, stats: Stats = None):
    """One implicit step by JFNK + PBP; returns X^{n+1}."""
    opts = opts or Opts()
    stats = stats if stats is not None else Stats()
    b = rhs_b(prob, Xn, dt)
    X = Xn.copy()
    for k in range(opts.newton_max):
        F = residual_F(prob, X, b, dt)
        L, R = scaling_LR(prob, X, opts.alpha1, opts.alpha2)
        Fs = F / L
        stats.f_norms.append(float(np.linalg.norm(Fs.ravel())))
        xnorm = float(np.linalg.norm((X / R).ravel()))

        if opts.jv_mode == "fd":
            def apply_op(z, X=X, F=F, L=L, R=R, xnorm=xnorm):
                zn = float(np.linalg.norm((z / R).ravel()))
                if zn == 0.0:
                    return np.zeros_like(z)
                delta = opts.fd_lambda * (opts.fd_lambda + xnorm / zn)
                return (residual_F(prob, X + delta * z, b, dt) - F) / (delta * L)
        else:
            def apply_op(z, X=X, L=L):
                return jvp_cs(prob, X, b, dt, z) / L

        if opts.precond == "none":
            apply_prec = lambda v, R=R: R * v
            solvers = []
        else:
            if opts.elliptic == "direct":
                pbp = PBP(prob, X, dt, opts.precond, schur=opts.pc_schur)
                solvers = []
            else:
                fac_list = []

                def fac(op):
                    s = PCGSolver(op, opts.cg_eta, opts.cg_maxit, opts.ell_dtype, opts.mg_levels, opts.mg_smooth)
                    fac_list.append(s)
                    return s
                pbp = PBP(prob, X, dt, opts.precond, solver_factory=fac, schur=opts.pc_schur)
                solvers = fac_list
            apply_prec = lambda v, L=L, pbp=pbp: pbp.apply(L * v)

        dX, info = fgmres(apply_op, apply_prec, -Fs, opts.gmres_eta, opts.gmres_m,
                          opts.gmres_maxit)
        stats.gmres_its.append(info["iters"])
        stats.cg_its.append(sum(sum(s.iters) for s in solvers))
        X = X + dX
        dxn = float(np.max(np.abs(dX / R)))
        stats.dx_norms.append(dxn)
        stats.newton_its = k + 1
        if dxn < opts.newton_tol and k + 1 >= opts.newton_min:
            stats.converged = True
            break
    return X
