"""Oracle: vector-Jacobian products and the adjoint of one implicit step.

TEST INFRASTRUCTURE ONLY.

For the step F(X^{n+1}; X^n) = 0 with F = U(X)/dt - theta R(X) - U(X^n)/dt - (1-theta) R(X^n)
(eq. crank_nicholson, theta-weighted) and a loss L(X^{n+1}), the implicit-function theorem
gives dL/dX^n = -(dF/dX^n)^T lam with J^T lam = dL/dX^{n+1}, J = dF/dX^{n+1}, i.e.
dL/dX^n = (dU/dX|_{X^n})^T lam / dt + (1 - theta) (dR/dX|_{X^n})^T lam.

* ``vjp_sparse``   J^T w from the coloured complex-step Jacobian (exact, frozen branches).
* ``dU_dX_T``      (dU/dX)^T lam written out from U = (rho, rho e, rho_f u_d).
* ``adjoint_step_exact``  lam by a sparse LU solve of J^T (the plain definition).
* ``adjoint_step_fgmres`` the same by FGMRES on the scaled transposed system
  (R J^T L^-1)(L lam) = R g with the transposed physics-based preconditioner
  L M^-T R^-1 on the right, mirroring the forward solver.

Pins (tests/test_oracle_newton_adjoint.py): dot-product tests <w, J v> = <J^T w, v> with the
complex-step J.v; dU_dX_T against complex steps of U; the step adjoint against central
finite differences of whole exact steps; FGMRES adjoint against the LU adjoint.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse.linalg as spla

from .jacobian import jacobian_sparse
from .krylov import fgmres
from .mg import PCGSolver
from .pbp import PBP, _roll, _wall_slice
from .residual import Problem, WALL, rhs_b
from .scaling import scaling_LR


def vjp_sparse(prob: Problem, X, b, dt, w, J=None):
    if J is None:
        J = jacobian_sparse(prob, X, b, dt)
    return (J.T @ w.ravel()).reshape(X.shape)


def dU_dX_T(prob: Problem, X, lam):
    out = np.zeros_like(X)
    rho, e = X[0], X[1]
    out[0] = lam[0] + e * lam[1]
    out[1] = rho * lam[1]
    for d in range(prob.nd):
        lower = _roll(rho, prob, d, -1)
        if prob.bc[d] == WALL:
            lower[_wall_slice(prob, d, 0)] = rho[_wall_slice(prob, d, 0)]
        rf = 0.5 * (lower + rho)
        out[2 + d] = rf * lam[2 + d]
        a = 0.5 * X[2 + d] * lam[2 + d]   # d(U_m)/d(rho[c-1]) = d(U_m)/d(rho[c]) = u/2
        up = _roll(a, prob, d, 1)
        if prob.bc[d] == WALL:
            up[_wall_slice(prob, d, -1)] = 0.0
            extra = np.zeros_like(a)
            extra[_wall_slice(prob, d, 0)] = a[_wall_slice(prob, d, 0)]
            out[0] += a + up + extra
        else:
            out[0] += a + up
    return out


def dXn_T(prob: Problem, Xn, dt, lam):
    """-(dF/dX^n)^T lam = (dU/dX)^T lam / dt + (1 - theta) (dR/dX)^T lam at X^n."""
    out = dU_dX_T(prob, Xn, lam) / dt
    if prob.theta != 1.0:
        # dR/dX from the complex-step Jacobian of the backward-Euler residual at X^n:
        # J1 = dU/dX / dt - dR/dX, so (dR/dX)^T lam = (dU/dX)^T lam / dt - J1^T lam
        p1 = dataclasses.replace(prob, theta=1.0)
        J1 = jacobian_sparse(p1, Xn, np.zeros_like(Xn), dt)
        dRT = dU_dX_T(prob, Xn, lam) / dt - (J1.T @ lam.ravel()).reshape(lam.shape)
        out = out + (1.0 - prob.theta) * dRT
    return out


def adjoint_step_exact(prob: Problem, Xn1, Xn, dt, gbar):
    b = rhs_b(prob, Xn, dt)
    J = jacobian_sparse(prob, Xn1, b, dt)
    lam = spla.spsolve(J.T.tocsc(), gbar.ravel()).reshape(Xn1.shape)
    return dXn_T(prob, Xn, dt, lam), lam


def adjoint_step_fgmres(prob: Problem, Xn1, Xn, dt, gbar, precond="sound", eta=1e-10,
                        m=30, maxit=300, alpha1=1e-5, alpha2=1.0, elliptic="direct",
                        cg_eta=1e-4, info_out=None, schur=False):
    b = rhs_b(prob, Xn, dt)
    J = jacobian_sparse(prob, Xn1, b, dt)
    L, R = scaling_LR(prob, Xn1, alpha1, alpha2)
    apply_op = lambda Z: R * (J.T @ Z.ravel()).reshape(Z.shape)
    if precond == "none":
        apply_prec = lambda v: v / L
    else:
        fac = None if elliptic == "direct" else PCGSolver.factory(cg_eta)
        pbp = PBP(prob, Xn1, dt, precond, solver_factory=fac, schur=schur)
        apply_prec = lambda v: pbp.apply_T(v / R)
    lam, info = fgmres(apply_op, apply_prec, R * gbar, eta, m, maxit)
    if info_out is not None:
        info_out.update(info)
    return dXn_T(prob, Xn, dt, lam), lam
