"""Where a central difference of the implicit steps can check the adjoint gradient.

F is piecewise smooth: every upwind choice (sign of a face velocity or mass flux) and
every van Leer limiter choice (sign of the product of two slopes) selects a branch, and the
adjoint differentiates the branch taken at the converged states.  A central difference whose
+eps and -eps trajectories converge to states with other branches somewhere measures the
mean slope across a kink instead.  On the 24^2 stratified box (chi ~ T^3, two steps at
CFL 50) the gradient of the kinetic energy with respect to the initial temperature, along
the seeded direction 2001 (and 2004), is a case with no branch change between the
trajectories at eps = 1e-7: there the difference quotient of the oracle's exact-Newton steps matches the
chain of exact (LU) adjoints to 1e-8.  Along 2002 the trajectories change branches at a few
faces and the two differ by more than 1e-7.  (At eps = 1e-5 every direction changes
several hundred branches and the two differ by 1e-4 to 4e-3.)
"""
import numpy as np
import pytest
import torch

import workloads as W
import oracle.residual as OR
from oracle.adjoint import adjoint_step_exact
from oracle.newton import exact_step
from oracle.residual import Problem, cfl_dt, residual_R

pytestmark = pytest.mark.slow


def _case():
    w_ = W.polytrope((24, 24), 10.0, mach=1e-3, seed=1004, chi_model="power", steps=2, cfl=50.0)
    P = Problem.from_dict(w_["problem"])
    return w_["problem"], P, w_["X0"], cfl_dt(P, w_["X0"], 50.0)


def _ke_np(pd, X):
    tot = 0.0
    for d in range(2):
        ax = 1 - d
        rho = X[0]
        lower = np.roll(rho, 1, axis=ax)
        if pd["bc"][d] == "wall":
            idx = [slice(None)] * 2
            idx[ax] = 0
            lower[tuple(idx)] = rho[tuple(idx)]
        tot += 0.5 * np.sum(0.5 * (lower + rho) * X[2 + d] ** 2)
    return tot


def _ke_grad(pd, X):
    Xt = torch.tensor(X, requires_grad=True)
    tot = 0.0
    for d in range(2):
        ax = 1 - d
        rho = Xt[0]
        lower = torch.roll(rho, 1, dims=ax)
        if pd["bc"][d] == "wall":
            idx = [slice(None)] * 2
            idx[ax] = 0
            lower[tuple(idx)] = rho[tuple(idx)]
        tot = tot + 0.5 * torch.sum(0.5 * (lower + rho) * Xt[2 + d] ** 2)
    tot.backward()
    return Xt.grad.numpy()


def _branches(P, X, monkeypatch_ctx):
    """Every upwind and limiter decision of R(X), in evaluation order."""
    rec = []
    vl0, up0 = OR.vl, OR.upwind

    def vl(a, b):
        rec.append(np.ravel(np.real(a) * np.real(b) > 0).copy())
        return vl0(a, b)

    def upwind(qm2, qm1, q0, qp1, w):
        rec.append(np.ravel(np.broadcast_to(np.real(w) >= 0, np.shape(qm1))).copy())
        return up0(qm2, qm1, q0, qp1, w)

    with monkeypatch_ctx() as m:
        m.setattr(OR, "vl", vl)
        m.setattr(OR, "upwind", upwind)
        residual_R(P, X)
    return np.concatenate(rec)


def _steps(P, X0, dt):
    X1, _ = exact_step(P, X0, dt)
    X2, _ = exact_step(P, X1, dt)
    return X1, X2


def test_fd_gradient_agrees_where_no_branch_changes(monkeypatch):
    pd, P, X0, dt = _case()
    X1, X2 = _steps(P, X0, dt)
    b1 = _branches(P, X1, monkeypatch.context)
    b2 = _branches(P, X2, monkeypatch.context)
    g1, _ = adjoint_step_exact(P, X2, X1, dt, _ke_grad(pd, X2))
    g0, _ = adjoint_step_exact(P, X1, X0, dt, g1)
    eps = 1e-7
    out = {}
    for seed in (2001, 2002):
        d = W.random_vector(X0[1:2], seed)[0]
        an = float(np.sum(g0[1] * X0[1] * d))   # dL/deps for e -> e (1 + eps d)
        vals, changed = [], 0
        for sgn in (1.0, -1.0):
            Xp = X0.copy()
            Xp[1] = X0[1] * (1.0 + sgn * eps * d)
            Y1, Y2 = _steps(P, Xp, dt)
            changed += int(np.sum(_branches(P, Y1, monkeypatch.context) != b1)
                           + np.sum(_branches(P, Y2, monkeypatch.context) != b2))
            vals.append(_ke_np(pd, Y2))
        out[seed] = (changed, abs((vals[0] - vals[1]) / (2 * eps) - an) / abs(an))
    assert out[2001][0] == 0 and out[2001][1] <= 1e-8, out
    assert out[2002][0] > 0 and out[2002][1] > 1e-7, out
