"""Pins of the oracle implicit step (Sect. 4) and its adjoint.

* exact Newton converges quadratically to roundoff;
* linear acoustics: one theta-step (backward Euler, Crank-Nicolson, theta = 3/4) of a
  standing sound wave scales it by the closed form of the discrete wave equation (Sect. 3.3.1
  derives the wave equation a^2 = Gamma1 p/rho; eq. crank_nicholson the theta-weighting);
* hydrostatic equilibrium survives a large step;
* JFNK + PBP (Sect. 4) reaches the exact root within its tolerance;
* the adjoint step matches central differences of whole exact steps.
"""
import numpy as np
import pytest

import workloads as W
from oracle.residual import Problem, residual_F, rhs_b, cfl_dt, conserved_U
from oracle.jacobian import jvp_cs
from oracle.newton import exact_step, jfnk_step, Opts, Stats
from oracle.scaling import scaling_LR
from oracle.adjoint import (vjp_sparse, dU_dX_T, adjoint_step_exact, adjoint_step_fgmres)


def test_exact_newton_quadratic():
    w = W.acoustic_bump_2d(n=16)
    P = Problem.from_dict(w["problem"])
    X0 = w["X0"]
    dt = cfl_dt(P, X0, 10.0)
    X, hist = exact_step(P, X0, dt)
    assert hist[-1] < 1e-14
    # quadratic phase: once below 1e-4 the next correction is far smaller than linear
    k = next(i for i, h in enumerate(hist) if h < 1e-4)
    if k + 1 < len(hist) and hist[k + 1] > 1e-15:
        assert hist[k + 1] < 10 * hist[k] ** 1.8
    F = residual_F(P, X, rhs_b(P, X0, dt), dt)
    assert np.max(np.abs(F)) < 1e-10


ACOUSTIC_CASES = [(shape, modes, cfl, theta)
                  for shape, modes, cfl in [((16, 16), (1, 2), 1.0), ((16, 16), (2, 1), 30.0)]
                  for theta in (1.0, 0.5, 0.75)] + [((8, 8, 8), (1, 1, 2), 100.0, 0.5)]


@pytest.mark.parametrize("shape,modes,cfl,theta", ACOUSTIC_CASES)
def test_linear_acoustics_theta_step(shape, modes, cfl, theta):
    """A standing wave at rest is the sum of the two modes exp(+-i w t); one theta-step maps
    each by g = (1 + i(1-theta) w dt)/(1 - i theta w dt), so the pressure amplitude scales by
    Re g = (1 - theta(1-theta) w^2 dt^2)/(1 + theta^2 w^2 dt^2): 1/(1 + w^2 dt^2) for
    backward Euler, (1 - w^2 dt^2/4)/(1 + w^2 dt^2/4) for Crank-Nicolson."""
    nd = len(shape)
    gamma, p0, rho0, A = 1.4, 1.0, 1.0, 1e-6
    L = 1.0
    h = L / shape[0]
    gs = W.grid_shape(shape)
    grids = np.meshgrid(*[(np.arange(n) + 0.5) * h for n in gs], indexing="ij")
    pos = [grids[nd - 1 - d] for d in range(nd)]
    k = [2 * np.pi * modes[d] / L for d in range(nd)]
    phase = sum(k[d] * pos[d] for d in range(nd))
    p = p0 + A * np.cos(phase)
    rho = rho0 * (p / p0) ** (1 / gamma)
    X = np.zeros((2 + nd,) + gs)
    X[0] = rho
    X[1] = p / ((gamma - 1) * rho)
    pd = W.make_problem(shape, (h,) * nd, ("periodic",) * nd, gamma, theta=theta)
    P = Problem.from_dict(pd)
    c = np.sqrt(gamma * p0 / rho0)
    dt = cfl * h / c
    Xn1, hist = exact_step(P, X, dt)
    pn1 = (gamma - 1) * Xn1[0] * Xn1[1] - p0
    basis = np.cos(phase)
    ratio = np.sum(pn1 * basis) / np.sum((p - p0) * basis)
    w2 = c ** 2 * sum((2 / h) ** 2 * np.sin(k[d] * h / 2) ** 2 for d in range(nd))
    expect = (1 - theta * (1 - theta) * w2 * dt ** 2) / (1 + theta ** 2 * w2 * dt ** 2)
    assert abs(ratio - expect) <= 1e-5 * max(abs(expect), 1e-3), (ratio, expect)


def test_hydrostatic_equilibrium_survives_step():
    w = W.polytrope((8, 16), 10.0, mach=0.0, chi_model="const", steps=1)
    P = Problem.from_dict(w["problem"])
    X0 = w["X0"]
    dt = cfl_dt(P, X0, 100.0)
    X, hist = exact_step(P, X0, dt)
    cs = np.sqrt(P.gamma * (P.gamma - 1) * X[1])
    assert np.max(np.abs(X[2:])) / cs.min() <= 1e-13


def test_uniform_state_fixed_point_jfnk():
    shape = (8, 8)
    X = np.zeros((4, 8, 8))
    X[0], X[1], X[2], X[3] = 1.2, 2.0, 0.3, -0.2
    P = Problem.from_dict(W.make_problem(shape, (0.125, 0.125), ("periodic",) * 2, 1.4))
    st = Stats()
    Xn1 = jfnk_step(P, X, 0.5, Opts(), st)
    assert np.array_equal(Xn1, X) and st.converged and st.newton_its == 2


@pytest.mark.parametrize("jv", ["fd", "exact"])
@pytest.mark.parametrize("elliptic", ["direct", "pcg"])
def test_jfnk_reaches_exact_root_bump(jv, elliptic):
    w = W.acoustic_bump_2d(n=16)
    P = Problem.from_dict(w["problem"])
    X0 = w["X0"]
    dt = cfl_dt(P, X0, 10.0)
    Xs, _ = exact_step(P, X0, dt)
    st = Stats()
    X = jfnk_step(P, X0, dt, Opts(jv_mode=jv, elliptic=elliptic, precond="sound"), st)
    _, R = scaling_LR(P, Xs)
    assert st.converged
    assert np.max(np.abs((X - Xs) / R)) <= 1e-9
    assert max(st.gmres_its) <= 20


@pytest.mark.parametrize("precond", ["sound", "sound_thermal"])
def test_jfnk_crank_nicolson(precond):
    """theta = 1/2: the preconditioner built with tau = dt/2 and scaled by 2 keeps GMRES as
    short as for backward Euler, and the step reaches the exact root."""
    w = W.polytrope((16, 16), 10.0, mach=1e-3, seed=5, chi_model="power", steps=1, cfl=50.0)
    pd = dict(w["problem"])
    pd["theta"] = 0.5
    P = Problem.from_dict(pd)
    X0 = w["X0"]
    dt = cfl_dt(P, X0, 50.0)
    Xs, _ = exact_step(P, X0, dt)
    st = Stats()
    X = jfnk_step(P, X0, dt, Opts(precond=precond, elliptic="direct"), st)
    _, R = scaling_LR(P, Xs)
    assert st.converged
    assert np.max(np.abs((X - Xs) / R)) <= 1e-9
    # the same step without the theta weighting of the preconditioner needs more iterations
    import oracle.pbp as pbp_mod
    st1 = Stats()
    orig = pbp_mod.PBP.__init__
    def unweighted(self, prob, X, dt, mode="sound", solver_factory=None, **kw):
        import dataclasses
        orig(self, dataclasses.replace(prob, theta=1.0), X, dt, mode, solver_factory, **kw)
    pbp_mod.PBP.__init__ = unweighted
    try:
        jfnk_step(P, X0, dt, Opts(precond=precond, elliptic="direct"), st1)
    finally:
        pbp_mod.PBP.__init__ = orig
    assert sum(st.gmres_its) < sum(st1.gmres_its)


def test_jfnk_stratified_thermal():
    w = W.polytrope((16, 16), 10.0, mach=1e-3, seed=5, chi_model="power", steps=1, cfl=50.0)
    P = Problem.from_dict(w["problem"])
    X0 = w["X0"]
    dt = cfl_dt(P, X0, 50.0)
    Xs, _ = exact_step(P, X0, dt)
    st = Stats()
    X = jfnk_step(P, X0, dt, Opts(precond="sound_thermal", elliptic="pcg"), st)
    _, R = scaling_LR(P, Xs)
    assert st.converged
    assert np.max(np.abs((X - Xs) / R)) <= 1e-9


def test_unpreconditioned_needs_more_iterations():
    w = W.acoustic_bump_2d(n=16)
    P = Problem.from_dict(w["problem"])
    X0 = w["X0"]
    dt = cfl_dt(P, X0, 10.0)
    s1, s2 = Stats(), Stats()
    jfnk_step(P, X0, dt, Opts(precond="sound", elliptic="direct"), s1)
    jfnk_step(P, X0, dt, Opts(precond="none", alpha1=1.0), s2)
    assert sum(s2.gmres_its) > 2 * sum(s1.gmres_its)


# ---------------------------------------------------------------------------------------
# adjoint
# ---------------------------------------------------------------------------------------
def _adj_case(seed=1, theta=1.0):
    pd, X = W.random_state((6, 8), ("periodic", "wall"), seed=seed, g=(0.0, -1.0),
                           chi_model="power", chi0=0.05, qwall=((0, 0), (0.1, 0.05)), umag=0.05)
    pd["theta"] = theta
    return Problem.from_dict(pd), X


def test_vjp_dot_product():
    P, X = _adj_case()
    dt = 0.05
    b = rhs_b(P, X, dt)
    v = W.random_vector(X, 2)
    w = W.random_vector(X, 3)
    lhs = np.sum(w * jvp_cs(P, X, b, dt, v))
    rhs = np.sum(vjp_sparse(P, X, b, dt, w) * v)
    assert abs(lhs - rhs) <= 1e-13 * np.linalg.norm(w) * np.linalg.norm(jvp_cs(P, X, b, dt, v))


def test_dU_dX_transpose():
    P, X = _adj_case()
    v = W.random_vector(X, 4)
    lam = W.random_vector(X, 5)
    h = 1e-30
    dU = np.imag(conserved_U(P, X + 1j * h * v)) / h
    assert abs(np.sum(lam * dU) - np.sum(dU_dX_T(P, X, lam) * v)) <= 1e-13 * np.abs(lam * dU).sum()


@pytest.mark.parametrize("theta", [1.0, 0.5])
def test_adjoint_step_matches_finite_differences(theta):
    P, X = _adj_case(seed=2, theta=theta)
    dt = 0.02
    Xn1, _ = exact_step(P, X, dt)
    # loss: kinetic energy sum rho_f u^2 / 2 on faces
    def loss(Y):
        U = conserved_U(P, Y)
        return 0.5 * sum(np.sum(U[2 + d] * Y[2 + d]) for d in range(P.nd))
    def loss_grad(Y):
        lam = np.zeros_like(Y)
        for d in range(P.nd):
            lam[2 + d] = 0.5 * Y[2 + d]
        g = dU_dX_T(P, Y, lam)
        for d in range(P.nd):
            U = conserved_U(P, Y)
            g[2 + d] += 0.5 * U[2 + d]
        return g
    gbar = loss_grad(Xn1)
    gn, _ = adjoint_step_exact(P, Xn1, X, dt, gbar)
    for s in range(3):
        d = W.random_vector(X, 10 + s, bc=P.bc)
        eps = 1e-5
        Lp = loss(exact_step(P, X + eps * d, dt)[0])
        Lm = loss(exact_step(P, X - eps * d, dt)[0])
        fd = (Lp - Lm) / (2 * eps)
        an = np.sum(gn * d)
        assert abs(fd - an) <= 1e-6 * abs(an), (fd, an)


@pytest.mark.parametrize("theta", [1.0, 0.5])
@pytest.mark.parametrize("precond", ["sound", "sound_thermal"])
def test_adjoint_fgmres_matches_lu(precond, theta):
    P, X = _adj_case(seed=3, theta=theta)
    dt = 0.05
    Xn1, _ = exact_step(P, X, dt)
    gbar = W.random_vector(X, 8)
    g1, lam1 = adjoint_step_exact(P, Xn1, X, dt, gbar)
    info = {}
    g2, lam2 = adjoint_step_fgmres(P, Xn1, X, dt, gbar, precond=precond, eta=1e-12, info_out=info)
    assert info["converged"]
    assert np.max(np.abs(g1 - g2)) <= 1e-9 * np.max(np.abs(g1))
