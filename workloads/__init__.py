"""Seeded synthetic input generators shared by the oracle tests, the GPU tests and bench.py.

This module builds initial states and problem descriptions only.  It holds none of the
solver's arithmetic (no residual, no time-step rule, no preconditioner): the time step each
side uses is computed by that side from the state.  Values the recipes need (sound speed for
noise amplitudes, a reference time step for sizing the conductivity) are recipe constants.

State layout: ``X`` has shape ``(nvar, *grid)`` where ``grid`` is ``(ny, nx)`` in 2D and
``(nz, ny, nx)`` in 3D (x fastest).  Variables: rho, e, u_x, u_y[, u_z].  Cell (i, j[, k])
is centred at ((i+1/2)dx, (j+1/2)dy, ...); ``u_d`` of cell c sits on the low-d face of c.

Problem descriptions are plain dicts (see ``make_problem``) so that the oracle and the
binding each translate them into their own structures.

Workloads follow the paper's test problems (isentropic vortex and Taylor-Green set-ups of
the Results section, stratified boxes for the stellar-interior runs), restated with explicit
sizes because the paper's own stellar models are not published.
"""
from __future__ import annotations

import math

import numpy as np

PERIODIC = "periodic"
WALL = "wall"


def make_problem(shape, dx, bc, gamma, g=None, chi_model="none", chi0=0.0, chi_tref=1.0,
                 chi_exp=3.0, qwall=None, theta=1.0, a_rad=0.0):
    """Plain-dict problem description.

    shape: cells per axis ordered (nx, ny[, nz]); dx: spacing per axis; bc: per-axis
    'periodic' | 'wall'; g: gravity vector per axis; chi_model: 'none' | 'const' | 'power'
    (chi = chi0 * (T/chi_tref)**chi_exp); qwall: per axis (lo, hi) prescribed conductive flux
    chi*dT/dx_d through the wall faces (only read on wall axes); theta: time-weighting of the
    step (1 backward Euler, 1/2 Crank-Nicolson); a_rad: radiation constant of the gas +
    radiation equation of state (0: ideal gas).
    """
    nd = len(shape)
    return dict(
        ndim=nd,
        shape=tuple(int(n) for n in shape),
        dx=tuple(float(h) for h in dx),
        bc=tuple(bc),
        gamma=float(gamma),
        g=tuple(float(x) for x in (g if g is not None else (0.0,) * nd)),
        chi_model=chi_model,
        chi0=float(chi0),
        chi_tref=float(chi_tref),
        chi_exp=float(chi_exp),
        qwall=tuple(tuple(float(q) for q in qw) for qw in (qwall if qwall is not None else ((0.0, 0.0),) * nd)),
        theta=float(theta),
        a_rad=float(a_rad),
    )


def grid_shape(shape):
    """numpy array shape of one field for a grid given as (nx, ny[, nz])."""
    return tuple(reversed(shape))


def _axis(nd, d):
    """numpy axis of spatial axis d inside a single field array."""
    return nd - 1 - d


def _centres(n, h, lo=0.0):
    return lo + (np.arange(n) + 0.5) * h


def _faces(n, h, lo=0.0):
    return lo + np.arange(n) * h


def _sound_speed(gamma, e):
    return np.sqrt(gamma * (gamma - 1.0) * e)


def _face_avg(q, nd, d, bc):
    """0.5*(q[c-e_d] + q[c]) with wrap (periodic) or copy (wall) for the missing neighbour."""
    a = _axis(nd, d)
    lower = np.roll(q, 1, axis=a)
    if bc[d] == WALL:
        sl = [slice(None)] * nd
        sl[a] = 0
        lower[tuple(sl)] = q[tuple(sl)]
    return 0.5 * (lower + q)


def _velocity_noise(rng, X, nd, bc, gamma, mach):
    """u_d = mach * c_s,f * xi, xi ~ U[-1, 1] i.i.d.; wall-normal faces at the wall are 0."""
    cs = _sound_speed(gamma, X[1])
    for d in range(nd):
        xi = rng.uniform(-1.0, 1.0, size=X[1].shape)
        u = mach * _face_avg(cs, nd, d, bc) * xi
        if bc[d] == WALL:
            sl = [slice(None)] * nd
            sl[_axis(nd, d)] = 0
            u[tuple(sl)] = 0.0
        X[2 + d] = u


# ----------------------------------------------------------------------------------------
# 2D acoustic pulse in a periodic box
# ----------------------------------------------------------------------------------------
def acoustic_bump_2d(n=32, seed=1001, gamma=5.0 / 3.0, amp=1e-3, width_cells=4.0, cfl=10.0):
    """Gaussian density bump on a uniform periodic box, isentropic pressure p = rho**gamma.

    The bump centre is drawn uniformly in the unit box; the distance is the periodic
    minimum-image distance; u = 0.
    """
    rng = np.random.default_rng(seed)
    centre = rng.uniform(0.0, 1.0, size=2)
    h = 1.0 / n
    x = _centres(n, h)
    dxv = np.abs(x[None, :] - centre[0])
    dyv = np.abs(x[:, None] - centre[1])
    dxv = np.minimum(dxv, 1.0 - dxv)
    dyv = np.minimum(dyv, 1.0 - dyv)
    r2 = dxv ** 2 + dyv ** 2
    sigma = width_cells * h
    rho = 1.0 + amp * np.exp(-r2 / (2.0 * sigma ** 2))
    p = rho ** gamma
    X = np.zeros((4, n, n))
    X[0] = rho
    X[1] = p / ((gamma - 1.0) * rho)
    prob = make_problem((n, n), (h, h), (PERIODIC, PERIODIC), gamma)
    return dict(name=f"acoustic_bump_2d_{n}x{n}", problem=prob, X0=X, cfl=cfl, steps=1,
                precond="sound", jv_mode="fd")


# ----------------------------------------------------------------------------------------
# Stratified polytropic boxes (2D 256^2 and 512^2, 3D 256^3)
# ----------------------------------------------------------------------------------------
def polytrope(shape, contrast, poly_n=1.5, gamma=5.0 / 3.0, mach=1e-3, seed=1002, cfl=100.0,
              cfl_rad=10.0, chi_model="const", chi_exp=3.0, steps=10, name="polytrope",
              a_rad=0.0):
    """Discretely hydrostatic polytrope on [0,1]^nd, gravity along -(last axis), walls there.

    T is linear in height at cell centres with T(top boundary) = 1 and
    T(bottom boundary) = contrast**(1/n); g = (n+1)(T_bot - T_top).  rho in the top cell is
    (T/T_top)**n and lower cells follow the recursion that makes the staggered pressure
    gradient balance rho_f * g exactly:  rho_{j-1} = rho_j (T_j + g h/2) / (T_{j-1} - g h/2).
    Face velocities get noise of amplitude mach * c_s,f.  The conductivity is sized so that
    max chi*dt_ref/(rho c_v dx^2) = cfl_rad with dt_ref = cfl*dx/max(c_s) (velocity ignored).
    The prescribed wall fluxes equal the conductive flux of the initial state at the first
    interior face next to each wall.

    a_rad > 0 (gas + radiation, p = rho T + a T^4/3, e = c_v T + a T^4/rho): the same T
    profile, g scaled by p/p_gas = 1 + a T_top^3/3 of the top, and the radiation pressure
    difference added to the balance,
    rho_{j-1} (T_{j-1} - g h/2) = rho_j (T_j + g h/2) - a (T_{j-1}^4 - T_j^4)/3.
    With poly_n = 3 this is the discrete form of a constant-beta (p_gas/p) polytrope.
    """
    nd = len(shape)
    vert = nd - 1
    nz = shape[vert]
    h = 1.0 / np.asarray(shape, dtype=float)
    hz = h[vert]
    t_bot = contrast ** (1.0 / poly_n)
    t_top = 1.0
    gmag = (poly_n + 1.0) * (t_bot - t_top) * (1.0 + a_rad * t_top ** 3 / 3.0)
    zc = _centres(nz, hz)
    T1 = t_top + (t_bot - t_top) * (1.0 - zc)
    rho1 = np.empty(nz)
    rho1[-1] = (T1[-1] / t_top) ** poly_n
    for j in range(nz - 1, 0, -1):
        rho1[j - 1] = (rho1[j] * (T1[j] + 0.5 * gmag * hz)
                       - a_rad * (T1[j - 1] ** 4 - T1[j] ** 4) / 3.0) / (T1[j - 1] - 0.5 * gmag * hz)
    if not np.all(rho1 > 0.0):
        raise ValueError("radiation pressure gradient exceeds gravity: lower a_rad")
    gs = grid_shape(shape)
    bshape = [1] * nd
    bshape[0] = nz  # vertical axis is numpy axis 0
    T = np.broadcast_to(T1.reshape(bshape), gs).copy()
    rho = np.broadcast_to(rho1.reshape(bshape), gs).copy()
    X = np.zeros((2 + nd,) + gs)
    X[0] = rho
    X[1] = T / (gamma - 1.0)
    if a_rad > 0.0:
        X[1] += a_rad * T ** 4 / rho
    bc = tuple([PERIODIC] * (nd - 1) + [WALL])
    rng = np.random.default_rng(seed)
    _velocity_noise(rng, X, nd, bc, gamma, mach)
    g = [0.0] * nd
    g[vert] = -gmag
    # conductivity sizing
    cv = 1.0 / (gamma - 1.0)
    hmin = float(h.min())
    dt_ref = cfl * hmin / float(_sound_speed(gamma, X[1]).max())
    if chi_model == "const":
        shape_fac = 1.0 / (rho1 * cv)
        chi_of_T = lambda t: np.ones_like(t)
    elif chi_model == "power":
        shape_fac = (T1 / t_top) ** chi_exp / (rho1 * cv)
        chi_of_T = lambda t: (t / t_top) ** chi_exp
    else:
        raise ValueError(chi_model)
    chi0 = cfl_rad * hmin ** 2 / (dt_ref * float(shape_fac.max()))
    chi1 = chi0 * chi_of_T(T1)
    q_lo = 0.5 * (chi1[0] + chi1[1]) * (T1[1] - T1[0]) / hz
    q_hi = 0.5 * (chi1[-2] + chi1[-1]) * (T1[-1] - T1[-2]) / hz
    qwall = [(0.0, 0.0)] * nd
    qwall[vert] = (q_lo, q_hi)
    prob = make_problem(shape, tuple(h), bc, gamma, g=g, chi_model=chi_model, chi0=chi0,
                        chi_tref=t_top, chi_exp=chi_exp, qwall=qwall, a_rad=a_rad)
    return dict(name=name, problem=prob, X0=X, cfl=cfl, steps=steps, precond="sound_thermal",
                jv_mode="fd", cfl_rad=cfl_rad)


def stratified_2d(n=256, seed=1002, steps=10, cfl=100.0):
    """2D polytrope n=1.5, density contrast 10, constant conductivity, Mach 1e-3 noise."""
    w = polytrope((n, n), 10.0, mach=1e-3, seed=seed, cfl=cfl, chi_model="const", steps=steps,
                  name=f"stratified_2d_{n}x{n}")
    return w


def stratified_2d_kappa(n=512, seed=1004, steps=5, cfl=50.0):
    """As stratified_2d (at 512^2) with chi = chi0 (T/T_top)^3 (the adjoint workload)."""
    return polytrope((n, n), 10.0, mach=1e-3, seed=seed, cfl=cfl, chi_model="power", steps=steps,
                     name=f"stratified_2d_kappa_{n}x{n}")


def radiative_2d(n=256, seed=1006, steps=5, cfl=50.0, a_rad=1.0):
    """Gas + radiation polytrope n = 3 (chi ~ T^3, density contrast 10): a_rad = 1 gives
    p_rad/p_gas = 1/3 (beta = 3/4) throughout, Gamma1 = 1.49 and Gamma3 = 1.42 instead of 5/3.
    n = 3 is below the adiabatic gradient of such a mixture, so the box is convectively stable
    (n = 1.5 with radiation would be unstable)."""
    return polytrope((n, n), 10.0, poly_n=3.0, mach=1e-3, seed=seed, cfl=cfl,
                     chi_model="power", steps=steps, name=f"radiative_2d_{n}x{n}", a_rad=a_rad)


def convective_box_3d(n=256, seed=1005, steps=10, cfl=500.0):
    """3D polytrope n=1.5, density contrast 20, chi ~ T^3, Mach 1e-4 noise."""
    return polytrope((n, n, n), 20.0, mach=1e-4, seed=seed, cfl=cfl, chi_model="power",
                     steps=steps, name=f"convective_box_3d_{n}^3")


# ----------------------------------------------------------------------------------------
# 3D Taylor-Green vortex at low Mach
# ----------------------------------------------------------------------------------------
def taylor_green_3d(n=128, seed=1003, mach=1e-6, gamma=1.4, noise=1e-8, cfl=1000.0, steps=5):
    """Taylor-Green velocity on [0, 2pi)^3 with the divergence-preserving pressure.

    rho0 = p0 = 1, u0 = mach * sqrt(gamma p0/rho0).  u_x, u_y are sampled at their face
    centres, p at cell centres; T = p/rho0 is then perturbed isobarically by
    (1 + noise*xi), rho = p/T, e = T/(gamma-1).
    """
    rng = np.random.default_rng(seed)
    L = 2.0 * math.pi
    h = L / n
    u0 = mach * math.sqrt(gamma)
    xc = _centres(n, h)
    xf = _faces(n, h)
    Z, Y, Xc = np.meshgrid(xc, xc, xc, indexing="ij")
    p = 1.0 + (1.0 / 16.0) * u0 ** 2 * (2.0 + np.cos(2 * Z)) * (np.cos(2 * Xc) + np.cos(2 * Y))
    T = p.copy()
    T *= 1.0 + noise * rng.uniform(-1.0, 1.0, size=T.shape)
    rho = p / T
    X = np.zeros((5, n, n, n))
    X[0] = rho
    X[1] = T / (gamma - 1.0)
    Zc, Yc, Xf = np.meshgrid(xc, xc, xf, indexing="ij")
    X[2] = u0 * np.sin(Xf) * np.cos(Yc) * np.cos(Zc)
    Zc, Yf, Xc2 = np.meshgrid(xc, xf, xc, indexing="ij")
    X[3] = -u0 * np.cos(Xc2) * np.sin(Yf) * np.cos(Zc)
    prob = make_problem((n, n, n), (h, h, h), (PERIODIC,) * 3, gamma)
    return dict(name=f"taylor_green_3d_{n}^3", problem=prob, X0=X, cfl=cfl, steps=steps,
                precond="sound", jv_mode="fd")


def _vortex_fields(x, y, gamma, beta):
    r2 = x ** 2 + y ** 2
    du = beta / (2 * math.pi) * np.exp(0.5 * (1 - r2)) * (-y)
    dv = beta / (2 * math.pi) * np.exp(0.5 * (1 - r2)) * x
    dT = -(gamma - 1.0) * beta ** 2 / (8 * gamma * math.pi ** 2) * np.exp(1 - r2)
    return du, dv, dT


def isentropic_vortex_u_exact(n=64, t=0.4, gamma=1.4, beta=0.75, u_inf=1.0):
    """u on the x-faces of the initial vortex translated by u_inf t along x on the periodic
    domain (the exact solution the semi-implicit test of Sect. 3.7 measures errors against;
    t = 8/u_inf is one full crossing)."""
    h = 8.0 / n
    yc = _centres(n, h, -4.0)
    xf = _faces(n, h, -4.0)
    Yc, Xf = np.meshgrid(yc, xf, indexing="ij")
    xs = np.mod(Xf - u_inf * t + 4.0, 8.0) - 4.0
    du, _, _ = _vortex_fields(xs, Yc, gamma, beta)
    return u_inf + du


def isentropic_vortex_2d(n=64, t_inf=1.0, gamma=1.4, beta=0.75, u_inf=1.0):
    """Isentropic vortex on [-4,4]^2 advected by a uniform flow along x (Results section)."""
    L = 8.0
    h = L / n
    xc = _centres(n, h, -4.0)
    xf = _faces(n, h, -4.0)

    def fields(x, y):
        return _vortex_fields(x, y, gamma, beta)

    Y, Xg = np.meshgrid(xc, xc, indexing="ij")
    _, _, dT = fields(Xg, Y)
    rho = (t_inf + dT) ** (1.0 / (gamma - 1.0))
    X = np.zeros((4, n, n))
    X[0] = rho
    # e from p = rho T (R = 1): e = T/(gamma-1)
    X[1] = (t_inf + dT) / (gamma - 1.0)
    Yc, Xf = np.meshgrid(xc, xf, indexing="ij")
    du, _, _ = fields(Xf, Yc)
    X[2] = u_inf + du
    Yf, Xc2 = np.meshgrid(xf, xc, indexing="ij")
    _, dv, _ = fields(Xc2, Yf)
    X[3] = dv
    prob = make_problem((n, n), (h, h), (PERIODIC, PERIODIC), gamma)
    return dict(name=f"isentropic_vortex_2d_{n}", problem=prob, X0=X, cfl=None, steps=None,
                precond="sound", jv_mode="fd")


# ----------------------------------------------------------------------------------------
# Small random states for Jacobian / parity tests
# ----------------------------------------------------------------------------------------
def random_state(shape, bc, seed, gamma=1.4, amp=0.3, umag=0.3, g=None, chi_model="none",
                 chi0=0.0, chi_tref=1.0, chi_exp=3.0, qwall=None, a_rad=0.0):
    """Smooth-free random state: rho, e = 1 + amp*xi; u = umag*xi (walls: normal faces 0).

    Random values avoid the branch ties of the upwind and limiter switches almost surely.
    """
    rng = np.random.default_rng(seed)
    nd = len(shape)
    gs = grid_shape(shape)
    X = np.zeros((2 + nd,) + gs)
    X[0] = 1.0 + amp * rng.uniform(-1, 1, gs)
    X[1] = 1.0 + amp * rng.uniform(-1, 1, gs)
    for d in range(nd):
        u = umag * rng.uniform(-1, 1, gs)
        if bc[d] == WALL:
            sl = [slice(None)] * nd
            sl[_axis(nd, d)] = 0
            u[tuple(sl)] = 0.0
        X[2 + d] = u
    h = tuple(1.0 / n for n in shape)
    prob = make_problem(shape, h, bc, gamma, g=g, chi_model=chi_model, chi0=chi0,
                        chi_tref=chi_tref, chi_exp=chi_exp, qwall=qwall, a_rad=a_rad)
    return prob, X


def random_vector(X, seed, amp=1.0, bc=None):
    """Random direction of the same shape as X (wall-normal wall faces zeroed if bc given)."""
    rng = np.random.default_rng(seed)
    v = amp * rng.uniform(-1, 1, X.shape)
    if bc is not None:
        nd = X.ndim - 1
        for d in range(nd):
            if bc[d] == WALL:
                sl = [slice(None)] * nd
                sl[_axis(nd, d)] = 0
                v[(2 + d,) + tuple(sl)] = 0.0
    return v


CONFIGS = {
    "acoustic_bump_2d": acoustic_bump_2d,
    "stratified_2d": stratified_2d,
    "taylor_green_3d": taylor_green_3d,
    "stratified_2d_kappa": stratified_2d_kappa,
    "convective_box_3d": convective_box_3d,
    "radiative_2d": radiative_2d,
}
