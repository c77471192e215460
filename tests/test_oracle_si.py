"""Pins of the stand-alone semi-implicit stepper (Sect. 3.6).

* Schur form (the scheme of Sect. 3.3, Laplacian on p^{n+1}): a small standing sound wave at
  a uniform rest state is scaled by the theta-step factor of the discrete wave equation,
  (1 - theta(1-theta) w^2 dt^2)/(1 + theta^2 w^2 dt^2), as for the exact implicit step (the
  scheme is exact for the linearised acoustics there);
* delta-form J~_V with F~_V = (dV/dU) F_U: the first step from rest leaves rho and e exactly
  unchanged and sets u = -dt (p[c] - p[c-1]) / (dx rho_f), the explicit pressure force;
* walls: the wall-normal velocity on wall faces stays exactly zero;
* the Schur form has a low-Mach limit: one step of the isentropic vortex changes u by an
  amount that converges as Mach^2 when T_inf grows.
"""
import numpy as np
import pytest

import workloads as W
from oracle import eos
from oracle.residual import Problem
from oracle.si import si_step


def _wave(shape, modes, theta, gamma=1.4, A=1e-7):
    nd = len(shape)
    h = 1.0 / shape[0]
    gs = W.grid_shape(shape)
    grids = np.meshgrid(*[(np.arange(n) + 0.5) * h for n in gs], indexing="ij")
    pos = [grids[nd - 1 - d] for d in range(nd)]
    k = [2 * np.pi * modes[d] for d in range(nd)]
    phase = sum(k[d] * pos[d] for d in range(nd))
    p = 1.0 + A * np.cos(phase)
    rho = p ** (1 / gamma)
    X = np.zeros((2 + nd,) + gs)
    X[0] = rho
    X[1] = p / ((gamma - 1) * rho)
    P = Problem.from_dict(W.make_problem(shape, (h,) * nd, ("periodic",) * nd, gamma, theta=theta))
    return P, X, phase, k, h


@pytest.mark.parametrize("theta", [1.0, 0.5])
@pytest.mark.parametrize("shape,modes,cfl", [((16, 16), (1, 2), 3.0), ((8, 8, 8), (1, 1, 2), 40.0)])
def test_schur_si_step_linear_acoustics(shape, modes, cfl, theta):
    gamma = 1.4
    P, X, phase, k, h = _wave(shape, modes, theta, gamma)
    nd = len(shape)
    c = np.sqrt(gamma)
    dt = cfl * h / c
    Xn1 = si_step(P, X, dt, "sound", schur=True)
    basis = np.cos(phase)
    p0 = eos.pressure(P, X[0], X[1]) - 1.0
    p1 = eos.pressure(P, Xn1[0], Xn1[1]) - 1.0
    ratio = np.sum(p1 * basis) / np.sum(p0 * basis)
    w2 = c ** 2 * sum((2 / h) ** 2 * np.sin(k[d] * h / 2) ** 2 for d in range(nd))
    expect = (1 - theta * (1 - theta) * w2 * dt ** 2) / (1 + theta ** 2 * w2 * dt ** 2)
    assert abs(ratio - expect) <= 1e-5 * max(abs(expect), 1e-3), (ratio, expect)


def test_delta_form_si_first_step_from_rest_is_explicit_momentum():
    P, X, phase, k, h = _wave((16, 8), (2, 1), 1.0, A=1e-3)
    dt = 0.01
    Xn1 = si_step(P, X, dt, "sound", schur=False)
    assert np.array_equal(Xn1[0], X[0]) and np.array_equal(Xn1[1], X[1])
    p = eos.pressure(P, X[0], X[1])
    for d in range(P.nd):
        ax = P.axis(d)
        rf = 0.5 * (np.roll(X[0], 1, axis=ax) + X[0])
        u = -dt * (p - np.roll(p, 1, axis=ax)) / (P.dx[d] * rf)
        assert np.max(np.abs(Xn1[2 + d] - u)) <= 1e-12 * np.max(np.abs(u))


@pytest.mark.parametrize("mode", ["sound", "sound_thermal"])
@pytest.mark.parametrize("schur", [True, False])
def test_si_step_keeps_wall_velocity_zero(mode, schur):
    w = W.polytrope((8, 16), 10.0, mach=1e-2, seed=3, chi_model="power", steps=1, cfl=50.0)
    P = Problem.from_dict(w["problem"])
    X = w["X0"]
    Xn1 = si_step(P, X, 0.05, mode, schur=schur)
    assert np.all(Xn1[3][0] == 0.0)
    assert np.all(np.isfinite(Xn1))


def test_schur_si_step_has_a_low_mach_limit():
    """Isentropic vortex (Sect. 3.7) at T_inf = 1e4, 1e6, 1e8 (Mach 8.5e-4 .. 8.5e-6): the
    velocity change of one step at the same advective CFL (0.1) converges as Mach^2 ~ 1/T_inf
    (each factor 100 in T_inf divides the difference by ~100), the Mach-independence the
    scheme was built for."""
    du = []
    for t_inf in (1e4, 1e6, 1e8):
        w = W.isentropic_vortex_2d(n=32, t_inf=t_inf)
        P = Problem.from_dict(w["problem"])
        X = w["X0"]
        dt = 0.1 * P.dx[0]
        du.append(si_step(P, X, dt, "sound", schur=True)[2:] - X[2:])
    d1 = np.max(np.abs(du[0] - du[1])) / np.max(np.abs(du[1]))
    d2 = np.max(np.abs(du[1] - du[2])) / np.max(np.abs(du[2]))
    assert d2 <= 1e-5 and 50.0 <= d1 / d2 <= 200.0, (d1, d2)
