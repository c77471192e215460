"""Pins of the gas + radiation equation of state (Sect. 2) and of the solver built on it.

* a_rad = 0 reproduces the ideal gas exactly (Gamma1 = Gamma3 = gamma);
* T(rho, e) inverts e = c_v T + a T^4/rho to rounding across gas- and radiation-dominated
  states;
* Gamma1 and Gamma3 (App. A: dp/drho|_e = (p/rho)(Gamma1 - Gamma3 + 1), dp/de|_rho =
  rho (Gamma3 - 1)) equal the textbook closed forms of an ideal gas mixed with black-body
  radiation in terms of beta = p_gas/p (Chandrasekhar's stellar-structure treatment);
* the analytic derivatives equal complex steps of p(rho, e) through the Newton iteration;
* a standing sound wave at rest travels at c^2 = Gamma1 p/rho with Gamma1 from the closed
  form (the residual's pressure is the one of the equation of state);
* a discretely balanced radiative polytrope is steady;
* at a uniform rest state the Schur-complement preconditioner is the exact inverse of the
  complex-step Jacobian (its transforms use the same dp/drho, dp/de, Gamma1 as the residual);
* JFNK + PBP reaches the exact root, and the adjoint step matches central differences.
"""
import dataclasses

import numpy as np
import pytest

import workloads as W
from oracle import eos
from oracle.residual import Problem, residual_F, rhs_b, cfl_dt, residual_R, conserved_U
from oracle.jacobian import jacobian_dense_cs, jacobian_dense_central
from oracle.newton import exact_step, jfnk_step, Opts, Stats
from oracle.scaling import scaling_LR
from oracle.pbp import PBP
from oracle.adjoint import adjoint_step_exact, adjoint_step_fgmres


def _prob(gamma=5.0 / 3.0, a_rad=0.0, shape=(4, 4)):
    nd = len(shape)
    return Problem.from_dict(W.make_problem(shape, tuple(1.0 / n for n in shape),
                                            ("periodic",) * nd, gamma, a_rad=a_rad))


def _closed_form(gamma, beta):
    """Gamma1, Gamma3 of an ideal gas (index gamma) + radiation with gas pressure fraction beta."""
    den = beta + 12.0 * (gamma - 1.0) * (1.0 - beta)
    g3 = 1.0 + (4.0 - 3.0 * beta) * (gamma - 1.0) / den
    g1 = beta + (4.0 - 3.0 * beta) ** 2 * (gamma - 1.0) / den
    return g1, g3


def _states(rng, n=200):
    rho = 10.0 ** rng.uniform(-3, 3, n)
    T = 10.0 ** rng.uniform(-2, 3, n)
    return rho, T


def test_ideal_limit_is_exact():
    g = 1.4
    P = _prob(g)
    rng = np.random.default_rng(0)
    rho, e = rng.uniform(0.1, 5, 50), rng.uniform(0.1, 5, 50)
    p, T, dpdr, dpde, G1, cv = eos.thermo(P, rho, e)
    assert np.array_equal(p, (g - 1.0) * rho * e) and np.array_equal(T, (g - 1.0) * e)
    assert np.array_equal(dpdr, (g - 1.0) * e) and np.array_equal(dpde, (g - 1.0) * rho)
    assert np.all(G1 == g) and np.all(cv == 1.0 / (g - 1.0))
    assert np.array_equal(eos.pressure(P, rho, e), p)
    assert np.array_equal(eos.temperature(P, rho, e), T)


@pytest.mark.parametrize("a_rad", [1e-6, 1e-2, 1.0, 1e3])
@pytest.mark.parametrize("gamma", [5.0 / 3.0, 1.4])
def test_temperature_inverts_energy(gamma, a_rad):
    P = _prob(gamma, a_rad)
    rho, T = _states(np.random.default_rng(1))
    e = T / (gamma - 1.0) + a_rad * T ** 4 / rho
    Tr = eos.temperature(P, rho, e)
    assert np.max(np.abs(Tr - T) / T) <= 4e-15
    p = eos.pressure(P, rho, e)
    assert np.max(np.abs(p - (rho * T + a_rad * T ** 4 / 3.0)) / p) <= 1e-14


@pytest.mark.parametrize("gamma", [5.0 / 3.0, 1.4, 1.2])
def test_adiabatic_indices_closed_form(gamma):
    a_rad = 0.3
    P = _prob(gamma, a_rad)
    rho, T = _states(np.random.default_rng(2))
    e = T / (gamma - 1.0) + a_rad * T ** 4 / rho
    p, _, dpdr, dpde, G1, cv = eos.thermo(P, rho, e)
    beta = rho * T / p
    g1, g3 = _closed_form(gamma, beta)
    assert np.min(beta) < 1e-3 and np.max(beta) > 1 - 1e-3  # both limits are visited
    assert np.max(np.abs(G1 - g1) / g1) <= 1e-12
    assert np.max(np.abs(dpde / rho + 1.0 - g3) / g3) <= 1e-12
    assert np.max(np.abs(dpdr - (p / rho) * (g1 - g3 + 1.0)) / np.abs(dpdr)) <= 1e-11
    assert np.max(np.abs(cv - (1.0 / (gamma - 1.0) + 4.0 * a_rad * T ** 3 / rho)) / cv) <= 1e-13
    c2 = eos.sound_speed(P, rho, e) ** 2
    assert np.max(np.abs(c2 - g1 * p / rho) / c2) <= 1e-12


def test_derivatives_match_complex_steps():
    gamma, a_rad = 5.0 / 3.0, 0.7
    P = _prob(gamma, a_rad)
    rho, T = _states(np.random.default_rng(3), 100)
    e = T / (gamma - 1.0) + a_rad * T ** 4 / rho
    _, _, dpdr, dpde, _, cv = eos.thermo(P, rho, e)
    h = 1e-200
    dpdr_cs = np.imag(eos.pressure(P, rho + 1j * h * rho, e)) / (h * rho)
    dpde_cs = np.imag(eos.pressure(P, rho, e + 1j * h * e)) / (h * e)
    dTde_cs = np.imag(eos.temperature(P, rho, e + 1j * h * e)) / (h * e)
    assert np.max(np.abs(dpdr_cs - dpdr) / np.abs(dpdr)) <= 1e-12
    assert np.max(np.abs(dpde_cs - dpde) / dpde) <= 1e-12
    assert np.max(np.abs(dTde_cs * cv - 1.0)) <= 1e-12


@pytest.mark.parametrize("theta", [1.0, 0.5])
@pytest.mark.parametrize("a_rad", [0.3, 30.0])
def test_linear_acoustics_radiation(a_rad, theta):
    """As the ideal-gas acoustics pin, with c^2 = Gamma1 p0/rho0 from the closed form."""
    shape, modes, cfl = (16, 16), (1, 2), 5.0
    gamma, rho0, T0, A = 5.0 / 3.0, 1.0, 1.0, 1e-7
    nd = 2
    h = 1.0 / shape[0]
    gs = W.grid_shape(shape)
    grids = np.meshgrid(*[(np.arange(n) + 0.5) * h for n in gs], indexing="ij")
    pos = [grids[nd - 1 - d] for d in range(nd)]
    k = [2 * np.pi * modes[d] for d in range(nd)]
    phase = sum(k[d] * pos[d] for d in range(nd))
    pg0, pr0 = rho0 * T0, a_rad * T0 ** 4 / 3.0
    p0 = pg0 + pr0
    g1, _ = _closed_form(gamma, pg0 / p0)
    c = np.sqrt(g1 * p0 / rho0)
    # adiabatic perturbation: drho = dp/c^2, de = (p0/rho0^2) drho
    drho = A * p0 * np.cos(phase) / c ** 2
    e0 = T0 / (gamma - 1.0) + a_rad * T0 ** 4 / rho0
    X = np.zeros((2 + nd,) + gs)
    X[0] = rho0 + drho
    X[1] = e0 + p0 / rho0 ** 2 * drho
    P = Problem.from_dict(W.make_problem(shape, (h,) * nd, ("periodic",) * nd, gamma,
                                         theta=theta, a_rad=a_rad))
    dt = cfl * h / c
    Xn1, _ = exact_step(P, X, dt)
    pn = eos.pressure(P, X[0], X[1]) - p0
    pn1 = eos.pressure(P, Xn1[0], Xn1[1]) - p0
    basis = np.cos(phase)
    ratio = np.sum(pn1 * basis) / np.sum(pn * basis)
    w2 = c ** 2 * sum((2 / h) ** 2 * np.sin(k[d] * h / 2) ** 2 for d in range(nd))
    expect = (1 - theta * (1 - theta) * w2 * dt ** 2) / (1 + theta ** 2 * w2 * dt ** 2)
    assert abs(ratio - expect) <= 2e-5 * max(abs(expect), 1e-3), (ratio, expect)


def test_hydrostatic_radiative_polytrope():
    w = W.polytrope((16, 32), 10.0, mach=0.0, chi_model="const", steps=1, a_rad=0.05)
    P = Problem.from_dict(w["problem"])
    X = w["X0"]
    dt = cfl_dt(P, X, 100.0)
    F = residual_F(P, X, rhs_b(P, X, dt), dt)
    _, Aabs = residual_R(P, X, with_abs=True)
    for k in range(P.nvar):
        assert np.max(np.abs(F[k])) <= 1e-13 * np.max(Aabs[k]), k
    pg = X[0] * eos.temperature(P, X[0], X[1])
    pr = eos.pressure(P, X[0], X[1]) - pg
    assert np.max(pr / pg) > 0.2  # radiation is not negligible at the bottom


@pytest.mark.parametrize("theta", [1.0, 0.5])
@pytest.mark.parametrize("shape,bc", [((6, 5), ("periodic", "periodic")), ((5, 6), ("periodic", "wall")),
                                      ((4, 3, 4), ("periodic", "wall", "periodic"))])
def test_schur_pbp_exact_inverse_radiation(shape, bc, theta):
    nd = len(shape)
    P = Problem.from_dict(W.make_problem(shape, tuple(1.0 / n for n in shape), bc, 5.0 / 3.0,
                                         theta=theta, a_rad=2.0))
    X = np.zeros((2 + nd,) + W.grid_shape(shape))
    X[0], X[1] = 1.3, 4.0
    dt = 0.3
    Jd = jacobian_dense_cs(P, X, rhs_b(P, X, dt), dt)
    r = W.random_vector(X, 12, bc=P.bc)
    z = PBP(P, X, dt, "sound", schur=True).apply(r)
    back = (Jd @ z.ravel()).reshape(r.shape)
    assert np.max(np.abs(back - r)) / np.max(np.abs(r)) <= 1e-11


def _rad_case(seed=1, theta=1.0, shape=(6, 8)):
    pd, X = W.random_state(shape, ("periodic", "wall"), seed=seed, g=(0.0, -1.0),
                           chi_model="power", chi0=0.05, qwall=((0, 0), (0.1, 0.05)), umag=0.05,
                           a_rad=0.5)
    pd["theta"] = theta
    return Problem.from_dict(pd), X


def test_complex_step_jacobian_radiation():
    P, X = _rad_case(seed=4, shape=(5, 6))
    dt = 0.02
    b = rhs_b(P, X, dt)
    Jc = jacobian_dense_cs(P, X, b, dt)
    Jd = jacobian_dense_central(P, X, b, dt)
    assert np.max(np.abs(Jc - Jd)) <= 1e-7 * np.max(np.abs(Jc))


@pytest.mark.parametrize("mode", ["sound", "sound_thermal"])
@pytest.mark.parametrize("schur", [False, True])
def test_pbp_transpose_radiation(mode, schur):
    P, X = _rad_case(seed=5)
    pbp = PBP(P, X, 0.15, mode, schur=schur)
    r = W.random_vector(X, 6)
    w = W.random_vector(X, 7)
    a = np.sum(w * pbp.apply(r))
    b = np.sum(pbp.apply_T(w) * r)
    assert abs(a - b) <= 1e-12 * (abs(a) + abs(b))


def test_jfnk_radiative_thermal():
    w = W.radiative_2d(n=8, seed=5, cfl=50.0)
    P = Problem.from_dict(w["problem"])
    X0 = w["X0"]
    dt = cfl_dt(P, X0, 50.0)
    Xs, _ = exact_step(P, X0, dt)
    st = Stats()
    X = jfnk_step(P, X0, dt, Opts(precond="sound_thermal", elliptic="pcg"), st)
    _, R = scaling_LR(P, Xs)
    assert st.converged
    assert np.max(np.abs((X - Xs) / R)) <= 1e-9


@pytest.mark.parametrize("theta", [1.0, 0.5])
def test_adjoint_step_radiation(theta):
    P, X = _rad_case(seed=2, theta=theta, shape=(4, 6))
    dt = 0.02
    Xn1, _ = exact_step(P, X, dt)

    def loss(Y):
        return float(np.sum(eos.pressure(P, Y[0], Y[1]) ** 2))

    def loss_grad(Y):
        p, _, dpdr, dpde, _, _ = eos.thermo(P, Y[0], Y[1])
        g = np.zeros_like(Y)
        g[0], g[1] = 2 * p * dpdr, 2 * p * dpde
        return g

    gbar = loss_grad(Xn1)
    gn, _ = adjoint_step_exact(P, Xn1, X, dt, gbar)
    for s in range(2):
        d = W.random_vector(X, 10 + s, bc=P.bc)
        eps = 1e-6
        fd = (loss(exact_step(P, X + eps * d, dt)[0]) - loss(exact_step(P, X - eps * d, dt)[0])) / (2 * eps)
        an = np.sum(gn * d)
        assert abs(fd - an) <= 1e-6 * abs(an), (fd, an)
    info = {}
    g2, _ = adjoint_step_fgmres(P, Xn1, X, dt, gbar, precond="sound_thermal", eta=1e-12,
                                info_out=info)
    assert info["converged"]
    assert np.max(np.abs(gn - g2)) <= 1e-9 * np.max(np.abs(gn))
