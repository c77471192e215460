"""Pins of the Newton scaling (Sect. 4.1) and the physics-based preconditioner (Sects. 3-4.3).

Scaling: hand-computed values on a two-cell state.  Preconditioner: transformation-matrix
identities of App. B; symmetry, positivity and Fourier eigenvalues of the elliptic operators;
the identity-based energy update equals the explicit-Laplacian semi-implicit equations
(Sect. 3.3 and 3.4); the transposed preconditioner passes the dot-product test.
"""
import dataclasses

import numpy as np
import pytest

import workloads as W
from oracle.residual import Problem, rhs_b
from oracle.scaling import scaling_LR
from oracle.pbp import (PBP, EllOp, pressure_operator, thermal_operator, transform_in,
                        grad_face, face_mean, eos_derivs)


def test_scaling_hand_values():
    """gamma = 2: c_s = sqrt(2 e).  Cells (x-periodic, 2 cells): rho = (1, 3), e = (2, 8)
    -> c_s = (2, 4), face means rho_f = 2, c_s,f = 3 at both faces.  u_x = (0.5, -6)."""
    pd = W.make_problem((2, 1), (0.5, 1.0), ("periodic", "periodic"), 2.0)
    P = Problem.from_dict(pd)
    X = np.zeros((4, 1, 2))
    X[0, 0] = [1.0, 3.0]
    X[1, 0] = [2.0, 8.0]
    X[2, 0] = [0.5, -6.0]
    X[3, 0] = [0.0, 0.0]
    L, R = scaling_LR(P, X, alpha1=1e-5, alpha2=1.0)
    assert np.allclose(L[0, 0], [1, 3]) and np.allclose(L[1, 0], [2, 24])
    assert np.allclose(R[0, 0], [1, 3]) and np.allclose(R[1, 0], [2, 8])
    assert np.allclose(R[2, 0], [3.0, 6.0])          # max(|u|, 1 * 3)
    assert np.allclose(L[2, 0], [2 * 0.5, 2 * 6.0])  # rho_f max(|u|, 1e-5 * 3)
    # y faces: each cell is its own periodic neighbour: rho_f = rho, c_s,f = c_s, u = 0
    assert np.allclose(R[3, 0], [2.0, 4.0])
    assert np.allclose(L[3, 0], [1 * 1e-5 * 2, 3 * 1e-5 * 4])


def test_transformation_identities():
    """dV/dX . dX/dU = dV/dU and dX/dV . dV/dX = I (App. B), pointwise on a uniform state
    (face means are then the cell values).  dp from the transform equals the EOS variation."""
    pd = W.make_problem((4, 4), (0.25, 0.25), ("periodic", "periodic"), 5.0 / 3.0)
    P = Problem.from_dict(pd)
    X = np.zeros((4, 4, 4))
    X[0], X[1], X[2], X[3] = 1.3, 0.7, 0.2, -0.1
    rng = np.random.default_rng(0)
    dX = rng.uniform(-1, 1, X.shape)
    dX[:, :, :] = dX[:, :1, :1]  # uniform perturbation
    rho, e = X[0], X[1]
    # dU = dU/dX dX for U = (rho, rho e, rho u)
    dU = np.stack([dX[0], e * dX[0] + rho * dX[1], X[2] * dX[0] + rho * dX[2],
                   X[3] * dX[0] + rho * dX[3]])
    Fp, Fe, Fu = transform_in(P, X, dU)
    g = P.gamma
    p = lambda r, ee: (g - 1) * r * ee
    h = 1e-30
    dp_cs = np.imag(p(rho + 1j * h * dX[0], e + 1j * h * dX[1])) / h
    assert np.allclose(Fp, dp_cs, rtol=1e-14)
    assert np.allclose(Fe, dX[1], rtol=1e-14)
    assert np.allclose(Fu[0], dX[2], rtol=1e-14) and np.allclose(Fu[1], dX[3], rtol=1e-14)
    dpdr, dpde = eos_derivs(P, X)
    assert np.allclose((Fp - dpde * Fe) / dpdr, dX[0], rtol=1e-13)
    # thermodynamic identity dp/drho|_e = p/rho for Gamma1 = Gamma3 (App. A)
    assert np.allclose(dpdr, p(rho, e) / rho, rtol=1e-15)


def _state(shape, bc, seed=1):
    nd = len(shape)
    g = tuple([0.0] * (nd - 1) + [-1.0]) if "wall" in bc else None
    pd, X = W.random_state(shape, bc, seed=seed, g=g, chi_model="power", chi0=0.05)
    return Problem.from_dict(pd), X


@pytest.mark.parametrize("shape,bc", [((8, 6), ("periodic", "wall")), ((4, 4, 6), ("periodic", "periodic", "wall")),
                                      ((8, 8), ("periodic", "periodic"))])
def test_elliptic_operators_spd(shape, bc):
    P, X = _state(shape, bc)
    for op in (pressure_operator(P, X, 0.3), thermal_operator(P, X, 0.3)):
        A = op.to_sparse().toarray()
        assert np.max(np.abs(A - A.T)) <= 1e-15 * np.max(np.abs(A))
        assert np.min(np.linalg.eigvalsh(A)) > 0
        phi = np.random.default_rng(2).uniform(-1, 1, P.field_shape)
        assert np.allclose(op.apply(phi).ravel(), A @ phi.ravel(), rtol=1e-13, atol=1e-13 * np.abs(A).max())


def test_pressure_operator_fourier_eigenvalue():
    """Constant coefficients, periodic: cos modes are eigenvectors with eigenvalue
    1/(Gamma1 p dt) + dt/rho sum_d (2/dx_d)^2 sin^2(k_d dx_d/2)."""
    nx, ny = 16, 8
    pd = W.make_problem((nx, ny), (1.0 / nx, 0.5 / ny), ("periodic", "periodic"), 1.4)
    P = Problem.from_dict(pd)
    X = np.zeros((4, ny, nx))
    X[0], X[1] = 2.0, 3.0
    dt = 0.01
    op = pressure_operator(P, X, dt)
    xc = (np.arange(nx) + 0.5) / nx
    yc = (np.arange(ny) + 0.5) * 0.5 / ny
    kx, ky = 2 * np.pi * 3, 2 * np.pi * 2 / 0.5
    phi = np.cos(kx * xc[None, :] + ky * yc[:, None])
    p = 0.4 * 2.0 * 3.0
    lam = 1 / (1.4 * p * dt) + dt / 2.0 * ((2 * nx) ** 2 * np.sin(kx / nx / 2) ** 2
                                           + (2 * ny / 0.5) ** 2 * np.sin(ky * 0.5 / ny / 2) ** 2)
    assert np.allclose(op.apply(phi), lam * phi, rtol=1e-12, atol=1e-12 * lam)


def _lap_rho(P, X, dp):
    """div_h(rho_f^-1 grad_h dp) written with face differences (explicit form)."""
    out = np.zeros_like(dp)
    for d in range(P.nd):
        gr = grad_face(P, X, dp, d)  # (dp[c]-dp[c-1])/(rho_f dx), zero on walls
        up = np.roll(gr, -1, axis=P.axis(d))
        if P.bc[d] == "wall":
            sl = [slice(None)] * P.nd
            sl[P.axis(d)] = -1
            up[tuple(sl)] = 0.0
        out += (up - gr) / P.dx[d]
    return out


def _div_chi(P, X, phi):
    op = thermal_operator(P, X, 1.0)
    return -(op.apply(phi) - op.diag * phi)


@pytest.mark.parametrize("theta", [1.0, 0.5])
@pytest.mark.parametrize("mode", ["sound", "sound_thermal"])
@pytest.mark.parametrize("shape,bc", [((8, 6), ("periodic", "wall")), ((4, 4, 6), ("periodic", "periodic", "wall"))])
def test_pbp_solves_semi_implicit_equations(mode, shape, bc, theta):
    """With direct elliptic solves, z = M^-1 r satisfies the semi-implicit equations in the
    explicit-Laplacian form (eqs. SI3_p..SI3_u; SI4_p_final..SI4_u_final with the conduction
    coupling of the pressure row lagged), the linearised EOS, and du = dt r_m/rho_f on walls.
    For a theta-step (J = dU/dX/dt - theta dR/dX) theta z satisfies them with the implicit
    time step theta dt."""
    P, X = _state(shape, bc, seed=3)
    P = dataclasses.replace(P, theta=theta)
    r = W.random_vector(X, 5)
    pbp = PBP(P, X, 0.2, mode)
    z = theta * pbp.apply(r)
    dt = theta * 0.2
    g = P.gamma
    rho, e = X[0], X[1]
    p = (g - 1) * rho * e
    dpdr, dpde = eos_derivs(P, X)
    dp = dpdr * z[0] + dpde * z[1]
    de = z[1]
    Fp, Fe, Fu = transform_in(P, X, r)
    L = _lap_rho(P, X, dp)
    scale = np.abs(Fp).max()
    assert np.allclose(dp / dt - g * p * dt * L, Fp, atol=1e-10 * scale)
    if mode == "sound":
        assert np.allclose(de / dt - (p / rho) * dt * L, Fe, atol=1e-10 * np.abs(Fe).max())
    else:
        cv = 1 / (g - 1)
        lhs = de / dt - (p / rho) * dt * L - _div_chi(P, X, de / cv) / rho
        assert np.allclose(lhs, Fe, atol=1e-10 * np.abs(Fe).max())
    for d in range(P.nd):
        rf = face_mean(P, rho, d)
        lhs = z[2 + d] / dt + grad_face(P, X, dp, d)
        assert np.allclose(lhs, Fu[d], atol=1e-10 * np.abs(Fu[d]).max())
        if P.bc[d] == "wall":
            sl = [slice(None)] * P.nd
            sl[P.axis(d)] = 0
            sl = tuple(sl)
            assert np.allclose(z[2 + d][sl], dt * r[2 + d][sl] / rf[sl])


@pytest.mark.parametrize("theta", [1.0, 0.5])
@pytest.mark.parametrize("mode", ["sound", "sound_thermal"])
def test_pbp_transpose_dot_product(mode, theta):
    P, X = _state((8, 6), ("periodic", "wall"), seed=4)
    P = dataclasses.replace(P, theta=theta)
    pbp = PBP(P, X, 0.15, mode)
    r = W.random_vector(X, 6)
    w = W.random_vector(X, 7)
    a = np.sum(w * pbp.apply(r))
    b = np.sum(pbp.apply_T(w) * r)
    assert abs(a - b) <= 1e-12 * (abs(a) + abs(b))


def _rest_state(shape, bc, seed):
    """Uniform rho, e at rest, no gravity, no conduction (a linearisation state where the
    eliminated system is exact)."""
    nd = len(shape)
    pd = W.make_problem(shape, tuple(1.0 / n for n in shape), bc, 1.4)
    rng = np.random.default_rng(seed)
    X = np.zeros((2 + nd,) + W.grid_shape(shape))
    X[0] = 1.0 + rng.uniform(0.5, 1.5)
    X[1] = 2.0 + rng.uniform(0.0, 1.0)
    return Problem.from_dict(pd), X


@pytest.mark.parametrize("theta", [1.0, 0.5])
@pytest.mark.parametrize("shape,bc", [((6, 5), ("periodic", "periodic")), ((5, 6), ("periodic", "wall")),
                                      ((4, 3, 4), ("periodic", "wall", "periodic"))])
def test_schur_pbp_is_exact_inverse_at_rest(shape, bc, theta):
    """At a uniform state at rest without gravity or conduction, eliminating du exactly makes
    the physics-based preconditioner the exact inverse of J (dense, complex step); the paper's
    J~_V, which drops F_u from the pressure equation, is not."""
    from oracle.jacobian import jacobian_dense_cs
    P, X = _rest_state(shape, bc, seed=11)
    P = dataclasses.replace(P, theta=theta)
    dt = 0.3
    b = rhs_b(P, X, dt)
    Jd = jacobian_dense_cs(P, X, b, dt)
    r = W.random_vector(X, 12, bc=P.bc)
    for schur, exact in ((True, True), (False, False)):
        z = PBP(P, X, dt, "sound", schur=schur).apply(r)
        back = (Jd @ z.ravel()).reshape(r.shape)
        err = np.max(np.abs(back - r)) / np.max(np.abs(r))
        if exact:
            assert err <= 1e-11, err
        else:
            assert err > 1e-3, err


@pytest.mark.parametrize("mode", ["sound", "sound_thermal"])
def test_schur_pbp_transpose_dot_product(mode):
    P, X = _state((8, 6), ("periodic", "wall"), seed=4)
    pbp = PBP(P, X, 0.15, mode, schur=True)
    r = W.random_vector(X, 6)
    w = W.random_vector(X, 7)
    a = np.sum(w * pbp.apply(r))
    b = np.sum(pbp.apply_T(w) * r)
    assert abs(a - b) <= 1e-12 * (abs(a) + abs(b))
