"""Pins of the oracle Jacobian products (Sect. 4.2).

The complex-step product is checked against an independent brute-force central-difference
dense Jacobian; the coloured sparse Jacobian against the dense one and against complex-step
products on grids where colouring groups many cells; the finite-difference product of
eq. jacobian_free converges to the exact product at first order in delta.
"""
import numpy as np
import pytest

import workloads as W
from oracle.residual import Problem, rhs_b
from oracle.jacobian import (jacobian_dense_central, jacobian_dense_cs, jacobian_sparse,
                             jvp_cs, jvp_fd, fd_delta)
from oracle.scaling import scaling_LR

CASES = [
    dict(shape=(6, 5), bc=("periodic", "periodic")),
    dict(shape=(5, 6), bc=("periodic", "wall"), g=(0.0, -1.5), chi_model="const", chi0=0.2,
         qwall=((0, 0), (0.3, -0.1))),
    dict(shape=(4, 5, 6), bc=("periodic", "periodic", "wall"), g=(0, 0, -1.0), chi_model="power",
         chi0=0.1, qwall=((0, 0), (0, 0), (0.2, 0.1))),
]


def _case(i, seed=7):
    c = dict(CASES[i])
    pd, X = W.random_state(c.pop("shape"), c.pop("bc"), seed=seed, **c)
    return Problem.from_dict(pd), X


@pytest.mark.parametrize("i", range(len(CASES)))
def test_complex_step_matches_central_difference(i):
    P, X = _case(i)
    dt = 0.02
    b = rhs_b(P, X, dt)
    Jc = jacobian_dense_cs(P, X, b, dt)
    Jd = jacobian_dense_central(P, X, b, dt)
    assert np.max(np.abs(Jc - Jd)) <= 1e-7 * np.max(np.abs(Jc))


@pytest.mark.parametrize("i", range(len(CASES)))
def test_sparse_coloured_equals_dense(i):
    P, X = _case(i)
    dt = 0.02
    b = rhs_b(P, X, dt)
    Jc = jacobian_dense_cs(P, X, b, dt)
    Js = jacobian_sparse(P, X, b, dt).toarray()
    assert np.max(np.abs(Jc - Js)) <= 1e-14 * np.max(np.abs(Jc))


@pytest.mark.parametrize("shape,bc", [((16, 24), ("periodic", "wall")),
                                      ((16, 8, 8), ("periodic", "periodic", "periodic"))])
def test_sparse_coloured_product_large(shape, bc):
    """Colouring with period 8 (several cells per colour) reproduces complex-step J v."""
    nd = len(shape)
    g = tuple([0.0] * (nd - 1) + [-1.0])
    pd, X = W.random_state(shape, bc, seed=9, g=g, chi_model="const", chi0=0.1)
    P = Problem.from_dict(pd)
    dt = 0.05
    b = rhs_b(P, X, dt)
    v = W.random_vector(X, 10)
    Js = jacobian_sparse(P, X, b, dt)
    Jv = jvp_cs(P, X, b, dt, v)
    assert np.max(np.abs(Js @ v.ravel() - Jv.ravel())) <= 1e-13 * np.max(np.abs(Jv))


def test_complex_step_is_linear_at_exact_ties():
    """The frozen-branch product must be linear in the direction, also on states with exact
    ties (Taylor-Green at Mach 1e-6 has u = 0 on whole planes, so mass fluxes vanish
    exactly): J(v1 + v2) = J v1 + J v2 for directions mixing density and velocity."""
    w = W.taylor_green_3d(n=8, mach=1e-6)
    P = Problem.from_dict(w["problem"])
    X = w["X0"]
    dt = 10.0
    b = rhs_b(P, X, dt)
    rng = np.random.default_rng(3)
    v1 = np.zeros_like(X)
    v2 = np.zeros_like(X)
    v1[0] = rng.uniform(-1, 1, X[0].shape)
    v2[2:] = rng.uniform(-1, 1, X[2:].shape)
    J1, J2, J12 = jvp_cs(P, X, b, dt, v1), jvp_cs(P, X, b, dt, v2), jvp_cs(P, X, b, dt, v1 + v2)
    scale = np.abs(J1).max() + np.abs(J2).max()
    assert np.max(np.abs(J12 - J1 - J2)) <= 1e-14 * scale


def test_fd_product_first_order():
    P, X = _case(1)
    dt = 0.02
    b = rhs_b(P, X, dt)
    v = W.random_vector(X, 3)
    Jv = jvp_cs(P, X, b, dt, v)
    errs = []
    for lam in (1e-3, 1e-4):
        errs.append(np.max(np.abs(jvp_fd(P, X, b, dt, v, lam=lam) - Jv)) / np.max(np.abs(Jv)))
    assert 5.0 < errs[0] / errs[1] < 20.0
    # the paper's lam = 1e-7 gives a product accurate to ~1e-7 relative
    e7 = np.max(np.abs(jvp_fd(P, X, b, dt, v, lam=1e-7) - Jv)) / np.max(np.abs(Jv))
    assert e7 < 1e-6


def test_fd_delta_is_scale_free():
    """delta uses scaled norms: rescaling the unknowns' units leaves it unchanged
    when R rescales with them (rho by s scales R_rho by s)."""
    P, X = _case(0)
    v = W.random_vector(X, 4)
    d1 = fd_delta(P, X, v)
    lam = 1e-7
    _, R = scaling_LR(P, X)
    expect = lam * (lam + np.linalg.norm(X / R) / np.linalg.norm(v / R))
    assert np.isclose(d1, expect, rtol=1e-15)
    # rho -> s rho, v_rho -> s v_rho: scaled vectors unchanged
    Y, w = X.copy(), v.copy()
    Y[0] *= 3.0
    w[0] *= 3.0
    # sound speed depends on e only, so R_u is unchanged
    assert np.isclose(fd_delta(P, Y, w), d1, rtol=1e-14)
