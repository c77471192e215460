"""Pins of the oracle's spatial reconstruction against what Sect. 2 states about the
fluxes: upwind, monotonicity preserving after van Leer (1974), second order in space, TVD.

* hand-computed values of the van Leer harmonic slope and of the upwind face value, on
  both signs of the face velocity and at the tie w = 0 (left state);
* second-order convergence: for smooth periodic profiles advected by a uniform flow the
  mean absolute error of R_rho, of R_m along the flow (cell-centre momentum fluxes) and of
  R_m across it (edge momentum fluxes) falls by about 4 per halving of the spacing;
* TVD: one forward-Euler step at Courant number 1/4 of a step profile of rho, e or a
  sheared u creates no new extremum and does not raise the total variation, and moves the
  jump downstream (an upstream-biased update would do neither).
"""
import numpy as np
import pytest

from oracle import residual as OR
from oracle.residual import Problem, residual_R


# ---- hand values ----------------------------------------------------------------------
def test_van_leer_slope_hand_values():
    # 2ab/(a+b) if ab > 0, else 0
    assert OR.vl(np.array(1.0), np.array(3.0)) == pytest.approx(1.5, abs=0, rel=1e-15)
    assert OR.vl(np.array(2.0), np.array(2.0)) == pytest.approx(2.0, abs=0, rel=1e-15)
    assert OR.vl(np.array(-1.0), np.array(-4.0)) == pytest.approx(-1.6, abs=0, rel=1e-15)
    assert OR.vl(np.array(1.0), np.array(-1.0)) == 0.0
    assert OR.vl(np.array(0.0), np.array(5.0)) == 0.0
    assert OR.vl(np.array(5.0), np.array(0.0)) == 0.0
    # bounded by twice the smaller slope (the monotonicity bound of the harmonic limiter)
    a = np.array([0.1, 1.0, 10.0])
    b = np.array([10.0, 1.0, 0.1])
    assert np.all(OR.vl(a, b) <= 2.0 * np.minimum(a, b) + 1e-15)


@pytest.mark.parametrize("w, expect", [
    (+1.0, 1.0 + 0.5 * (2.0 * 1.0 * 2.0 / 3.0)),   # left: q[c-1] + vl(q[c-1]-q[c-2], q[c]-q[c-1])/2
    (0.0, 1.0 + 0.5 * (2.0 * 1.0 * 2.0 / 3.0)),    # tie: the left state
    (-1.0, 3.0 - 0.5 * (2.0 * 2.0 * 1.0 / 3.0)),   # right: q[c] - vl(q[c]-q[c-1], q[c+1]-q[c])/2
])
def test_upwind_face_value_hand(w, expect):
    qm2, qm1, q0, qp1 = (np.array(v) for v in (0.0, 1.0, 3.0, 4.0))
    assert OR.upwind(qm2, qm1, q0, qp1, np.array(w)) == pytest.approx(expect, abs=0, rel=1e-15)


def test_upwind_face_value_at_an_extremum_is_first_order():
    # q[c-1] is a local maximum: the left slope is clipped to zero, the face takes q[c-1]
    qm2, qm1, q0, qp1 = (np.array(v) for v in (0.0, 2.0, 1.0, 0.5))
    assert OR.upwind(qm2, qm1, q0, qp1, np.array(1.0)) == 2.0
    # right state: slopes (q0-qm1, qp1-q0) = (-1, -0.5), vl = -2/3
    assert OR.upwind(qm2, qm1, q0, qp1, np.array(-1.0)) == pytest.approx(1.0 + 1.0 / 3.0, rel=1e-15)


# ---- second-order convergence of smooth advection ---------------------------------------
def _box(n):
    h = 1.0 / n
    return Problem(shape=(n, n), dx=(h, h), bc=("periodic", "periodic"), gamma=1.4, g=(0.0, 0.0)), h


def _smooth_case(n, kind):
    """State, the exact row at the sample points, and the variable index."""
    P, h = _box(n)
    xc = (np.arange(n) + 0.5) * h
    xf = np.arange(n) * h
    X = np.zeros((4, n, n))
    X[0] = 1.0
    X[1] = 1.0
    ones = np.ones((n, n))
    if kind == "mass":        # rho(x) carried by u_x = 1: R_rho = -d rho/dx
        X[0] = (2.0 + np.sin(2 * np.pi * xc))[None, :] * ones
        X[2] = 1.0
        exact = -2 * np.pi * np.cos(2 * np.pi * xc)[None, :] * ones
        var = 0
    elif kind == "momentum_along":   # rho = 1, u_x(x) > 0: R_m,x = -d(u_x^2)/dx at the faces
        u = 1.0 + 0.1 * np.sin(2 * np.pi * xf)
        X[2] = u[None, :] * ones
        exact = (-2.0 * u * 0.2 * np.pi * np.cos(2 * np.pi * xf))[None, :] * ones
        var = 2
    else:                     # shear: u_x(y) carried by u_y = 1 through the edge fluxes
        X[3] = 1.0
        X[2] = (1.0 + 0.1 * np.sin(2 * np.pi * xc))[:, None] * ones
        exact = (-0.2 * np.pi * np.cos(2 * np.pi * xc))[:, None] * ones
        var = 2
    return P, X, exact, var


@pytest.mark.parametrize("kind", ["mass", "momentum_along", "momentum_across"])
def test_smooth_advection_is_second_order(kind):
    errs = []
    for n in (32, 64, 128):
        P, X, exact, var = _smooth_case(n, kind)
        errs.append(float(np.mean(np.abs(residual_R(P, X)[var] - exact))))
    ratios = [errs[0] / errs[1], errs[1] / errs[2]]
    # second order: 4 per halving (3.7-3.9 at these sizes, the limiter clips at the extrema);
    # a first-order reconstruction gives 2
    assert all(3.5 < r < 4.5 for r in ratios), (errs, ratios)


# ---- TVD -------------------------------------------------------------------------------
def _tv(a):
    return float(np.sum(np.abs(a - np.roll(a, 1))))


def _step_profile(n, lo, hi, a=0.3, b=0.7):
    x = (np.arange(n) + 0.5) / n
    return np.where((x > a) & (x < b), hi, lo)


@pytest.mark.parametrize("what", ["rho", "e", "u_sheared"])
def test_one_explicit_step_of_a_jump_is_tvd(what):
    n = 64
    P, h = _box(n)
    dt = 0.25 * h   # Courant number 1/4 at unit speed
    X = np.zeros((4, n, n))
    X[0] = 1.0
    X[1] = 1.0
    if what == "rho":
        X[0] = _step_profile(n, 1.0, 2.0)[None, :] * np.ones((n, n))
        X[2] = 1.0
        before = X[0, 0].copy()
        after = (X[0] + dt * residual_R(P, X)[0])[0]
    elif what == "e":
        X[1] = _step_profile(n, 1.0, 3.0)[None, :] * np.ones((n, n))
        X[2] = 1.0
        before = X[1, 0].copy()
        after = ((X[0] * X[1] + dt * residual_R(P, X)[1]) / X[0])[0]
    else:   # u_x(y), carried along y by u_y = 1 (rho = 1: rho_f = 1)
        X[3] = 1.0
        X[2] = _step_profile(n, 1.0, 1.5)[:, None] * np.ones((n, n))
        before = X[2, :, 0].copy()
        after = (X[2] + dt * residual_R(P, X)[2])[:, 0]
    tol = 1e-13
    assert after.min() >= before.min() - tol and after.max() <= before.max() + tol, (after.min(), after.max())
    assert _tv(after) <= _tv(before) + tol
    # the raised region moves downstream (+ along the flow): its first cell falls, the cell
    # after its last one rises, and the cell before it (low on both of its faces) is unchanged
    raised = np.where(before > before.min())[0]
    i0, i1 = int(raised[0]), int(raised[-1])
    assert after[i0] < before[i0] - 1e-3
    assert after[i1 + 1] > before[i1 + 1] + 1e-3
    assert abs(after[i0 - 1] - before[i0 - 1]) <= tol
