"""Pins of the oracle residual against properties the paper and the mathematics fix.

Conservative form (Sect. 2: finite volumes, conserved U): flux sums vanish on a periodic box.
Uniform states are steady.  The discretely balanced polytrope is an equilibrium.  Mirror and
axis-swap symmetry catch sign and index errors in the staggered stencil.  The stencil
footprint (radius 3) fixes the halo width of the GPU tiles.
"""
import numpy as np
import pytest

import workloads as W
from oracle.residual import Problem, residual_R, residual_F, rhs_b, conserved_U, cfl_dt


def _prob(pd):
    return Problem.from_dict(pd)


@pytest.mark.parametrize("shape,chi", [((8, 6), "const"), ((6, 5, 4), "power"), ((16, 16), "none")])
def test_conservation_periodic(shape, chi):
    """Sum of R_rho and R_m,d over a periodic box vanishes (no gravity)."""
    pd, X = W.random_state(shape, ("periodic",) * len(shape), seed=11, chi_model=chi, chi0=0.2)
    P = _prob(pd)
    R, A = residual_R(P, X, with_abs=True)
    sums = R.reshape(P.nvar, -1).sum(1)
    scale = A.reshape(P.nvar, -1).sum(1)
    assert abs(sums[0]) <= 1e-13 * scale[0]
    for d in range(P.nd):
        assert abs(sums[2 + d]) <= 1e-13 * scale[2 + d]


def test_conduction_conserves_energy_and_wall_flux():
    """u = 0: R_E is the divergence of the conductive flux.  Periodic: sums to 0; walls with
    prescribed fluxes: sum * cell volume = (q_hi - q_lo) * wall area."""
    pd, X = W.random_state((8, 6), ("periodic", "periodic"), seed=3, chi_model="power", chi0=0.3)
    X[2:] = 0.0
    P = _prob(pd)
    R, A = residual_R(P, X, with_abs=True)
    assert abs(R[1].sum()) <= 1e-13 * A[1].sum()
    qlo, qhi = 0.37, -0.21
    pd, X = W.random_state((6, 8), ("periodic", "wall"), seed=4, chi_model="const", chi0=0.3,
                           qwall=((0.0, 0.0), (qlo, qhi)))
    X[2:] = 0.0
    P = _prob(pd)
    R = residual_R(P, X)
    vol = P.dx[0] * P.dx[1]
    area = 1.0 * 1.0  # the box is the unit square: wall length 1
    assert np.isclose(R[1].sum() * vol, (qhi - qlo) * area, rtol=1e-12, atol=1e-14)
    # mass and momentum along the periodic axis are still conserved
    assert abs(R[0].sum()) < 1e-12 and abs(R[2].sum()) < 1e-12


@pytest.mark.parametrize("shape,bc", [((8, 8), ("periodic", "periodic")),
                                      ((4, 6, 8), ("periodic", "periodic", "periodic"))])
def test_uniform_state_is_steady(shape, bc):
    nd = len(shape)
    gs = W.grid_shape(shape)
    X = np.zeros((2 + nd,) + gs)
    X[0] = 1.7
    X[1] = 2.3
    for d in range(nd):
        X[2 + d] = 0.3 * (d + 1) - 0.5
    pd = W.make_problem(shape, tuple(1.0 / n for n in shape), bc, 1.4)
    P = _prob(pd)
    R = residual_R(P, X)
    assert np.all(R == 0.0)
    b = rhs_b(P, X, 0.1)
    assert np.all(np.abs(residual_F(P, X, b, 0.1)) <= 1e-15 * np.abs(b).max())


def test_pressure_equilibrium_bump():
    """Uniform p = 1 with a density bump at rest is steady up to rounding of p = (g-1) rho e."""
    w = W.acoustic_bump_2d(n=16)
    X = w["X0"].copy()
    P = _prob(w["problem"])
    X[1] = 1.0 / ((P.gamma - 1.0) * X[0])
    R, A = residual_R(P, X, with_abs=True)
    assert np.max(np.abs(R)) <= 1e-13 * np.max(A)


@pytest.mark.parametrize("chi", ["const"])
def test_hydrostatic_polytrope(chi):
    """The discretely balanced polytrope at rest has F(X^n) = 0 to rounding."""
    w = W.polytrope((16, 32), 10.0, mach=0.0, chi_model=chi, steps=1)
    P = _prob(w["problem"])
    X = w["X0"]
    dt = cfl_dt(P, X, 100.0)
    b = rhs_b(P, X, dt)
    F = residual_F(P, X, b, dt)
    _, A = residual_R(P, X, with_abs=True)
    for k in range(P.nvar):
        assert np.max(np.abs(F[k])) <= 1e-13 * np.max(A[k]), k


def _mirror_x(P, X):
    """Reflect x -> L - x: cells i -> n-1-i, x-faces i -> n-i (mod n), u_x changes sign."""
    ax = P.axis(0)
    Y = np.flip(X, axis=1 + ax).copy()
    ux = np.flip(X[2], axis=ax)
    Y[2] = -np.roll(ux, 1, axis=ax)
    return Y


def test_mirror_symmetry():
    pd, X = W.random_state((8, 6), ("periodic", "periodic"), seed=21, chi_model="const", chi0=0.1)
    P = _prob(pd)
    R = residual_R(P, X)
    Rm = residual_R(P, _mirror_x(P, X))
    assert np.allclose(Rm, _mirror_x(P, R), rtol=0, atol=1e-12 * np.abs(R).max())


def test_mirror_symmetry_3d_walls():
    pd, X = W.random_state((6, 5, 8), ("periodic", "periodic", "wall"), seed=22, g=(0, 0, -2.0),
                           chi_model="power", chi0=0.1, qwall=((0, 0), (0, 0), (0.1, -0.2)))
    P = _prob(pd)
    R = residual_R(P, X)
    Rm = residual_R(P, _mirror_x(P, X))
    assert np.allclose(Rm, _mirror_x(P, R), rtol=0, atol=1e-12 * np.abs(R).max())


def test_axis_swap_symmetry():
    """Swapping x and y on a square grid maps the residual consistently."""
    pd, X = W.random_state((8, 8), ("periodic", "periodic"), seed=23, chi_model="power", chi0=0.1)
    P = _prob(pd)
    R = residual_R(P, X)
    sw = lambda A: np.stack([A[0].T, A[1].T, A[3].T, A[2].T])
    Rs = residual_R(P, sw(X))
    assert np.allclose(Rs, sw(R), rtol=0, atol=1e-12 * np.abs(R).max())


def test_stencil_footprint_radius3():
    """Perturbing one cell changes residual rows only within [-3, +3] cells per axis, and the
    reach is exactly 3 (the momentum row sees rho three cells upstream through Phi_dd when
    the flow runs towards +d)."""
    pd, X = W.random_state((16, 16), ("periodic", "periodic"), seed=5)
    X[2:] = np.abs(X[2:]) + 0.1  # flow towards +x, +y: left-biased upwind states everywhere
    jj, ii = np.meshgrid(np.arange(16), np.arange(16), indexing="ij")
    X[0] = 1.0 + 0.02 * (ii + jj) + 0.001 * X[0]  # monotone around the probe: active limiter
    P = _prob(pd)
    R0 = residual_R(P, X)
    reach = 0
    for var in range(P.nvar):
        Y = X.copy()
        Y[var, 8, 8] += 1e-3
        dR = np.abs(residual_R(P, Y) - R0).max(axis=0)
        jj, ii = np.nonzero(dR > 0)
        reach = max(reach, np.abs(ii - 8).max(), np.abs(jj - 8).max())
    assert reach == 3
