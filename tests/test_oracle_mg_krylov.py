"""Pins of the multigrid-preconditioned CG (Sect. 3.5 replacement) and of flexible GMRES
(Sects. 4.1, 4.3)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as W
from oracle.residual import Problem
from oracle.pbp import pressure_operator, thermal_operator
from oracle.mg import Multigrid, pcg
from oracle.krylov import fgmres


def _state(shape, bc, seed=1, amp=0.3):
    nd = len(shape)
    g = tuple([0.0] * (nd - 1) + [-1.0]) if "wall" in bc else None
    pd, X = W.random_state(shape, bc, seed=seed, g=g, chi_model="power", chi0=0.05, amp=amp)
    return Problem.from_dict(pd), X


def _stiff_dt(P, cfl=1000.0):
    return cfl * min(P.dx) / np.sqrt(1.4 * 0.4)


@pytest.mark.parametrize("shape,bc", [((8, 8), ("periodic", "periodic")), ((16, 8), ("periodic", "wall")),
                                      ((8, 8, 8), ("periodic", "periodic", "wall"))])
def test_vcycle_is_spd(shape, bc):
    P, X = _state(shape, bc)
    op = pressure_operator(P, X, _stiff_dt(P, 30.0))
    mg = Multigrid(op)
    assert len(mg.levels) >= 2
    N = P.ncell
    B = np.empty((N, N))
    for k in range(N):
        e = np.zeros(N)
        e[k] = 1.0
        B[:, k] = mg.vcycle(e.reshape(P.field_shape)).ravel()
    assert np.max(np.abs(B - B.T)) <= 1e-12 * np.max(np.abs(B))
    assert np.min(np.linalg.eigvalsh(0.5 * (B + B.T))) > 0


@pytest.mark.parametrize("eta", [1e-4, 1e-10])
def test_pcg_meets_stopping_rule_and_matches_direct(eta):
    P, X = _state((32, 32), ("periodic", "wall"), seed=2)
    op = pressure_operator(P, X, _stiff_dt(P, 100.0))
    b = np.random.default_rng(3).uniform(-1, 1, P.field_shape)
    its = []
    x = pcg(op, b, eta=eta, maxit=100, stats=its)
    A = op.to_sparse()
    res = np.linalg.norm(b.ravel() - A @ x.ravel())
    assert res < eta * np.linalg.norm(b)
    xd = spla.spsolve(A.tocsc(), b.ravel())
    ev = np.linalg.eigvalsh(A.toarray())
    cond = ev[-1] / ev[0]
    assert np.linalg.norm(x.ravel() - xd) <= eta * cond * np.linalg.norm(xd)
    assert its[0] < 40


def test_pcg_iterations_grid_independent():
    counts = []
    for n in (16, 32, 64, 128):
        P, X = _state((n, n), ("periodic", "wall"), seed=4, amp=0.2)
        op = pressure_operator(P, X, _stiff_dt(P, 1000.0))
        b = np.random.default_rng(5).uniform(-1, 1, P.field_shape)
        its = []
        pcg(op, b, eta=1e-8, maxit=100, stats=its)
        counts.append(its[0])
    assert max(counts) <= 30 and counts[-1] <= 2 * counts[0] + 4, counts


def test_pcg_fp32_variant():
    """FP32 operator, vectors and dots: the normalised solve reaches ~1e-5 relative accuracy."""
    P, X = _state((64, 64), ("periodic", "wall"), seed=6)
    op = thermal_operator(P, X, _stiff_dt(P, 100.0))
    b = 1e3 * np.random.default_rng(7).uniform(-1, 1, P.field_shape)
    x32 = pcg(op, b, eta=1e-4, dtype=np.float32)
    x64 = pcg(op, b, eta=1e-4)
    A = op.to_sparse()
    r32 = np.linalg.norm(b.ravel() - A @ x32.ravel()) / np.linalg.norm(b)
    assert r32 < 2e-4
    assert x32.dtype == np.float64
    assert np.linalg.norm(x32 - x64) / np.linalg.norm(x64) < 1e-3


def test_fgmres_small_exact():
    rng = np.random.default_rng(1)
    n = 20
    A = np.eye(n) * 4 + rng.uniform(-1, 1, (n, n))
    b = rng.uniform(-1, 1, n)
    rec = []
    x, info = fgmres(lambda z: A @ z, lambda v: v, b, eta=1e-14, m=30, record=rec)
    assert info["converged"] and info["iters"] <= n
    assert np.allclose(x, np.linalg.solve(A, b), rtol=0, atol=1e-12 * np.abs(x).max())
    cyc = rec[0]
    V = np.stack(cyc["V"], axis=1)
    Z = np.stack(cyc["Z"], axis=1)
    k = Z.shape[1]
    H = cyc["H"]
    # Arnoldi relation A Z_k = V_{k+1} H_k (happy breakdown may drop the last basis vector)
    AZ = A @ Z
    VH = V[:, : H.shape[0]] @ H[: V.shape[1]]
    assert np.max(np.abs(AZ - VH)) <= 1e-12 * np.max(np.abs(AZ))
    assert np.max(np.abs(V.T @ V - np.eye(V.shape[1]))) <= 1e-14


def test_fgmres_restart_and_residual_estimates():
    """Restarted FGMRES with a variable (noisy) preconditioner: residual estimates are
    non-increasing within a cycle and the reported convergence is real."""
    rng = np.random.default_rng(2)
    n = 80
    A = np.diag(np.linspace(1, 50, n)) + 0.3 * rng.uniform(-1, 1, (n, n))
    b = rng.uniform(-1, 1, n)
    D = np.diag(A)
    prec = lambda v: v / D * (1 + 1e-3 * rng.uniform(-1, 1, n))
    x, info = fgmres(lambda z: A @ z, prec, b, eta=1e-8, m=10, maxit=300)
    assert info["converged"]
    assert np.linalg.norm(b - A @ x) < 1e-8 * np.linalg.norm(b) * 1.0001


def test_single_vcycle_solve_is_a_symmetric_contraction():
    """maxit = 0 makes the elliptic solve the preconditioning V-cycle alone (x = M b): a fixed,
    symmetric operator whose error propagation I - M A is a contraction (spectral radius
    below 1, so M is a usable approximate inverse of A)."""
    P, X = _state((16, 8), ("periodic", "wall"), seed=5)
    op = pressure_operator(P, X, _stiff_dt(P, 30.0))
    N = P.ncell
    M = np.empty((N, N))
    for k in range(N):
        e = np.zeros(N)
        e[k] = 1.0
        M[:, k] = pcg(op, e.reshape(P.field_shape), maxit=0).ravel()
    assert np.max(np.abs(M - M.T)) <= 1e-12 * np.max(np.abs(M))
    A = op.to_sparse().toarray()
    rho = np.max(np.abs(np.linalg.eigvals(np.eye(N) - M @ A)))
    assert rho < 0.5, rho
    b = np.random.default_rng(6).uniform(-1, 1, P.field_shape)
    assert np.array_equal(pcg(op, b, maxit=0), Multigrid(op).vcycle(b.astype(np.float64)))


@pytest.mark.parametrize("shape,bc", [((9, 7), ("periodic", "wall")), ((16, 8), ("periodic", "wall")),
                                      ((5, 7, 6), ("wall", "periodic", "wall"))])
def test_vcycle_with_smoothed_bottom_is_spd(shape, bc, monkeypatch):
    """A coarsest level too large for the dense solve (here forced with a dense limit of 8
    cells; odd axes stop the coarsening at once) is smoothed instead of solved: the V-cycle
    stays a symmetric positive definite operator, and CG preconditioned by it still meets
    its stopping rule."""
    monkeypatch.setattr(Multigrid, "DENSE_MAX", 8)
    P, X = _state(shape, bc)
    op = pressure_operator(P, X, _stiff_dt(P, 30.0))
    mg = Multigrid(op)
    assert mg.coarse_chol is None
    N = P.ncell
    B = np.empty((N, N))
    for k in range(N):
        e = np.zeros(N)
        e[k] = 1.0
        B[:, k] = mg.vcycle(e.reshape(P.field_shape)).ravel()
    assert np.max(np.abs(B - B.T)) <= 1e-12 * np.max(np.abs(B))
    assert np.min(np.linalg.eigvalsh(0.5 * (B + B.T))) > 0
    b = np.random.default_rng(3).uniform(-1, 1, P.field_shape)
    its = []
    x = pcg(op, b, eta=1e-8, maxit=400, stats=its)
    assert np.linalg.norm(b.ravel() - op.to_sparse() @ x.ravel()) < 1e-8 * np.linalg.norm(b)


def test_level_cap():
    """max_levels caps the hierarchy (16^2 coarsens to 8^2 and 4^2 by itself).  One level: the
    V-cycle is the dense solve of the level itself, i.e. A^-1 b.  Two levels: still a symmetric
    positive definite operator, and CG preconditioned by it meets its stopping rule."""
    P, X = _state((16, 16), ("periodic", "wall"))
    op = pressure_operator(P, X, _stiff_dt(P, 30.0))
    assert [lev.prob.shape for lev in Multigrid(op).levels] == [(16, 16), (8, 8), (4, 4)]
    for L in (1, 2, 3, 7):
        assert len(Multigrid(op, max_levels=L).levels) == min(L, 3)
    A = op.to_sparse()
    b = np.random.default_rng(4).uniform(-1, 1, P.field_shape)
    x1 = Multigrid(op, max_levels=1).vcycle(b)
    xd = spla.spsolve(A.tocsc(), b.ravel())
    assert np.max(np.abs(x1.ravel() - xd)) <= 1e-11 * np.max(np.abs(xd))
    mg2 = Multigrid(op, max_levels=2)
    N = P.ncell
    B = np.empty((N, N))
    for k in range(N):
        e = np.zeros(N)
        e[k] = 1.0
        B[:, k] = mg2.vcycle(e.reshape(P.field_shape)).ravel()
    assert np.max(np.abs(B - B.T)) <= 1e-12 * np.max(np.abs(B))
    assert np.min(np.linalg.eigvalsh(0.5 * (B + B.T))) > 0
    its = []
    x = pcg(op, b, eta=1e-8, maxit=200, mg=mg2, stats=its)
    assert np.linalg.norm(b.ravel() - A @ x.ravel()) < 1e-8 * np.linalg.norm(b)



@pytest.mark.parametrize("degree", [1, 2, 3, 4])
def test_smoother_is_the_scaled_chebyshev_polynomial(degree):
    """k steps of the smoother from x = 0 give x = S b whose error propagator I - S A equals
    P_k(D^-1 A) with P_k(l) = T_k((theta - l)/delta) / T_k(theta/delta), theta = 1.25,
    delta = 0.75 (the interval [0.5, 2]): the closed form of the Chebyshev semi-iteration,
    evaluated through the eigenvectors of D^-1/2 A D^-1/2 and numpy's Chebyshev series."""
    from numpy.polynomial import chebyshev as C
    P, X = _state((6, 5), ("periodic", "wall"))
    op = pressure_operator(P, X, _stiff_dt(P, 30.0))
    mg = Multigrid(op, max_levels=1, degree=degree)
    lev = mg.levels[0]
    A = op.to_sparse().toarray()
    N = A.shape[0]
    S = np.empty((N, N))
    for k in range(N):
        e = np.zeros(N)
        e[k] = 1.0
        S[:, k] = mg.smooth(lev, e.reshape(P.field_shape), np.zeros(P.field_shape)).ravel()
    E = np.eye(N) - S @ A
    Dh = np.sqrt(np.diag(A))
    lam, Q = np.linalg.eigh(A / np.outer(Dh, Dh))
    coef = np.zeros(degree + 1)
    coef[degree] = 1.0
    p = C.chebval((1.25 - lam) / 0.75, coef) / C.chebval(1.25 / 0.75, coef)
    Eref = (Q * p) @ Q.T / Dh[:, None] * Dh[None, :]
    assert np.max(np.abs(E - Eref)) <= 1e-12
    # and the smoothing damps the upper part of the spectrum [0.5, 2] at least by T_k(5/3)^-1
    assert np.max(np.abs(p[lam >= 0.5])) <= 1.0 / C.chebval(1.25 / 0.75, coef) + 1e-12


@pytest.mark.parametrize("degree", [1, 3])
def test_vcycle_other_degrees_is_spd(degree):
    """The V-cycle with the degree-1 or degree-3 smoother is symmetric positive definite
    and preconditions CG to its stopping rule."""
    P, X = _state((16, 8), ("periodic", "wall"))
    op = pressure_operator(P, X, _stiff_dt(P, 30.0))
    mg = Multigrid(op, degree=degree)
    assert len(mg.levels) >= 2
    N = P.ncell
    B = np.empty((N, N))
    for k in range(N):
        e = np.zeros(N)
        e[k] = 1.0
        B[:, k] = mg.vcycle(e.reshape(P.field_shape)).ravel()
    assert np.max(np.abs(B - B.T)) <= 1e-12 * np.max(np.abs(B))
    assert np.min(np.linalg.eigvalsh(0.5 * (B + B.T))) > 0
    b = np.random.default_rng(5).uniform(-1, 1, P.field_shape)
    x = pcg(op, b, eta=1e-8, maxit=200, mg=mg)
    assert np.linalg.norm(b.ravel() - op.to_sparse() @ x.ravel()) < 1e-8 * np.linalg.norm(b)
