"""GPU parity with the gas + radiation equation of state (a_rad > 0) against the oracle.

Same bars as the ideal-gas parity tests: residual and exact J.v <= 1e-12 of the per-variable
scale, finite-difference J.v <= 1e-7, preconditioner (sound, sound + thermal, Schur variant,
and its transpose) <= 1e-10 with tight inner solves, J^T w element by element <= 1e-12 of
|J|^T |w|, converged steps and adjoint steps <= 1e-8 against the oracle's exact roots.  The
random states put radiation pressure at a sizeable fraction of the gas pressure, so that
Gamma1, Gamma3 and c_v differ from their ideal-gas values.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import eos
from oracle.residual import Problem, residual_F, rhs_b, residual_scale, cfl_dt
from oracle.jacobian import jvp_cs, jvp_fd, jacobian_sparse
from oracle.scaling import scaling_LR
from oracle.pbp import PBP
from oracle.adjoint import adjoint_step_exact
from oracle.newton import exact_step

from test_gpu_parity import TINY, T, H, _sample_err  # noqa: E402

pytestmark = pytest.mark.gpu

A_RAD = 30.0


def _lib():
    import paper_1512_03662_amd as J
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return J


def _rad(name_cfg, seed):
    name, c = name_cfg
    c = dict(c)
    pd, X = W.random_state(c.pop("shape"), c.pop("bc"), seed=seed, a_rad=A_RAD, **c)
    P = Problem.from_dict(pd)
    T_ = eos.temperature(P, X[0], X[1])
    assert np.min(A_RAD * T_ ** 3 / (3 * X[0])) > 0.1  # p_rad / p_gas
    return pd, P, X


@pytest.mark.parametrize("case", TINY, ids=[c[0] for c in TINY])
def test_residual_parity_radiation(case):
    J = _lib()
    pd, P, X = _rad(case, 7)
    Xn = X.copy()
    Xn[0] *= 1.01
    dt = 0.03
    b = rhs_b(P, Xn, dt)
    F = residual_F(P, X, b, dt)
    S = residual_scale(P, X, b, dt)
    ctx = J.Context(pd)
    ctx.set_state_n(T(Xn), dt)
    assert _sample_err(H(ctx.residual(T(X))), F, S) <= 1e-12


@pytest.mark.parametrize("case", TINY, ids=[c[0] for c in TINY])
def test_exact_jvp_parity_radiation(case):
    J = _lib()
    pd, P, X = _rad(case, 8)
    dt = 0.03
    b = rhs_b(P, X, dt)
    v = W.random_vector(X, 9)
    ref = jvp_cs(P, X, b, dt, v)
    ctx = J.Context(pd)
    ctx.set_state_n(T(X), dt)
    got = H(ctx.jvp(T(X), T(v), mode="exact"))
    assert _sample_err(got, ref, residual_scale(P, X, b, dt)) <= 1e-12


@pytest.mark.parametrize("case", TINY[:3], ids=[c[0] for c in TINY[:3]])
def test_fd_jvp_parity_radiation(case):
    J = _lib()
    pd, P, X = _rad(case, 10)
    dt = 0.03
    b = rhs_b(P, X, dt)
    v = W.random_vector(X, 11)
    ref = jvp_fd(P, X, b, dt, v, lam=1e-7)
    ctx = J.Context(pd)
    ctx.set_state_n(T(X), dt)
    got = H(ctx.jvp(T(X), T(v), mode="fd"))
    assert _sample_err(got, ref, residual_scale(P, X, b, dt)) <= 1e-7


@pytest.mark.parametrize("case", TINY, ids=[c[0] for c in TINY])
def test_vjp_parity_radiation(case):
    J = _lib()
    pd, P, X = _rad(case, 21)
    dt = 0.03
    b = rhs_b(P, X, dt)
    w = W.random_vector(X, 22)
    Jm = jacobian_sparse(P, X, b, dt)
    ref = (Jm.T @ w.ravel()).reshape(X.shape)
    scale = (abs(Jm).T @ np.abs(w.ravel())).reshape(X.shape)
    ctx = J.Context(pd)
    ctx.set_state_n(T(X), dt)
    got = H(ctx.vjp(T(X), T(w)))
    assert np.all(np.abs(got - ref) <= 1e-12 * scale + 1e-300)


PC_CASES = [("sound", 0), ("sound_thermal", 0), ("sound", 1), ("sound_thermal", 1)]


@pytest.mark.parametrize("a_rad", [0.0, A_RAD], ids=["ideal", "radiation"])
@pytest.mark.parametrize("mode,schur", PC_CASES, ids=[f"{m}-schur{s}" for m, s in PC_CASES])
@pytest.mark.parametrize("shape,bc", [((32, 16), ("periodic", "wall")), ((8, 8, 16), ("periodic", "periodic", "wall"))])
def test_precond_and_transpose_parity(mode, schur, shape, bc, a_rad):
    """M^-1 r and M^-T r (the adjoint's preconditioner, through its own entry point)."""
    J = _lib()
    nd = len(shape)
    pd, X = W.random_state(shape, bc, seed=12, g=tuple([0.0] * (nd - 1) + [-1.0]), chi_model="power",
                           chi0=0.02, amp=0.2, a_rad=a_rad)
    P = Problem.from_dict(pd)
    dt = 0.05
    r = W.random_vector(X, 13)
    pbp = PBP(P, X, dt, mode, schur=bool(schur))
    ctx = J.Context(pd, precond=mode, pc_schur=schur, cg_eta=1e-13, cg_maxit=200)
    ctx.set_state_n(T(X), dt)
    ref = pbp.apply(r)
    got = H(ctx.precond_apply(T(X), T(r)))
    for k in range(P.nvar):
        assert np.max(np.abs(got[k] - ref[k])) <= 1e-10 * np.max(np.abs(ref[k])), k
    refT = pbp.apply_T(r)
    gotT = H(ctx.precond_apply_transpose(T(X), T(r)))
    for k in range(P.nvar):
        assert np.max(np.abs(gotT[k] - refT[k])) <= 1e-10 * np.max(np.abs(refT[k])), k


def test_implicit_step_radiative_polytrope():
    J = _lib()
    w = W.radiative_2d(n=16, seed=5, cfl=50.0)
    pd, X0 = w["problem"], w["X0"]
    P = Problem.from_dict(pd)
    dt = cfl_dt(P, X0, w["cfl"])
    ctx = J.Context(pd, precond="sound_thermal", jv_mode="fd")
    Xg = T(X0)
    assert abs(ctx.cfl_dt(Xg, w["cfl"]) - dt) <= 1e-14 * dt
    st = ctx.implicit_step(Xg, dt)
    assert st["converged"] == 1, st
    Xs, _ = exact_step(P, X0, dt)
    _, R = scaling_LR(P, Xs)
    err = np.max(np.abs((H(Xg) - Xs) / R))
    assert err <= 1e-8, (err, st)


def test_adjoint_step_parity_radiation():
    J = _lib()
    w = W.radiative_2d(n=16, seed=5, cfl=50.0)
    pd, X0 = w["problem"], w["X0"]
    P = Problem.from_dict(pd)
    dt = cfl_dt(P, X0, 10.0)
    Xs, _ = exact_step(P, X0, dt)
    gbar = W.random_vector(X0, 31)
    ref, _ = adjoint_step_exact(P, Xs, X0, dt, gbar)
    ctx = J.Context(pd, precond="sound_thermal", gmres_eta=1e-12, cg_eta=1e-6)
    got, st = ctx.adjoint_step(T(Xs), T(X0), dt, T(gbar))
    got = H(got)
    assert st["converged"] == 1
    assert np.max(np.abs(got - ref)) <= 1e-8 * np.max(np.abs(ref)), (np.max(np.abs(got - ref)), st)
