"""Parity at the full workload sizes, in the launch configuration bench.py times, on sampled
outputs the oracle computes one by one.

* F and exact J.v at sampled cells of the 256^3 convective box and the 128^3 Taylor-Green
  box (oracle evaluated only at the sampled cells);
* J^T w at sampled unknowns: the oracle perturbs one unknown by a complex step and reads its
  Jacobian column on the rows that can depend on it (a box of radius 3), then dots it with w;
* the finite-difference J.v at sampled cells, with the perturbation size from full-grid norms.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle.residual import Problem, residual_F, residual_R, conserved_U, cfl_dt, WALL
from oracle.jacobian import H_CS, fd_delta

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _lib():
    import paper_1512_03662_amd as J
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return J


def _rhs_b_cells(P, Xn, dt, cells):
    # b = U(X^n)/dt (theta = 1) at the sampled cells
    return conserved_U(P, Xn, cells) / dt


def _sample(P, k, seed):
    rng = np.random.default_rng(seed)
    cells = [rng.integers(0, P.shape[d], size=k) for d in range(P.nd)]
    # include boundary-adjacent cells on every axis
    for d in range(P.nd):
        cells[d][:2] = [0, P.shape[d] - 1]
    return tuple(cells)


def _at(A, P, cells):
    idx = tuple(np.asarray(cells[d]) for d in reversed(range(P.nd)))
    return np.stack([A[v][idx] for v in range(A.shape[0])])


def _workload(name):
    if name == "convective_3d_256":
        return W.convective_box_3d(n=256)
    return W.taylor_green_3d(n=128)


@pytest.mark.parametrize("name", ["convective_3d_256", "taylor_green_3d_128"])
def test_fullsize_residual_and_jv_sampled(name):
    J = _lib()
    w = _workload(name)
    pd, X = w["problem"], w["X0"]
    P = Problem.from_dict(pd)
    dt = cfl_dt(P, X, w["cfl"])
    # X^n: the same state slightly changed so that F(X) != 0
    Xn = X.copy()
    Xn[0] *= 1.0 + 1e-3 * np.sin(np.arange(Xn[0].size).reshape(Xn[0].shape) * 0.37)
    ctx = J.Context(pd, gmres_m=1, precond="none")
    Xg = torch.tensor(X, device=DEV)
    ctx.set_state_n(torch.tensor(Xn, device=DEV), dt)
    Fg = ctx.residual(Xg).cpu().numpy()
    rng = np.random.default_rng(77)
    v = rng.uniform(-1, 1, X.shape)
    Jvg = ctx.jvp(Xg, torch.tensor(v, device=DEV), "exact").cpu().numpy()
    cells = _sample(P, 48, 5)
    b = _rhs_b_cells(P, Xn, dt, cells)
    # residual at the sampled cells: F = U/dt - R - b
    F = conserved_U(P, X, cells) / dt - residual_R(P, X, cells) - b
    _, A = residual_R(P, X, cells, with_abs=True)
    U = conserved_U(P, X, cells)
    S = np.max(np.abs(U) / dt + np.abs(b), axis=1) + np.max(A, axis=1)
    err = np.max(np.abs(_at(Fg, P, cells) - F), axis=1) / S
    assert np.all(err <= 1e-12), err
    # exact J v at the sampled cells by the complex step
    Xc = X.astype(np.complex128) + 1j * H_CS * v
    Jv = np.imag(conserved_U(P, Xc, cells) / dt - residual_R(P, Xc, cells)) / H_CS
    errj = np.max(np.abs(_at(Jvg, P, cells) - Jv), axis=1) / S
    assert np.all(errj <= 1e-12), errj
    # finite-difference J v (pert_old with scaled norms) at the sampled cells
    Jfd = ctx.jvp(Xg, torch.tensor(v, device=DEV), "fd").cpu().numpy()
    delta = fd_delta(P, X, v)
    Xp = X + delta * v
    Jf = ((conserved_U(P, Xp, cells) / dt - residual_R(P, Xp, cells))
          - (conserved_U(P, X, cells) / dt - residual_R(P, X, cells))) / delta
    errf = np.max(np.abs(_at(Jfd, P, cells) - Jf), axis=1) / S
    assert np.all(errf <= 1e-7), errf


def _box_cells(P, c, r=3):
    """All cells within distance r of cell c (wrapped on periodic axes, clipped at walls)."""
    axes = []
    for d in range(P.nd):
        idx = np.arange(c[d] - r, c[d] + r + 1)
        if P.bc[d] == WALL:
            idx = idx[(idx >= 0) & (idx < P.shape[d])]
        else:
            idx = np.mod(idx, P.shape[d])
        axes.append(idx)
    grids = np.meshgrid(*axes, indexing="ij")
    return tuple(g.ravel() for g in grids)


@pytest.mark.parametrize("name", ["convective_3d_256"])
def test_fullsize_vjp_sampled(name):
    J = _lib()
    w = _workload(name)
    pd, X = w["problem"], w["X0"]
    P = Problem.from_dict(pd)
    dt = cfl_dt(P, X, w["cfl"])
    ctx = J.Context(pd, gmres_m=1, precond="none")
    Xg = torch.tensor(X, device=DEV)
    ctx.set_state_n(Xg, dt)
    rng = np.random.default_rng(78)
    wv = rng.uniform(-1, 1, X.shape)
    JTw = ctx.vjp(Xg, torch.tensor(wv, device=DEV)).cpu().numpy()
    Xc = X.astype(np.complex128)
    cells = _sample(P, 6, 9)
    for s in range(len(cells[0])):
        c = [int(cells[d][s]) for d in range(P.nd)]
        box = _box_cells(P, c)
        for var in range(P.nvar):
            idx = (var,) + tuple(c[d] for d in reversed(range(P.nd)))
            Xc[idx] += 1j * H_CS
            col = np.imag(conserved_U(P, Xc, box) / dt - residual_R(P, Xc, box)) / H_CS
            Xc[idx] -= 1j * H_CS
            wb = _at(wv, P, box)
            ref = float(np.sum(col * wb))
            scale = float(np.sum(np.abs(col * wb)))
            assert abs(JTw[idx] - ref) <= 1e-12 * scale + 1e-300, (c, var, JTw[idx], ref)


def test_fullsize_gradient_through_steps_fd():
    """The 512^2 adjoint workload (stratified box, chi ~ T^3, CFL 50, 5 steps): the gradient
    of the total kinetic energy w.r.t. the initial temperature through ImplicitSteps, against
    central differences of the forward steps along 8 seeded directions.  eps = 1e-7 and a bar
    of 3e-4: on 512^2 the difference quotient straddles a few upwind switches (measured
    errors 5e-6 .. 1e-4), which the exact gradient of the frozen branches does not see."""
    J = _lib()
    w = W.stratified_2d_kappa(n=512)
    pd, X0np = w["problem"], w["X0"]
    ctx = J.Context(pd, precond="sound_thermal", jv_mode="exact", newton_tol=1e-13, newton_max=30,
                    gmres_eta=1e-11, gmres_maxit=600, cg_eta=1e-8)
    X0 = torch.tensor(X0np, dtype=torch.float64, device=DEV)
    dt = ctx.cfl_dt(X0, w["cfl"])
    dts = [dt] * int(w["steps"])

    def ke(Xt):
        rho = Xt[0]
        tot = 0.0
        for d in range(2):
            ax = 1 - d
            lower = torch.roll(rho, 1, dims=ax)
            if pd["bc"][d] == "wall":
                idx = [slice(None)] * 2
                idx[ax] = 0
                lower[tuple(idx)] = rho[tuple(idx)]
            tot = tot + 0.5 * torch.sum(0.5 * (lower + rho) * Xt[2 + d] ** 2)
        return tot

    Xg = X0.clone().requires_grad_(True)
    ke(J.ImplicitSteps.apply(Xg, ctx, dts)).backward()
    grad_e = Xg.grad[1]
    eps = 1e-7
    for k in range(8):
        d = torch.tensor(W.random_vector(X0np[1:2], 2001 + k)[0], dtype=torch.float64, device=DEV)
        an = float(torch.sum(grad_e * X0[1] * d))
        vals = []
        for sgn in (1.0, -1.0):
            Xp = X0.clone()
            Xp[1] = X0[1] * (1.0 + sgn * eps * d)
            for dtk in dts:
                ctx.implicit_step(Xp, dtk)
            vals.append(float(ke(Xp)))
        fd = (vals[0] - vals[1]) / (2 * eps)
        assert abs(fd - an) <= 3e-4 * abs(an), (k, fd, an)
    ctx.close()


@pytest.mark.parametrize("form", ["fd_fp64", "exact_fp32"])
@pytest.mark.parametrize("name", ["convective_3d_256", "taylor_green_3d_128"])
def test_fullsize_first_step_is_a_root_of_the_oracle_residual(name, form):
    """The first implicit step of the 256^3 convective box (CFL 500) and of the 128^3
    Taylor-Green box (CFL 1000) in both forms, as bench.py runs them: at 4096 sampled cells
    (boundary cells included) the oracle's F at the GPU's X^1 (b from X^0) matches the
    library's F there to 1e-12 of S_k (operator parity at the converged state) and is itself
    below 1e-10 of S_k (X^1 is a root of the oracle's residual to the Newton tolerance; a wrong
    step leaves O(1e-6) or more), S_k = max(|U_k|/dt + |b_k|) + max A_k over the sampled cells."""
    J = _lib()
    w = _workload(name)
    pd, X0 = w["problem"], w["X0"]
    P = Problem.from_dict(pd)
    jv, ell = form.split("_")
    print(f"# full-size first step {name} {form}", flush=True)
    ctx = J.Context(pd, precond=w["precond"], jv_mode=jv, ell_precision=ell)
    Xg = torch.tensor(X0, dtype=torch.float64, device=DEV)
    dt = ctx.cfl_dt(Xg, w["cfl"])
    st = ctx.implicit_step(Xg, dt)
    assert st["converged"] == 1
    Xn = torch.tensor(X0, dtype=torch.float64, device=DEV)
    ctx.set_state_n(Xn, dt)
    Fg = ctx.residual(Xg).cpu().numpy()
    X1 = Xg.cpu().numpy()
    ctx.close()
    cells = _sample(P, 4096, 91)
    b = _rhs_b_cells(P, X0, dt, cells)
    U1 = conserved_U(P, X1, cells)
    R1, A1 = residual_R(P, X1, cells, with_abs=True)
    Fo = U1 / dt - R1 - b
    S = np.max(np.abs(U1) / dt + np.abs(b), axis=1) + np.max(A1, axis=1)
    par = float(np.max(np.max(np.abs(_at(Fg, P, cells) - Fo), axis=1) / S))
    root = float(np.max(np.max(np.abs(Fo), axis=1) / S))
    print(f"#   newton {st['newton_its']} gmres {st['gmres_its']}: F parity {par:.2e}, oracle F at X^1 {root:.2e}",
          flush=True)
    assert par <= 1e-12, par
    assert root <= 1e-10, root
