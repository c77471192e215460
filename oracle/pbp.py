"""Oracle: physics-based preconditioner (semi-implicit scheme used as right preconditioner).

TEST INFRASTRUCTURE ONLY.

Follows Sect. 4.3 (the four-step algorithm: transform the U-residual to primitive variables,
apply the semi-implicit scheme, transform back) with the semi-implicit schemes of Sect. 3.3
(sound waves: eqs. SI3_p, SI3_e, SI3_u and the identity that replaces the Laplacian of dp in
the energy row) and Sect. 3.4 (sound + thermal diffusion, eqs. SI4_p_final..SI4_u_final),
and the transformation matrices of Sect. 3.2 (internal-energy form, derived in App. B).

Readings where the paper is silent:
* the operator maps r -> z ~ +J^-1 r (the paper's delta form gives -J^-1 r);
* coefficients are frozen at the current Newton iterate;
* the pressure row is row-scaled by 1/(Gamma1 p) so that
  A_p = diag(1/(Gamma1 p dt)) - dt div_h(rho_f^-1 grad_h) is symmetric positive definite
  (it equals the paper's 1/dt - a^2 dt d^2/dx^2 divided by Gamma1 p for uniform rho);
* thermal diffusion: one block Gauss-Seidel sweep, pressure first with the conduction
  coupling lagged, then A_T dT = rho Fe + (dp/dt - Fp)/Gamma1 with
  A_T = diag(rho c_v/dt) - div_h(chi_f grad_h) and de = c_v dT (dT ~ de/c_v, Sect. 3.4);
* wall faces: zero face weights (homogeneous Neumann) and du = dt r_m/rho_f there (the
  inverse of the diagonal Jacobian row of a wall face).

The elliptic systems are solved here directly (scipy splu) or by ``mg.pcg`` (the same
multigrid-preconditioned CG the GPU uses).

Pins (tests/test_oracle_scaling_pbp.py): symmetry and positivity of A_p, A_T; Fourier eigenvalues
for constant coefficients; the identity-based energy update equals the explicit Laplacian
form; transformation matrix identities of App. B; M^-1 equals the exact inverse of the
linearised semi-implicit system written out densely; the transposed operator passes the
dot-product test.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import eos
from .residual import Problem, WALL


def _roll(a, prob, d, k):
    """a[c + k e_d] with periodic wrap (wall handling is done by the caller)."""
    return np.roll(a, -k, axis=prob.axis(d))


def _wall_slice(prob, d, idx):
    sl = [slice(None)] * prob.nd
    sl[prob.axis(d)] = idx
    return tuple(sl)


def face_mean(prob: Problem, q, d):
    """0.5 (q[c - e_d] + q[c]) on the low-d faces; mirror ghost at a wall."""
    lower = _roll(q, prob, d, -1)
    if prob.bc[d] == WALL:
        lower[_wall_slice(prob, d, 0)] = q[_wall_slice(prob, d, 0)]
    return 0.5 * (lower + q)


class EllOp:
    """Variable-coefficient operator (A phi)[c] = diag phi - sum_d [w_d[c+1](phi[c+1]-phi[c])
    - w_d[c](phi[c]-phi[c-1])], w_d on low-d faces (zero on wall faces), 5/7-point stencil."""

    def __init__(self, prob: Problem, diag, w):
        self.prob = prob
        self.diag = diag
        self.w = w  # list over d of face weights

    def face_flux(self, phi, d):
        prob = self.prob
        return self.w[d] * (phi - _roll(phi, prob, d, -1))

    def apply(self, phi):
        prob = self.prob
        out = self.diag * phi
        for d in range(prob.nd):
            fl = self.face_flux(phi, d)
            fl_up = _roll(fl, prob, d, 1)
            if prob.bc[d] == WALL:
                fl_up[_wall_slice(prob, d, -1)] = 0.0
            out = out - (fl_up - fl)
        return out

    def dinv(self):
        """1/diag(A)."""
        prob = self.prob
        D = self.diag.copy()
        for d in range(prob.nd):
            w_up = _roll(self.w[d], prob, d, 1)
            if prob.bc[d] == WALL:
                w_up[_wall_slice(prob, d, -1)] = 0.0
            D = D + self.w[d] + w_up
        return 1.0 / D

    def to_sparse(self):
        prob = self.prob
        fs = prob.field_shape
        N = prob.ncell
        lin = np.arange(N).reshape(fs)
        rows = [lin.ravel()]
        cols = [lin.ravel()]
        vals = [self.diag.ravel().astype(np.float64)]
        for d in range(prob.nd):
            w = self.w[d].astype(np.float64)
            lower = _roll(lin, prob, d, -1)
            # each face couples c-1 and c with weight w: +w on both diagonals, -w off-diagonal
            rows += [lin.ravel(), lower.ravel(), lin.ravel(), lower.ravel()]
            cols += [lin.ravel(), lower.ravel(), lower.ravel(), lin.ravel()]
            vals += [w.ravel(), w.ravel(), -w.ravel(), -w.ravel()]
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(N, N))


def _zero_wall_faces(prob, w):
    for d in range(prob.nd):
        if prob.bc[d] == WALL:
            w[d][_wall_slice(prob, d, 0)] = 0.0
    return w


def pressure_operator(prob: Problem, X, dt):
    """A_p = diag(1/(Gamma1 p dt)) - dt div_h(rho_f^-1 grad_h)  (Sect. 3.3, row-scaled)."""
    p, _, _, _, G1, _ = eos.thermo(prob, X[0], X[1])
    diag = 1.0 / (G1 * p * dt)
    w = [dt / (face_mean(prob, X[0], d) * prob.dx[d] ** 2) for d in range(prob.nd)]
    return EllOp(prob, diag, _zero_wall_faces(prob, w))


def chi_cells(prob: Problem, X):
    T = eos.temperature(prob, X[0], X[1])
    if prob.chi_model == "none":
        return np.zeros_like(T)
    if prob.chi_model == "const":
        return np.full_like(T, prob.chi0)
    return prob.chi0 * (T / prob.chi_tref) ** prob.chi_exp


def thermal_operator(prob: Problem, X, dt):
    """A_T = diag(rho c_v/dt) - div_h(chi_f grad_h)  (Sect. 3.4 with dT = de/c_v,
    c_v = de/dT|_rho)."""
    cv = eos.thermo(prob, X[0], X[1])[5]
    diag = X[0] * cv / dt
    chi = chi_cells(prob, X)
    w = [face_mean(prob, chi, d) / prob.dx[d] ** 2 for d in range(prob.nd)]
    return EllOp(prob, diag, _zero_wall_faces(prob, w))


def eos_derivs(prob: Problem, X):
    """dp/drho|_e and dp/de|_rho (App. A; ideal gas: (gamma-1) e and (gamma-1) rho)."""
    _, _, dpdr, dpde, _, _ = eos.thermo(prob, X[0], X[1])
    return dpdr, dpde


def transform_in(prob: Problem, X, r):
    """F_V = dV/dU r (Sect. 3.2, internal energy form), velocity rows on faces."""
    rho, e = X[0], X[1]
    dpdr, dpde = eos_derivs(prob, X)
    Fp = (dpdr - (e / rho) * dpde) * r[0] + (dpde / rho) * r[1]
    Fe = (r[1] - e * r[0]) / rho
    Fu = []
    for d in range(prob.nd):
        rf = face_mean(prob, rho, d)
        rbar = face_mean(prob, r[0], d)
        Fu.append((r[2 + d] - X[2 + d] * rbar) / rf)
    return Fp, Fe, Fu


def transform_in_T(prob: Problem, X, Fp_b, Fe_b, Fu_b):
    """Transpose of transform_in: returns r_bar."""
    rho, e = X[0], X[1]
    dpdr, dpde = eos_derivs(prob, X)
    rb = np.zeros((prob.nvar,) + prob.field_shape)
    rb[0] = (dpdr - (e / rho) * dpde) * Fp_b - (e / rho) * Fe_b
    rb[1] = (dpde / rho) * Fp_b + Fe_b / rho
    for d in range(prob.nd):
        rf = face_mean(prob, rho, d)
        rb[2 + d] = Fu_b[d] / rf
        a = -X[2 + d] * Fu_b[d] / rf  # coefficient on rbar at each face
        # rbar[c] = 0.5 (r0[c-1] + r0[c]); at a wall face 0 the ghost r0[-1] = r0[0]
        up = _roll(a, prob, d, 1)
        if prob.bc[d] == WALL:
            up[_wall_slice(prob, d, -1)] = 0.0
            lowfix = np.zeros_like(a)
            lowfix[_wall_slice(prob, d, 0)] = a[_wall_slice(prob, d, 0)]
            rb[0] += 0.5 * (a + up) + 0.5 * lowfix
        else:
            rb[0] += 0.5 * (a + up)
    return rb


def grad_face(prob: Problem, X, phi, d):
    """(phi[c] - phi[c-1]) / (rho_f dx_d) on the low-d faces, zero on wall faces."""
    rf = face_mean(prob, X[0], d)
    gr = (phi - _roll(phi, prob, d, -1)) / (rf * prob.dx[d])
    if prob.bc[d] == WALL:
        gr[_wall_slice(prob, d, 0)] = 0.0
    return gr


def grad_face_T(prob: Problem, X, a, d):
    """Transpose of grad_face."""
    rf = face_mean(prob, X[0], d)
    c = a / (rf * prob.dx[d])
    if prob.bc[d] == WALL:
        c = c.copy()
        c[_wall_slice(prob, d, 0)] = 0.0
    up = _roll(c, prob, d, 1)
    if prob.bc[d] == WALL:
        up[_wall_slice(prob, d, -1)] = 0.0
    return c - up


def div_face(prob: Problem, F, d):
    """(F[c + e_d] - F[c]) / dx_d of values F on the low-d faces; wall faces (the low face of
    the first cell and the high face of the last) carry zero."""
    Fz = F
    if prob.bc[d] == WALL:
        Fz = F.copy()
        Fz[_wall_slice(prob, d, 0)] = 0.0
    up = _roll(Fz, prob, d, 1)
    if prob.bc[d] == WALL:
        up[_wall_slice(prob, d, -1)] = 0.0
    return (up - Fz) / prob.dx[d]


def div_face_T(prob: Problem, s, d):
    """Transpose of div_face: face f receives (s[f - e_d] - s[f]) / dx_d, zero on wall faces."""
    out = (_roll(s, prob, d, -1) - s) / prob.dx[d]
    if prob.bc[d] == WALL:
        out[_wall_slice(prob, d, 0)] = 0.0
    return out


class DirectSolver:
    def __init__(self, op: EllOp):
        self.op = op
        self.lu = spla.splu(op.to_sparse().tocsc())

    def __call__(self, b):
        return self.lu.solve(b.ravel()).reshape(b.shape)


class PBP:
    """M^-1 r for the sound (mode='sound') or sound+thermal (mode='sound_thermal') scheme.

    ``solver_factory(op)`` returns a callable b -> A^-1 b; default: direct sparse LU.
    """

    def __init__(self, prob: Problem, X, dt, mode="sound", solver_factory=None, schur=False):
        # theta-weighted step (eq. crank_nicholson): J = dU/dX / dt - theta dR/dX
        # = theta (dU/dX / tau - dR/dX) with tau = theta dt, so the scheme is built with the
        # implicit time step tau and its result divided by theta (theta = 1: tau = dt).
        # schur: keep the velocity residual in the pressure equation (eliminate du exactly
        # instead of dropping F_u there): rhs_p = F_p/(Gamma1 p) - tau div F_u.  The energy
        # update goes through the pressure equation's identity, where the term cancels.
        self.prob, self.X, self.mode, self.schur = prob, X, mode, schur
        self.dt = prob.theta * dt
        self.zscale = 1.0 / prob.theta
        dt = self.dt
        sf = solver_factory or DirectSolver
        self.Ap = pressure_operator(prob, X, dt)
        self.solve_p = sf(self.Ap)
        if mode == "sound_thermal":
            self.AT = thermal_operator(prob, X, dt)
            self.solve_T = sf(self.AT)
        elif mode != "sound":
            raise ValueError(mode)

    def apply(self, r):
        prob, X, dt = self.prob, self.X, self.dt
        rho = X[0]
        p, _, dpdr, dpde, g, cv = eos.thermo(prob, X[0], X[1])
        Fp, Fe, Fu = transform_in(prob, X, r)
        rhs_p = Fp / (g * p)
        if self.schur:
            for d in range(prob.nd):
                rhs_p = rhs_p - dt * div_face(prob, Fu[d], d)
        dp = self.solve_p(rhs_p)
        if self.mode == "sound":
            de = dt * Fe + (dp - dt * Fp) / (g * rho)
        else:
            dT = self.solve_T(rho * Fe + (dp / dt - Fp) / g)
            de = cv * dT
        z = np.empty_like(r)
        for d in range(prob.nd):
            z[2 + d] = dt * (Fu[d] - grad_face(prob, X, dp, d))
        z[1] = de
        z[0] = (dp - dpde * de) / dpdr
        return z * self.zscale

    def apply_T(self, w):
        """Transpose of ``apply`` (the elliptic solves are self-adjoint)."""
        prob, X, dt = self.prob, self.X, self.dt
        rho = X[0]
        p, _, dpdr, dpde, g, cv = eos.thermo(prob, X[0], X[1])
        # z0 = (dp - dpde de)/dpdr
        dp_b = w[0] / dpdr
        de_b = w[1] - dpde / dpdr * w[0]
        Fu_b = []
        for d in range(prob.nd):
            Fu_b.append(dt * w[2 + d])
            dp_b = dp_b - dt * grad_face_T(prob, X, w[2 + d], d)
        if self.mode == "sound":
            Fe_b = dt * de_b
            dp_b = dp_b + de_b / (g * rho)
            Fp_b = -dt * de_b / (g * rho)
        else:
            t = self.solve_T(cv * de_b)
            Fe_b = rho * t
            dp_b = dp_b + t / (g * dt)
            Fp_b = -t / g
        s = self.solve_p(dp_b)
        Fp_b = Fp_b + s / (g * p)
        if self.schur:
            for d in range(prob.nd):
                Fu_b[d] = Fu_b[d] - dt * div_face_T(prob, s, d)
        return transform_in_T(prob, X, Fp_b, Fe_b, Fu_b) * self.zscale
